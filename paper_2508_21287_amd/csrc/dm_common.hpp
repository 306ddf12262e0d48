// Internal definitions shared by the planner, the runtime and the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmotif.h"

namespace dm {

constexpr int kMaxMotif = DM_MAX_MOTIF_VERTICES;  // vertices in the largest motif (M18-O-6)
constexpr int kNarrowNew = 12;  // new values per step of the join kernels' common instantiation
constexpr int kMaxCols = DM_MAX_PATTERN_VERTICES; // columns of a partial-embedding table
constexpr int kMaxEdgeChecks = 24;                // explicit edge checks per join step
constexpr int kMaxSteps = DM_MAX_PATTERN_VERTICES;
constexpr int kNumMotifs = DM_NUM_MOTIFS;
constexpr int kMaxMotifEdges = 18;  // edges of a general-shape motif

// Motif catalogue (Sec. III-A "Motifs": M_i = path of i vertices, -O =
// cycle; the general shapes of Sec. VI-B: M4-1 = claw, M6-2O = 2x3 grid,
// M18-O-6 = the heavy-hex cell with a pendant at every other vertex; M7, a
// longer path keyed at its ends only, for two-key joins of path tables).
// Index order matches dm_datagraph_info.motif_rows.
enum MotifIndex { MOT_P2 = 0, MOT_P3, MOT_P4, MOT_P5, MOT_P6, MOT_C4, MOT_C6, MOT_C12, MOT_K13, MOT_G23, MOT_H18,
                  MOT_P7 };

struct MotifInfo {
    int size;
    bool cycle;
    uint32_t bit;  // DM_MOTIF_* bit (0 for M2: always present)
    const char* name;
    bool general;  // neither path nor cycle: shape given by `edges`
    int n_edges;
    int8_t edges[kMaxMotifEdges][2];
    // a path whose table is keyed at its ends only (slices must share an end)
    bool ends_only;
};

// General shapes are labelled so that positions 0..K-1 are one
// representative of each orbit of the motif's automorphism group (K = the
// number of orbits), as for paths (0..(L-1)/2) and cycles (0): the motif
// table keyed on position j serves every position of j's orbit.
inline const MotifInfo& motif_info(int m) {
    static const MotifInfo kInfo[kNumMotifs] = {
        {2, false, 0u, "M2", false, 0, {}},
        {3, false, DM_MOTIF_M3, "M3", false, 0, {}},
        {4, false, DM_MOTIF_M4, "M4", false, 0, {}},
        {5, false, DM_MOTIF_M5, "M5", false, 0, {}},
        {6, false, DM_MOTIF_M6, "M6", false, 0, {}},
        {4, true, DM_MOTIF_C4, "M4-O", false, 0, {}},
        {6, true, DM_MOTIF_C6, "M6-O", false, 0, {}},
        {12, true, DM_MOTIF_C12, "M12-O", false, 0, {}},
        // claw: centre 0, leaves 1..3 (orbits {0}, {1,2,3})
        {4, false, DM_MOTIF_M4_1, "M4-1", true, 3, {{0, 1}, {0, 2}, {0, 3}}},
        // 2x3 grid: rows 0-1-2 over 3-4-5 (orbits: corners {0,2,3,5}, middles {1,4})
        {6, false, DM_MOTIF_M6_2O, "M6-2O", true, 7, {{0, 1}, {1, 2}, {3, 4}, {4, 5}, {0, 3}, {1, 4}, {2, 5}}},
        // heavy-hex cell: cycle 0-1-3-4-...-12-0; pendants 2,13..17 on the even
        // cycle vertices 0,3,5,7,9,11 (orbits: those {0,..}, the odd ones {1,..},
        // the pendants {2,..})
        {18, false, DM_MOTIF_M18_O_6, "M18-O-6", true, 18,
         {{0, 1}, {1, 3}, {3, 4}, {4, 5}, {5, 6}, {6, 7}, {7, 8}, {8, 9}, {9, 10}, {10, 11}, {11, 12}, {12, 0},
          {0, 2}, {3, 13}, {5, 14}, {7, 15}, {9, 16}, {11, 17}}},
        {7, false, DM_MOTIF_M7, "M7", false, 0, {}, true}};
    return kInfo[m];
}

// Automorphism orbits of a general-shape motif (computed once).
int general_motif_orbits(int m);                 // number of orbits
int general_motif_orbit_rep(int m, int pos);     // the orbit's representative position (< orbits)
// an automorphism (position -> position) mapping `pos` to its representative
const int8_t* general_motif_to_rep(int m, int pos);

// Distinct key positions up to the motif's symmetry: a path reads the same
// reversed, a cycle the same rotated, a general shape by its automorphisms.
inline int motif_key_positions(int m) {
    const MotifInfo& mi = motif_info(m);
    if (mi.general) return general_motif_orbits(m);
    if (mi.ends_only) return 1;
    return mi.cycle ? 1 : (mi.size + 1) / 2;
}

// One join-and-filter iteration (Algorithm 1 body) in table-column space.
// Input table R has c_in columns; the step joins R with the motif table
// Res(M) indexed on motif position key_pos by the value in R column key_col,
// requires R[eq_col[i]] == M[eq_pos[i]] (further join keys), appends the
// motif positions new_pos[] as new columns c_in.., rejects rows where a new
// value repeats any value of the row (injectivity filter), and checks
// adjacency for each (edge_a, edge_b) column pair (pattern edges not carried
// by the motif).  motif == -1: filter only (no expansion).
struct StepDesc {
    int32_t motif;
    int32_t key_pos;
    int32_t key_col;
    int32_t c_in;
    int32_t n_new;
    int32_t n_eq;
    int32_t n_edge;
    int32_t pad_;
    int8_t new_pos[kMaxMotif];
    int8_t eq_col[kMaxMotif];
    int8_t eq_pos[kMaxMotif];
    uint8_t edge_a[kMaxEdgeChecks];
    uint8_t edge_b[kMaxEdgeChecks];
    // Induced variant: bit c of padj[t] is set when the pattern vertices of
    // column c and of new column c_in + t are adjacent (c < c_in + t); every
    // other earlier column must hold a data vertex not adjacent to the new one.
    uint64_t padj[kMaxMotif][2];
};

struct PlanStep {
    StepDesc d;
    int32_t slice_len = 0;
    int32_t slice[kMaxMotif];  // pattern vertices in motif position order
    double est_rows = 0;       // predicted rows after this step
};

struct Plan {
    int32_t k = 0;     // pattern vertices
    int32_t root = 0;  // pattern vertex held by table column 0
    std::vector<PlanStep> steps;
    int32_t col_of[kMaxCols];  // pattern vertex -> table column
    int32_t pv_of[kMaxCols];   // table column -> pattern vertex
    double est_peak_rows_cols = 0;  // max over steps of rows*cols (in + out)
    double est_final_rows = 0;
    double est_cost = 0;            // table values read, tested and written over all steps
    std::string cache_key;          // its entry in the context's plan cache
    // whether the streaming sort pass pays for this plan's tables: -1 not yet
    // known, 1 the last one found its root segments (nearly all) in order,
    // 0 it did not (the per-segment tiers then take them directly)
    int32_t sort_stream = -1;
};

struct NormPattern {
    int32_t k = 0;
    std::vector<std::pair<int32_t, int32_t>> edges;  // u < v, unique
};

// Validate and normalize a pattern (ids, self-loops, connectivity, merge repeats).
dm_status normalize_pattern(const dm_graph_desc* gp, NormPattern* out, std::string* err);

// Motif-table statistics used by the estimator (rows per motif; 0 = absent).
struct MotifStats {
    int32_t n_vertices = 0;
    double rows[kNumMotifs] = {};
    double avg_degree = 0;
};

// Decompose a pattern into motif slices (Sec. III-C).  `avail` = motifs that
// may be used (bit per MotifIndex; M2 always allowed).  stats may be null
// (then estimates are left at 0).
dm_status plan_pattern(const NormPattern& p, int32_t root, uint32_t avail_motif_bits,
                       const MotifStats* stats, Plan* out, std::string* err);

// Serialize a plan in the dm_plan() int32 format.
std::vector<int32_t> serialize_plan(const Plan& plan);

// Map DM_MOTIF_* mask to a bitset over MotifIndex (bit 0 = M2 always set).
uint32_t motif_bits_from_mask(uint32_t dm_mask);

}  // namespace dm
