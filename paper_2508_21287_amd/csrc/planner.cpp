// Pattern validation and decomposition into motif slices (paper Sec. III-C).
//
// The decomposition repeatedly picks a slice: a match of a motif in the
// *reduced* pattern (the pattern's still-uncovered edges), trying motifs in
// descending size order.  A slice must share at least one vertex with the
// vertices already placed (those shared vertices become the join keys,
// Sec. III-B) and covers at least one uncovered edge; vertices whose edges
// are all covered drop out of the reduced pattern, the others stay as
// boundary nodes for later slices.  Any valid decomposition gives the same
// embedding set (the paper needs only one, not the ideal one); among the
// matches of the chosen motif this planner prefers the one with the most
// shared vertices plus edge checks, since extra join keys and edge checks
// shrink the next table.  Pattern edges that end up joining two placed
// vertices without being an edge of some slice (chords, cycle closures) get
// an explicit adjacency check at the step that places their second endpoint;
// this is the paper's all-overlap join written as a filter.
#include <algorithm>
#include <array>
#include <functional>
#include <cmath>
#include <cstring>

#include "dm_common.hpp"

namespace dm {

// ---- general-shape motifs: automorphisms by brute force (size <= 6)

namespace {

struct GeneralMotif {
    int orbits = 0;
    int8_t rep[kMaxMotif];               // position -> representative
    int8_t to_rep[kMaxMotif][kMaxMotif]; // position -> an automorphism taking it to rep
};

// Automorphisms by backtracking over positions in BFS order (each later
// position has an earlier neighbour), matching degrees and adjacency to the
// positions already mapped.
void motif_automorphisms(int L, const bool (&adj)[kMaxMotif][kMaxMotif], std::vector<std::array<int8_t, kMaxMotif>>* out) {
    int deg[kMaxMotif] = {};
    for (int a = 0; a < L; a++)
        for (int b = 0; b < L; b++) deg[a] += adj[a][b];
    int ord[kMaxMotif], head = 0, tail = 0;
    bool seen[kMaxMotif] = {};
    ord[tail++] = 0;
    seen[0] = true;
    while (head < tail) {
        const int x = ord[head++];
        for (int y = 0; y < L; y++)
            if (adj[x][y] && !seen[y]) {
                seen[y] = true;
                ord[tail++] = y;
            }
    }
    std::array<int8_t, kMaxMotif> img{};
    bool used[kMaxMotif] = {};
    std::function<void(int)> go = [&](int d) {
        if (d == L) {
            out->push_back(img);
            return;
        }
        const int x = ord[d];
        for (int w = 0; w < L; w++) {
            if (used[w] || deg[w] != deg[x]) continue;
            bool ok = true;
            for (int e = 0; e < d && ok; e++) ok = adj[x][ord[e]] == adj[w][img[ord[e]]];
            if (!ok) continue;
            img[x] = (int8_t)w;
            used[w] = true;
            go(d + 1);
            used[w] = false;
        }
    };
    go(0);
}

GeneralMotif compute_general(int m) {
    const MotifInfo& mi = motif_info(m);
    const int L = mi.size;
    bool adj[kMaxMotif][kMaxMotif] = {};
    for (int e = 0; e < mi.n_edges; e++) adj[mi.edges[e][0]][mi.edges[e][1]] = adj[mi.edges[e][1]][mi.edges[e][0]] = true;
    std::vector<std::array<int8_t, kMaxMotif>> auts;
    motif_automorphisms(L, adj, &auts);
    GeneralMotif g;
    for (int i = 0; i < L; i++) {
        g.rep[i] = (int8_t)i;
        for (int j = 0; j < L; j++) g.to_rep[i][j] = (int8_t)j;  // the identity
    }
    // the representative of i is the smallest position an automorphism takes it to
    for (auto& a : auts)
        for (int i = 0; i < L; i++)
            if (a[i] < g.rep[i]) {
                g.rep[i] = a[i];
                for (int q = 0; q < L; q++) g.to_rep[i][q] = a[q];
            }
    int reps = 0;
    for (int i = 0; i < L; i++) reps += g.rep[i] == i;
    g.orbits = reps;
    return g;
}

const GeneralMotif& general(int m) {
    static const std::vector<GeneralMotif> table = [] {
        std::vector<GeneralMotif> t(kNumMotifs);
        for (int q = 0; q < kNumMotifs; q++)
            if (motif_info(q).general) t[q] = compute_general(q);
        return t;
    }();
    return table[m];
}

}  // namespace

int general_motif_orbits(int m) { return general(m).orbits; }
int general_motif_orbit_rep(int m, int pos) { return general(m).rep[pos]; }
const int8_t* general_motif_to_rep(int m, int pos) { return general(m).to_rep[pos]; }

uint32_t motif_bits_from_mask(uint32_t m) {
    uint32_t bits = 1u << MOT_P2;
    if (m & DM_MOTIF_M2_ONLY) return bits;
    for (int i = 1; i < kNumMotifs; i++)
        if (m & motif_info(i).bit) bits |= 1u << i;
    return bits;
}

dm_status normalize_pattern(const dm_graph_desc* gp, NormPattern* out, std::string* err) {
    if (!gp || !out) {
        *err = "pattern descriptor is NULL";
        return DM_ERR_INVALID_ARG;
    }
    const int32_t k = gp->n_vertices;
    if (k < 1) {
        *err = "pattern needs at least one vertex";
        return DM_ERR_INVALID_ARG;
    }
    if (k > kMaxCols) {
        *err = "pattern has more than " + std::to_string(kMaxCols) + " vertices";
        return DM_ERR_UNSUPPORTED;
    }
    if (gp->n_edges < 0 || (gp->n_edges > 0 && !gp->edges)) {
        *err = "pattern edge array is invalid";
        return DM_ERR_INVALID_ARG;
    }
    std::vector<std::pair<int32_t, int32_t>> e;
    e.reserve((size_t)gp->n_edges);
    for (int64_t i = 0; i < gp->n_edges; i++) {
        int32_t u = gp->edges[2 * i], v = gp->edges[2 * i + 1];
        if (u < 0 || v < 0 || u >= k || v >= k) {
            *err = "pattern vertex id out of range";
            return DM_ERR_VERTEX_RANGE;
        }
        if (u == v) {
            *err = "pattern has a self-loop";
            return DM_ERR_PATTERN_SELF_LOOP;
        }
        e.emplace_back(std::min(u, v), std::max(u, v));
    }
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    // connectivity (the paper assumes connected graphs, Sec. III-A)
    std::vector<std::vector<int32_t>> adj(k);
    for (auto& x : e) {
        adj[x.first].push_back(x.second);
        adj[x.second].push_back(x.first);
    }
    std::vector<char> seen(k, 0);
    std::vector<int32_t> st{0};
    seen[0] = 1;
    int32_t cnt = 1;
    while (!st.empty()) {
        int32_t u = st.back();
        st.pop_back();
        for (int32_t w : adj[u])
            if (!seen[w]) {
                seen[w] = 1;
                cnt++;
                st.push_back(w);
            }
    }
    if (cnt != k) {
        *err = "pattern is not connected";
        return DM_ERR_PATTERN_DISCONNECTED;
    }
    out->k = k;
    out->edges = std::move(e);
    return DM_OK;
}

namespace {

struct Planner {
    int32_t k;
    std::vector<std::vector<int32_t>> nbrs;
    std::vector<std::vector<char>> uncov;  // uncovered pattern edges
    int32_t col_of[kMaxCols];
    int32_t ncols = 0;

    // search state
    int32_t L = 0;
    bool cyc = false;
    bool ends_only = false;
    bool ends_expand = false;  // end-keyed motifs may extend a chain from one placed end
    int32_t seq[kMaxMotif];
    char inseq[kMaxCols];
    int64_t expansions = 0, found = 0;
    int best_score = -1;
    int32_t best[kMaxMotif];
    static constexpr int64_t kMaxExpansions = 200000;
    static constexpr int64_t kMaxFound = 4096;

    bool mapped(int32_t v) const { return col_of[v] >= 0; }

    // Edge checks a slice would need: uncovered pattern edges from a new
    // slice vertex to a placed or slice vertex that are not motif edges.
    int count_checks(const int32_t* s) const {
        char ins[kMaxCols];
        std::memset(ins, 0, sizeof ins);
        for (int i = 0; i < L; i++) ins[s[i]] = 1;
        int c = 0;
        for (int i = 0; i < L; i++) {
            int32_t u = s[i];
            if (mapped(u)) continue;
            for (int32_t w : nbrs[u]) {
                if (!uncov[u][w]) continue;
                if (!(mapped(w) || ins[w])) continue;
                if (is_motif_edge(s, u, w)) continue;
                if (!mapped(w) && w < u) continue;  // count new-new pairs once
                c++;
            }
        }
        return c;
    }

    bool is_motif_edge(const int32_t* s, int32_t a, int32_t b) const {
        for (int i = 0; i + 1 < L; i++)
            if ((s[i] == a && s[i + 1] == b) || (s[i] == b && s[i + 1] == a)) return true;
        if (cyc && ((s[L - 1] == a && s[0] == b) || (s[L - 1] == b && s[0] == a))) return true;
        return false;
    }

    void consider() {
        found++;
        int keys = 0, nnew = 0;
        for (int i = 0; i < L; i++) (mapped(seq[i]) ? keys : nnew)++;
        if (keys == 0 || nnew == 0) return;
        // A motif keyed at its ends only covers a chain of the pattern (its
        // inner vertices have no other pattern edges), as the first slice
        // (its table read in place), to close a chain between two placed
        // vertices (a two-key join, binary-searched), or, where its table has
        // few rows per key, to extend a chain from one placed end; with many
        // rows per key that would be a candidate loop as long as the fan-out.
        if (ends_only) {
            for (int i = 1; i + 1 < L; i++)
                if ((int)nbrs[seq[i]].size() != 2) return;
            const bool first = ncols == 1, both = mapped(seq[0]) && mapped(seq[L - 1]);
            if (!(first || both || ends_expand)) return;
        }
        int score = 2 * keys + count_checks(seq);
        if (score > best_score) {
            best_score = score;
            std::memcpy(best, seq, sizeof(int32_t) * L);
        }
    }

    void dfs(int depth) {
        if (found >= kMaxFound || expansions >= kMaxExpansions) return;
        expansions++;
        if (depth == L) {
            if (cyc && !uncov[seq[L - 1]][seq[0]]) return;
            consider();
            return;
        }
        int32_t last = seq[depth - 1];
        for (int32_t w : nbrs[last]) {
            if (!uncov[last][w] || inseq[w]) continue;
            seq[depth] = w;
            inseq[w] = 1;
            dfs(depth + 1);
            inseq[w] = 0;
            if (found >= kMaxFound || expansions >= kMaxExpansions) return;
        }
    }

    bool search(int32_t size, bool cycle, bool ends = false) {
        L = size;
        cyc = cycle;
        ends_only = ends;
        expansions = found = 0;
        best_score = -1;
        std::memset(inseq, 0, sizeof inseq);
        // starts: placed vertices in placement order, then (paths only) the
        // rest, so slices whose shared vertex is interior are found too
        std::vector<int32_t> starts;
        std::vector<std::pair<int32_t, int32_t>> placed;
        for (int32_t v = 0; v < k; v++)
            if (mapped(v)) placed.emplace_back(col_of[v], v);
        std::sort(placed.begin(), placed.end());
        for (auto& pv : placed) starts.push_back(pv.second);
        if (!cycle && !ends)
            for (int32_t v = 0; v < k; v++)
                if (!mapped(v)) starts.push_back(v);
        for (int32_t s : starts) {
            bool has_uncov = false;
            for (int32_t w : nbrs[s]) has_uncov |= (bool)uncov[s][w];
            if (!has_uncov) continue;
            seq[0] = s;
            inseq[s] = 1;
            dfs(1);
            inseq[s] = 0;
            if (found >= kMaxFound || expansions >= kMaxExpansions) break;
        }
        return best_score >= 0;
    }

    // ---- general-shape motifs: embeddings of the motif graph into the
    // pattern (motif edges onto pattern edges, covered or not) that share a
    // placed vertex, bring a new one and cover at least one uncovered edge
    const MotifInfo* gm = nullptr;
    bool gadj[kMaxMotif][kMaxMotif];
    int32_t gord[kMaxMotif], gpar[kMaxMotif];
    int32_t gseq[kMaxMotif];  // motif position -> pattern vertex
    std::vector<std::vector<char>> padj;  // pattern adjacency (all edges)

    bool is_gmotif_edge(const int32_t* sq, int32_t a, int32_t b) const {
        for (int e = 0; e < gm->n_edges; e++) {
            const int32_t x = sq[gm->edges[e][0]], y = sq[gm->edges[e][1]];
            if ((x == a && y == b) || (x == b && y == a)) return true;
        }
        return false;
    }

    int count_checks_general(const int32_t* sq) const {
        char ins[kMaxCols];
        std::memset(ins, 0, sizeof ins);
        for (int i = 0; i < L; i++) ins[sq[i]] = 1;
        int c = 0;
        for (int i = 0; i < L; i++) {
            int32_t u = sq[i];
            if (mapped(u)) continue;
            for (int32_t w : nbrs[u]) {
                if (!uncov[u][w]) continue;
                if (!(mapped(w) || ins[w])) continue;
                if (is_gmotif_edge(sq, u, w)) continue;
                if (!mapped(w) && w < u) continue;
                c++;
            }
        }
        return c;
    }

    void consider_general() {
        found++;
        int keys = 0, nnew = 0;
        for (int i = 0; i < L; i++) (mapped(gseq[i]) ? keys : nnew)++;
        if (keys == 0 || nnew == 0) return;
        bool covers = false;
        for (int e = 0; e < gm->n_edges && !covers; e++) covers = uncov[gseq[gm->edges[e][0]]][gseq[gm->edges[e][1]]];
        if (!covers) return;
        int score = 2 * keys + count_checks_general(gseq);
        if (score > best_score) {
            best_score = score;
            std::memcpy(best, gseq, sizeof(int32_t) * L);
        }
    }

    void gdfs(int depth) {
        if (found >= kMaxFound || expansions >= kMaxExpansions) return;
        expansions++;
        if (depth == L) {
            consider_general();
            return;
        }
        const int pos = gord[depth];
        const int32_t anchor = gseq[gpar[pos]];
        for (int32_t w : nbrs[anchor]) {
            if (inseq[w]) continue;
            bool ok = true;
            for (int d = 0; d < depth && ok; d++) {
                const int q = gord[d];
                if (gadj[pos][q] && !padj[w][gseq[q]]) ok = false;
            }
            if (!ok) continue;
            gseq[pos] = w;
            inseq[w] = 1;
            gdfs(depth + 1);
            inseq[w] = 0;
            if (found >= kMaxFound || expansions >= kMaxExpansions) return;
        }
    }

    bool search_general(int m) {
        gm = &motif_info(m);
        L = gm->size;
        cyc = false;
        expansions = found = 0;
        best_score = -1;
        std::memset(inseq, 0, sizeof inseq);
        std::memset(gadj, 0, sizeof gadj);
        for (int e = 0; e < gm->n_edges; e++) gadj[gm->edges[e][0]][gm->edges[e][1]] = gadj[gm->edges[e][1]][gm->edges[e][0]] = true;
        // anchor: a placed vertex (placement order) at each motif position in turn
        std::vector<std::pair<int32_t, int32_t>> placed;
        for (int32_t v = 0; v < k; v++)
            if (mapped(v)) placed.emplace_back(col_of[v], v);
        std::sort(placed.begin(), placed.end());
        for (auto& pv : placed) {
            const int32_t v = pv.second;
            bool has_uncov = false;
            for (int32_t w : nbrs[v]) has_uncov |= (bool)uncov[v][w];
            if (!has_uncov) continue;
            for (int a = 0; a < L; a++) {
                // BFS order of the motif from position a
                int head = 0, tail = 0;
                bool seen[kMaxMotif] = {};
                gord[tail++] = a;
                seen[a] = true;
                gpar[a] = a;
                while (head < tail) {
                    const int x = gord[head++];
                    for (int y = 0; y < L; y++)
                        if (gadj[x][y] && !seen[y]) {
                            seen[y] = true;
                            gpar[y] = x;
                            gord[tail++] = y;
                        }
                }
                gseq[a] = v;
                inseq[v] = 1;
                gdfs(1);
                inseq[v] = 0;
                if (found >= kMaxFound || expansions >= kMaxExpansions) break;
            }
            if (found >= kMaxFound || expansions >= kMaxExpansions) break;
        }
        return best_score >= 0;
    }
};

// Fixed cost of one launched join step in table values (about 16 us of
// launch and dependent-round latency at a few TB/s).
constexpr double kStepCost = 16.0 * 1024 * 1024;

double estimate_fanout(const MotifStats* st, int m) {
    if (!st || st->n_vertices <= 0) return 0;
    return st->rows[m] / (double)st->n_vertices;
}

}  // namespace

dm_status plan_pattern(const NormPattern& p, int32_t root, uint32_t avail, const MotifStats* stats,
                       Plan* out, std::string* err) {
    const int32_t k = p.k;
    if (root < 0 || root >= k) {
        *err = "plan root out of range";
        return DM_ERR_INVALID_ARG;
    }
    avail |= 1u << MOT_P2;
    Planner pl;
    pl.k = k;
    pl.nbrs.assign(k, {});
    pl.uncov.assign(k, std::vector<char>(k, 0));
    for (auto& e : p.edges) {
        pl.nbrs[e.first].push_back(e.second);
        pl.nbrs[e.second].push_back(e.first);
        pl.uncov[e.first][e.second] = pl.uncov[e.second][e.first] = 1;
    }
    for (auto& nb : pl.nbrs) std::sort(nb.begin(), nb.end());
    pl.padj.assign(k, std::vector<char>(k, 0));
    for (auto& e : p.edges) pl.padj[e.first][e.second] = pl.padj[e.second][e.first] = 1;
    for (int32_t v = 0; v < kMaxCols; v++) pl.col_of[v] = -1;
    pl.col_of[root] = 0;
    pl.ncols = 1;

    Plan plan;
    plan.k = k;
    plan.root = root;
    for (int i = 0; i < kMaxCols; i++) plan.col_of[i] = plan.pv_of[i] = -1;

    // motif order: descending size, cycles before paths of equal size
    std::vector<int> order;
    for (int m = 0; m < kNumMotifs; m++)
        if (avail & (1u << m)) order.push_back(m);
    std::sort(order.begin(), order.end(), [](int a, int b) {
        const MotifInfo &x = motif_info(a), &y = motif_info(b);
        if (x.size != y.size) return x.size > y.size;
        const int rx = x.cycle ? 0 : (x.general ? 1 : 2), ry = y.cycle ? 0 : (y.general ? 1 : 2);
        return rx < ry;
    });

    const double nv = stats ? (double)stats->n_vertices : 0.0;
    const double deg = stats ? std::max(stats->avg_degree, 1.0) : 1.0;
    // extending from one end reads every row of the end's key group: only
    // where those groups are small
    for (int m = 0; m < kNumMotifs; m++)
        if (motif_info(m).ends_only && (avail >> m) & 1 && nv > 0 && stats->rows[m] / nv <= 64.0)
            pl.ends_expand = true;
    const double br = std::max(deg - 1.0, 1.0);
    double rows = nv;  // identity table: one row per data vertex
    double peak = rows * 1;
    double cost = 0;

    while (pl.ncols < k) {
        int chosen = -1;
        for (int m : order) {
            const MotifInfo& mi = motif_info(m);
            if (mi.size > k) continue;
            if (mi.general ? pl.search_general(m) : pl.search(mi.size, mi.cycle, mi.ends_only)) {
                chosen = m;
                break;
            }
        }
        if (chosen < 0) {
            *err = "decomposition found no slice (internal)";
            return DM_ERR_INTERNAL;
        }
        const MotifInfo& mi = motif_info(chosen);
        const int L = mi.size;
        int32_t s[kMaxMotif];
        std::memcpy(s, pl.best, sizeof(int32_t) * L);
        // canonical orientation: key at the smallest available key position
        int key = -1;
        if (mi.general) {
            // key: the placed position with the smallest orbit representative,
            // moved onto that representative by an automorphism
            int bestrep = 1 << 30;
            for (int i = 0; i < L; i++)
                if (pl.mapped(s[i]) && general_motif_orbit_rep(chosen, i) < bestrep) {
                    bestrep = general_motif_orbit_rep(chosen, i);
                    key = i;
                }
            const int8_t* a = general_motif_to_rep(chosen, key);
            int32_t r[kMaxMotif];
            for (int i = 0; i < L; i++) r[a[i]] = s[i];
            std::memcpy(s, r, sizeof(int32_t) * L);
            key = bestrep;
        } else if (mi.cycle) {
            for (int i = 0; i < L && key < 0; i++)
                if (pl.mapped(s[i])) key = i;
            int32_t r[kMaxMotif];
            for (int i = 0; i < L; i++) r[i] = s[(key + i) % L];
            std::memcpy(s, r, sizeof(int32_t) * L);
            key = 0;
        } else {
            int bestd = 1 << 30;
            for (int i = 0; i < L; i++)
                if (pl.mapped(s[i]) && std::min(i, L - 1 - i) < bestd) {
                    bestd = std::min(i, L - 1 - i);
                    key = i;
                }
            if (L >= 3 && pl.mapped(s[0]) && pl.mapped(s[L - 1])) {
                // both ends placed: key at position 0, the path oriented so that
                // its new vertices run in ascending label order (the join emits
                // each row's candidates in motif-position order, so rows then
                // come out in label order and the final sort finds them sorted)
                if (s[1] > s[L - 2]) std::reverse(s, s + L);
                key = 0;
            } else if (key > (L - 1) / 2) {
                std::reverse(s, s + L);
                key = L - 1 - key;
            }
        }
        PlanStep ps;
        std::memset(&ps.d, 0, sizeof ps.d);
        StepDesc& d = ps.d;
        d.motif = chosen;
        d.key_pos = key;
        d.key_col = pl.col_of[s[key]];
        d.c_in = pl.ncols;
        ps.slice_len = L;
        std::memcpy(ps.slice, s, sizeof(int32_t) * L);
        int min_eq_dist = 0;
        for (int i = 0; i < L; i++) {
            if (i == key) continue;
            if (pl.mapped(s[i])) {
                d.eq_col[d.n_eq] = (int8_t)pl.col_of[s[i]];
                d.eq_pos[d.n_eq] = (int8_t)i;
                d.n_eq++;
                int dist = std::abs(i - key);
                if (mi.cycle) dist = std::min(dist, L - dist);
                if (mi.general) dist = 1;
                min_eq_dist = std::max(min_eq_dist, dist);
            }
        }
        for (int i = 0; i < L; i++) {
            if (!pl.mapped(s[i])) {
                d.new_pos[d.n_new++] = (int8_t)i;
                pl.col_of[s[i]] = pl.ncols++;
            }
        }
        // motif edges are now covered
        if (mi.general) {
            for (int e = 0; e < mi.n_edges; e++) {
                const int32_t x = s[mi.edges[e][0]], y = s[mi.edges[e][1]];
                pl.uncov[x][y] = pl.uncov[y][x] = 0;
            }
        } else {
            for (int i = 0; i + 1 < L; i++) pl.uncov[s[i]][s[i + 1]] = pl.uncov[s[i + 1]][s[i]] = 0;
            if (mi.cycle) pl.uncov[s[L - 1]][s[0]] = pl.uncov[s[0]][s[L - 1]] = 0;
        }
        // explicit edge checks for remaining pattern edges among placed vertices
        std::vector<std::pair<int, int>> checks;
        for (int i = 0; i < L; i++) {
            int32_t u = s[i];
            bool is_new = false;
            for (int t = 0; t < d.n_new; t++) is_new |= (d.new_pos[t] == i);
            if (!is_new) continue;
            for (int32_t w : pl.nbrs[u]) {
                if (!pl.uncov[u][w] || !pl.mapped(w)) continue;
                checks.emplace_back(pl.col_of[u], pl.col_of[w]);
                pl.uncov[u][w] = pl.uncov[w][u] = 0;
            }
        }
        size_t first = std::min(checks.size(), (size_t)kMaxEdgeChecks);
        for (size_t i = 0; i < first; i++) {
            d.edge_a[d.n_edge] = (uint8_t)checks[i].first;
            d.edge_b[d.n_edge] = (uint8_t)checks[i].second;
            d.n_edge++;
        }
        // estimate: motif rows per key vertex; once the key vertex already has
        // placed neighbours, each motif edge at the key competes with them
        double fan = estimate_fanout(stats, chosen);
        if (d.c_in > 1) {
            int key_deg = mi.cycle ? 2 : ((key == 0 || key == L - 1) ? 1 : 2);
            if (mi.general) {
                key_deg = 0;
                for (int e = 0; e < mi.n_edges; e++) key_deg += (mi.edges[e][0] == key) + (mi.edges[e][1] == key);
            }
            fan *= std::pow(std::max(deg - 1.0, 0.5) / deg, key_deg);
        }
        double nrows = rows * fan;
        for (int e = 0; e < d.n_eq; e++) nrows /= std::max(1.0, deg * std::pow(br, std::max(0, min_eq_dist - 1)));
        for (int e = 0; e < (int)checks.size(); e++) nrows /= std::max(1.0, deg * br);
        peak = std::max(peak, rows * d.c_in + nrows * (d.c_in + d.n_new));
        // work of the step in table values: the input rows read, every
        // candidate's loaded values and checks, the output rows written; a
        // first step that only copies a motif table keyed at position 0 is
        // taken in place (no work)
        // taken in place (no work).  A path keyed at one end whose further key
        // is the other end is binary-searched on a copy ordered by that end:
        // only the matching run is tested.
        const bool in_place = plan.steps.empty() && d.key_pos == 0 && d.n_eq == 0 && checks.empty() && !mi.general;
        double cand = rows * fan;
        if (!mi.general && !mi.cycle && d.key_pos == 0 && d.n_eq > 0 && d.eq_pos[0] == L - 1)
            cand = cand / std::max(1.0, deg * std::pow(br, std::max(0, L - 2))) + rows * std::log2(std::max(fan, 2.0));
        // each launched step also costs a fixed latency (launch, look-back
        // chain, readbacks), here as many table values as move in that time
        if (!in_place)
            cost += kStepCost + rows * d.c_in + cand * (d.n_new + d.n_eq + (double)checks.size()) +
                    nrows * (d.c_in + d.n_new);
        rows = nrows;
        ps.est_rows = rows;
        plan.steps.push_back(ps);
        // edge checks beyond one step's capacity become filter-only steps
        for (size_t i = first; i < checks.size();) {
            PlanStep fs;
            std::memset(&fs.d, 0, sizeof fs.d);
            fs.d.motif = -1;
            fs.d.c_in = pl.ncols;
            fs.d.key_col = 0;
            for (; i < checks.size() && fs.d.n_edge < kMaxEdgeChecks; i++) {
                fs.d.edge_a[fs.d.n_edge] = (uint8_t)checks[i].first;
                fs.d.edge_b[fs.d.n_edge] = (uint8_t)checks[i].second;
                fs.d.n_edge++;
            }
            fs.est_rows = rows;
            plan.steps.push_back(fs);
        }
    }
    for (int32_t v = 0; v < k; v++) {
        plan.col_of[v] = pl.col_of[v];
        plan.pv_of[pl.col_of[v]] = v;
    }
    // pattern adjacency of each new column to the earlier ones (induced variant)
    {
        std::vector<std::vector<char>> padj(k, std::vector<char>(k, 0));
        for (auto& e : p.edges) padj[e.first][e.second] = padj[e.second][e.first] = 1;
        for (auto& ps : plan.steps) {
            StepDesc& d = ps.d;
            std::memset(d.padj, 0, sizeof d.padj);
            const int nn = d.motif >= 0 ? d.n_new : 0;
            for (int t = 0; t < nn; t++) {
                const int32_t u = plan.pv_of[d.c_in + t];
                for (int c = 0; c < d.c_in + t; c++)
                    if (padj[u][plan.pv_of[c]]) d.padj[t][c >> 6] |= 1ull << (c & 63);
            }
        }
    }
    plan.est_final_rows = rows;
    plan.est_peak_rows_cols = peak;
    plan.est_cost = cost;
    *out = std::move(plan);
    return DM_OK;
}

std::vector<int32_t> serialize_plan(const Plan& plan) {
    std::vector<int32_t> b;
    b.push_back(plan.k);
    b.push_back((int32_t)plan.steps.size());
    for (int32_t v = 0; v < plan.k; v++) b.push_back(plan.col_of[v]);
    for (auto& ps : plan.steps) {
        const StepDesc& d = ps.d;
        b.push_back(d.motif);
        b.push_back(d.key_pos);
        b.push_back(d.key_col);
        b.push_back(d.c_in);
        b.push_back(d.n_new);
        for (int i = 0; i < d.n_new; i++) b.push_back(d.new_pos[i]);
        b.push_back(d.n_eq);
        for (int i = 0; i < d.n_eq; i++) {
            b.push_back(d.eq_col[i]);
            b.push_back(d.eq_pos[i]);
        }
        b.push_back(d.n_edge);
        for (int i = 0; i < d.n_edge; i++) {
            b.push_back(d.edge_a[i]);
            b.push_back(d.edge_b[i]);
        }
        b.push_back(ps.slice_len);
        for (int i = 0; i < ps.slice_len; i++) b.push_back(ps.slice[i]);
    }
    return b;
}

}  // namespace dm
