// Host-side checks of the library's CPU code, built with g++ under the
// address/undefined-behaviour sanitizers and, separately, the thread
// sanitizer (see tests/test_host_sanitizers.py).  Only host code is tested
// here: the planner (pattern decomposition), pattern validation, the worker
// pool that plans a batch and the plan cache that server workers share.
//
//   host_checks plan     random patterns through validation and the planner
//   host_checks threads  the pool and the plan cache under concurrent use
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_2508_21287_amd/csrc/dm_common.hpp"
#include "../../paper_2508_21287_amd/csrc/host_pool.hpp"

using namespace dm;

static int failures = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            if (failures++ < 20) {                     \
                std::fprintf(stderr, "FAIL %s: ", #c); \
                std::fprintf(stderr, __VA_ARGS__);     \
                std::fprintf(stderr, "\n");            \
            }                                          \
        }                                              \
    } while (0)

// A random connected pattern: a random tree on k vertices plus `extra`
// random edges (duplicates merge).
static std::vector<int32_t> random_pattern(std::mt19937& rng, int k, int extra) {
    std::vector<int32_t> e;
    for (int v = 1; v < k; v++) {
        e.push_back((int32_t)(rng() % v));
        e.push_back(v);
    }
    for (int i = 0; i < extra && k > 1; i++) {
        int a = (int)(rng() % k), b = (int)(rng() % k);
        if (a == b) continue;
        e.push_back(a);
        e.push_back(b);
    }
    return e;
}

static MotifStats lattice_stats(bool grid) {
    MotifStats st;
    if (grid) {  // a 100 x 100 square grid
        st.n_vertices = 10000;
        st.avg_degree = 3.96;
        st.rows[MOT_P2] = 39600, st.rows[MOT_P3] = 117608, st.rows[MOT_P4] = 350056, st.rows[MOT_C4] = 78408;
        st.rows[MOT_P7] = 7408432;
    } else {  // a heavy-hex lattice of 56 x 56
        st.n_vertices = 3906;
        st.avg_degree = 2.0 * 4620 / 3906;
        st.rows[MOT_P2] = 9240, st.rows[MOT_P3] = 13636, st.rows[MOT_P4] = 17924, st.rows[MOT_K13] = 8904;
        st.rows[MOT_P7] = 51642;
    }
    return st;
}

// Every pattern edge is covered: by a slice's motif edges (slices may cover
// an edge again, e.g. a further key between placed vertices) or by an
// explicit check; every covered pair is a pattern edge; columns are a
// permutation; keys and further keys read placed columns.
static void check_plan(const NormPattern& p, const Plan& pl, uint32_t avail) {
    const int k = p.k;
    std::vector<int> seen(k, 0);
    for (int v = 0; v < k; v++) {
        CHECK(pl.col_of[v] >= 0 && pl.col_of[v] < k, "col_of[%d] = %d", v, pl.col_of[v]);
        if (pl.col_of[v] >= 0 && pl.col_of[v] < k) seen[pl.col_of[v]]++;
    }
    for (int c = 0; c < k; c++) CHECK(seen[c] == 1, "column %d used %d times", c, seen[c]);
    std::set<std::pair<int, int>> want(p.edges.begin(), p.edges.end()), got;
    auto add = [&](int a, int b) {
        auto e = std::make_pair(std::min(a, b), std::max(a, b));
        CHECK(want.count(e), "covered pair %d-%d is not a pattern edge", a, b);
        got.insert(e);
    };
    int ncols = 1;
    for (auto& ps : pl.steps) {
        const StepDesc& d = ps.d;
        CHECK(d.c_in == ncols, "step reads %d columns, %d placed", d.c_in, ncols);
        if (d.motif >= 0) {
            CHECK((avail >> d.motif) & 1, "motif %d not available", d.motif);
            const MotifInfo& mi = motif_info(d.motif);
            CHECK(d.key_col < d.c_in && d.key_pos < motif_key_positions(d.motif), "key %d/%d", d.key_col, d.key_pos);
            for (int e = 0; e < d.n_eq; e++) CHECK(d.eq_col[e] < d.c_in, "further key column %d", d.eq_col[e]);
            if (mi.general) {
                for (int e = 0; e < mi.n_edges; e++) add(ps.slice[mi.edges[e][0]], ps.slice[mi.edges[e][1]]);
            } else {
                for (int i = 0; i + 1 < mi.size; i++) add(ps.slice[i], ps.slice[i + 1]);
                if (mi.cycle) add(ps.slice[mi.size - 1], ps.slice[0]);
            }
            ncols += d.n_new;
        }
        for (int e = 0; e < d.n_edge; e++) {
            CHECK(d.edge_a[e] < ncols && d.edge_b[e] < ncols, "check columns %d %d", d.edge_a[e], d.edge_b[e]);
            add(pl.pv_of[d.edge_a[e]], pl.pv_of[d.edge_b[e]]);
        }
    }
    CHECK(ncols == k, "%d of %d columns placed", ncols, k);
    CHECK(got == want, "%zu of %zu pattern edges covered", got.size(), want.size());
}

static int run_plan_checks() {
    std::mt19937 rng(12345);
    const MotifStats stats[2] = {lattice_stats(false), lattice_stats(true)};
    int plans = 0;
    // validation errors
    {
        NormPattern p;
        std::string err;
        int32_t loop[] = {0, 0, 0, 1};
        dm_graph_desc g{2, 2, loop};
        CHECK(normalize_pattern(&g, &p, &err) == DM_ERR_PATTERN_SELF_LOOP, "self-loop");
        int32_t split[] = {0, 1, 2, 3};
        dm_graph_desc g2{4, 2, split};
        CHECK(normalize_pattern(&g2, &p, &err) == DM_ERR_PATTERN_DISCONNECTED, "disconnected");
        int32_t range[] = {0, 5};
        dm_graph_desc g3{2, 1, range};
        CHECK(normalize_pattern(&g3, &p, &err) == DM_ERR_VERTEX_RANGE, "range");
        CHECK(normalize_pattern(nullptr, &p, &err) != DM_OK, "null");
    }
    for (int t = 0; t < 3000; t++) {
        const int k = t < 2900 ? 1 + (int)(rng() % 40) : 1 + (int)(rng() % DM_MAX_PATTERN_VERTICES);
        const int extra = (int)(rng() % 6);
        std::vector<int32_t> e = random_pattern(rng, k, extra);
        dm_graph_desc g{k, (int64_t)e.size() / 2, e.empty() ? nullptr : e.data()};
        NormPattern p;
        std::string err;
        if (normalize_pattern(&g, &p, &err) != DM_OK) {
            CHECK(false, "valid pattern refused: %s", err.c_str());
            continue;
        }
        uint32_t avail = 1u | (uint32_t)(rng() & ((1u << kNumMotifs) - 1));
        const MotifStats* st = (t % 3 == 0) ? nullptr : &stats[t % 2];
        Plan pl;
        const dm_status s = plan_pattern(p, 0, avail, st, &pl, &err);
        CHECK(s == DM_OK, "plan failed: %s", err.c_str());
        if (s != DM_OK) continue;
        check_plan(p, pl, avail);
        std::vector<int32_t> ser = serialize_plan(pl);
        CHECK(!ser.empty() && ser[0] == k, "serialized plan");
        plans++;
    }
    std::printf("plan checks: %d plans, %d failures\n", plans, failures);
    return failures ? 1 : 0;
}

static int run_thread_checks() {
    HostPool pool(7);
    PlanCache cache(64);
    std::atomic<long> sum{0};
    std::vector<std::thread> th;
    for (int c = 0; c < 6; c++) {
        th.emplace_back([&, c] {
            std::mt19937 rng(100 + c);
            for (int it = 0; it < 200; it++) {
                // a batch: every index once, from whichever thread runs it
                std::vector<std::atomic<int>> hit(37);
                for (auto& h : hit) h = 0;
                pool.parallel_for(37, [&](int i) { hit[i]++; });
                for (auto& h : hit) CHECK(h.load() == 1, "index run %d times", h.load());
                // plans shared through the cache
                const int k = 2 + (int)(rng() % 12);
                std::vector<int32_t> e = random_pattern(rng, k, 1);
                dm_graph_desc g{k, (int64_t)e.size() / 2, e.data()};
                NormPattern p;
                std::string err;
                if (normalize_pattern(&g, &p, &err) != DM_OK) continue;
                std::string key((const char*)e.data(), e.size() * sizeof(int32_t));
                Plan pl;
                if (!cache.get(key, &pl)) {
                    CHECK(plan_pattern(p, 0, (1u << kNumMotifs) - 1, nullptr, &pl, &err) == DM_OK, "plan");
                    cache.put(key, pl);
                }
                CHECK(pl.k == k, "cached plan for %d vertices", pl.k);
                sum += pl.k;
            }
        });
    }
    for (auto& t : th) t.join();
    std::printf("thread checks: %ld, %d failures\n", sum.load(), failures);
    return failures ? 1 : 0;
}

int main(int argc, char** argv) {
    const std::string mode = argc > 1 ? argv[1] : "plan";
    if (mode == "plan") return run_plan_checks();
    if (mode == "threads") return run_thread_checks();
    std::fprintf(stderr, "usage: host_checks plan|threads\n");
    return 2;
}
