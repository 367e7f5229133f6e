// Drives the oracle and the host planner over random and edge-case inputs in a
// build with AddressSanitizer and UndefinedBehaviorSanitizer (host code only;
// nothing here touches a GPU).  Exits non-zero on the first inconsistency; the
// sanitizers abort on the first memory or undefined-behaviour error.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "ss_arena.h"

extern "C" {
typedef struct { int64_t checkpoints, c_last, cells; } ss_oracle_stats;
int ss_oracle_pair_ex(const uint8_t* R, const uint8_t* Q, int m, int E, int stop_early, int32_t* edits,
                      ss_oracle_stats* st, int32_t* seg_rows, int32_t* seg_ends, int cap, int32_t* nseg);
int ss_oracle_submaze(const uint8_t* R, const uint8_t* Q, int m, int E, int t, int stop_early, int32_t* edits);
int ss_oracle_min_obstacles(const uint8_t* R, const uint8_t* Q, int m, int E);
int ss_oracle_levenshtein(const uint8_t* a, int la, const uint8_t* b, int lb);
int ss_oracle_pair_uneq(const uint8_t* R, int m, const uint8_t* Q, int n, int E, int32_t* edits, int32_t* full,
                        int32_t* net_out);
double ss_oracle_batch(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets, const int32_t* lengths,
                       int64_t n, const int32_t* E_per_pair, int32_t E, int threads, int stop_early, uint8_t* accept,
                       int32_t* edits, int64_t* stats);
int ss_plan_items_host(const int32_t* lengths, const int32_t* E_per_pair, int64_t n_pairs, int32_t slices_per_lane,
                       int64_t* n_items, int64_t* items, int64_t max_items, int64_t* perm);
}

static int fail(const char* what, long a, long b)
{
    std::fprintf(stderr, "FAIL %s (%ld, %ld)\n", what, a, b);
    return 1;
}

int main()
{
    std::mt19937_64 rng(19100902);
    const char* A = "ACGT";
    // oracle: pairs of equal and unequal length, every threshold from 0 to beyond the length
    for (int it = 0; it < 3000; it++) {
        const int m = (int)(rng() % 40), n = (int)(rng() % 40);
        std::vector<uint8_t> R(m + 1), Q(n + 1), Qe(m + 1);
        for (int i = 0; i < m; i++) R[i] = (uint8_t)A[rng() % 4];
        for (int i = 0; i < n; i++) Q[i] = (uint8_t)A[rng() % 4];
        for (int i = 0; i < m; i++) Qe[i] = rng() % 5 ? R[i] : (uint8_t)A[rng() % 4];
        const int E = (int)(rng() % (m + 3));
        int32_t ed = -1, full = -1, net = -1;
        ss_oracle_stats st;
        std::vector<int32_t> rows(4), ends(4);      // room for fewer segments than a walk may take
        int32_t nseg = -1;
        const int acc = ss_oracle_pair_ex(R.data(), Qe.data(), m, E, (int)(rng() & 1), &ed, &st, rows.data(),
                                          ends.data(), 4, &nseg);
        if (nseg < 0 || st.c_last > m) return fail("segments", nseg, (long)st.c_last);
        const int lev = ss_oracle_levenshtein(R.data(), m, Qe.data(), m);
        if (lev <= E && !acc) return fail("lossless", lev, E);
        if (ed < 0) return fail("count", ed, 0);
        const int mo = ss_oracle_min_obstacles(R.data(), Qe.data(), m, E);
        if (mo < 0) return fail("min_obstacles", mo, 0);
        for (int t = 1; t <= m + 2; t += 1 + (int)(rng() % 4)) {
            int32_t se = -1;
            (void)ss_oracle_submaze(R.data(), Qe.data(), m, E, t, (int)(rng() & 1), &se);
            if (se < 0) return fail("submaze", se, t);
        }
        const int ua = ss_oracle_pair_uneq(R.data(), m, Q.data(), n, E, &ed, &full, &net);
        const int ul = ss_oracle_levenshtein(R.data(), m, Q.data(), n);
        if (ul <= E && !ua) return fail("lossless unequal", ul, E);
    }
    // batch with per-pair thresholds on several threads
    {
        const int64_t np = 2000;
        std::vector<int32_t> len(np), Ep(np);
        std::vector<int64_t> off(np);
        int64_t tot = 0;
        for (int64_t p = 0; p < np; p++) {
            len[p] = (int32_t)(rng() % 300);
            Ep[p] = (int32_t)(rng() % 20);
            off[p] = tot;
            tot += len[p];
        }
        std::vector<uint8_t> rd(tot + 1), rf(tot + 1), acc(np);
        for (int64_t i = 0; i < tot; i++) {
            rd[i] = (uint8_t)A[rng() % 4];
            rf[i] = rng() % 8 ? rd[i] : (uint8_t)A[rng() % 4];
        }
        std::vector<int32_t> ed(np);
        std::vector<int64_t> stats(np * 3);
        (void)ss_oracle_batch(rd.data(), rf.data(), off.data(), len.data(), np, Ep.data(), 0, 4, 1, acc.data(),
                              ed.data(), stats.data());
        for (int64_t p = 0; p < np; p++)
            if (acc[p] > 1 || ed[p] < 0) return fail("batch", (long)p, ed[p]);
    }
    // planner: the items cover every pair once, in shapes that fit the slice width
    for (int it = 0; it < 400; it++) {
        const int64_t np = (int64_t)(rng() % 3000);
        std::vector<int32_t> len(np + 1), Ep(np + 1);
        for (int64_t p = 0; p < np; p++) {
            len[p] = (int32_t)(rng() % 3 == 0 ? rng() % 20000 : rng() % 300);
            Ep[p] = (int32_t)(rng() % 4 == 0 ? rng() % 9000 : rng() % 40);
        }
        const int32_t rs = 1 << (rng() % 4);
        int64_t ni = -1;
        const int rc = ss_plan_items_host(len.data(), Ep.data(), np, rs, &ni, nullptr, 0, nullptr);
        if (rc != 0) continue;                   // a threshold too large for this slice width is refused
        std::vector<int64_t> items((size_t)ni * 5 + 5), perm((size_t)np + 1);
        int64_t ni2 = -1;
        if (ss_plan_items_host(len.data(), Ep.data(), np, rs, &ni2, items.data(), ni, perm.data()) != 0 || ni2 != ni)
            return fail("planner repeat", (long)ni, (long)ni2);
        std::vector<char> seen((size_t)np + 1, 0);
        for (int64_t p = 0; p < np; p++) {
            if (perm[p] < 0 || perm[p] >= np || seen[(size_t)perm[p]]) return fail("permutation", (long)p, (long)perm[p]);
            seen[(size_t)perm[p]] = 1;
        }
        int64_t covered = 0;
        for (int64_t k = 0; k < ni; k++) {
            const int64_t first = items[5 * k], cnt = items[5 * k + 1], lp = items[5 * k + 2], r = items[5 * k + 3];
            if (first < 0 || cnt <= 0 || first + cnt > np || lp < 1 || lp > 64 || r < 1 || r > 8)
                return fail("item", (long)k, (long)first);
            covered += cnt;
        }
        if (covered != np) return fail("coverage", (long)covered, (long)np);
    }
    // the serving arena's first-fit allocator: random allocations and releases never overlap, stay
    // inside the arena, and the free ranges merge back into one at the end
    for (int it = 0; it < 200; it++) {
        const size_t cap = 256 * (1 + rng() % 4096);
        Arena ar;
        ar.reset(cap);
        std::vector<std::pair<size_t, size_t>> live;
        for (int op = 0; op < 400; op++) {
            if (live.empty() || rng() % 3) {
                const size_t want = 256 * (1 + rng() % 64);
                size_t off = 0;
                if (!ar.alloc(want, &off)) continue;
                if (off + want > cap) return fail("arena bound", (long)off, (long)want);
                for (auto& l : live)
                    if (off < l.first + l.second && l.first < off + want) return fail("arena overlap", (long)off, (long)l.first);
                live.emplace_back(off, want);
            } else {
                const size_t k = rng() % live.size();
                ar.release(live[k].first, live[k].second);
                live.erase(live.begin() + (long)k);
            }
        }
        for (auto& l : live) ar.release(l.first, l.second);
        if (ar.free_ranges.size() != 1 || ar.free_ranges.begin()->first != 0 || ar.free_ranges.begin()->second != cap)
            return fail("arena merge", (long)ar.free_ranges.size(), (long)cap);
    }
    std::printf("sanitized drive: ok\n");
    return 0;
}
