// Host planner of the batched launch (pure host code; the kernels that run the
// plans are in ss_batch.hip).
//
// Every pair gets a shape class from its threshold (lanes per pair LP and
// 32-row slices per lane rs, see wave::shape_for).  Pairs are sorted by class
// and length, cut into work items of one block-round (four wavefronts of
// 64 / LP pairs each) and the items are ordered by estimated cost, largest
// first (in levels of powers of four, by input position within a level), so
// that the long pairs start early, the short ones fill in behind, and short
// items that read the same stretch of the input run together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "ss.h"
#include "ss_common.h"
#include "ss_wave.h"

namespace ss {

int plan_min_slices(const int32_t* E, int64_t n)
{
    int32_t emax = 0;
    for (int64_t i = 0; i < n; i++) emax = std::max(emax, E[i]);
    const int64_t slices = cdiv(2 * (int64_t)emax + 1, 32);
    for (int rs = 1; rs <= 8; rs <<= 1)
        if (64 * (int64_t)rs >= slices) return rs;
    return 0;
}

bool plan_items(const int32_t* lengths, const int32_t* E, int64_t n, int rsmax, std::vector<PItem>& items,
                std::vector<int64_t>& perm, int* n_classes, double* est_cost)
{
    items.clear();
    perm.clear();
    *n_classes = 0;
    *est_cost = 0;
    // shape class per pair, numbered in order of first appearance (lanes per pair a power of two
    // up to 64, slices per lane 1..8: a table of the (lp, rs) seen so far)
    std::vector<int32_t> cls((size_t)n);
    int class_id[7][9];
    for (auto& row : class_id)
        for (int& x : row) x = -1;
    std::vector<std::pair<int, int>> shapes;
    for (int64_t i = 0; i < n; i++) {
        int lp, rs;
        wave::shape_for(E[i], rsmax, &lp, &rs);
        if (lp > 64) return false;          // more rows than a wavefront holds at this width
        if (rs < 1 || rs > 8) return false;
        const int l2 = 31 - __builtin_clz((unsigned)lp);
        int& id = class_id[l2][rs];
        if (id < 0) {
            id = (int)shapes.size();
            shapes.emplace_back(lp, rs);
        }
        cls[(size_t)i] = id;
    }
    *n_classes = (int)shapes.size();
    // Sort by (class, chunk, length desc, E desc): pairs of one wavefront share
    // the column loop.  One-lane classes are cut in chunks of one block round
    // (256 pairs) in input order and sorted within a chunk, so that an item's
    // pairs lie close together in the stream (the kernel stages them in LDS);
    // other classes form a single chunk.
    std::vector<int64_t> chunk((size_t)n, 0);
    {
        std::vector<int64_t> seen(shapes.size(), 0);
        for (int64_t i = 0; i < n; i++) {
            const int c = cls[(size_t)i];
            if (shapes[(size_t)c].first == 1) chunk[(size_t)i] = seen[(size_t)c]++ / 256;
        }
    }
    // one 128-bit key per pair holding the whole order, the pair's index last (so the sort is
    // stable): class (6 bits), chunk (34), length descending (25), threshold descending (15),
    // index (48).  A comparator reaching into four arrays through the permutation cost a request
    // of 4,000 pairs half a millisecond, and one comparing two words a third of one.
    if (n >= ((int64_t)1 << 42)) return false;
    std::vector<unsigned __int128> key((size_t)n);
    for (int64_t i = 0; i < n; i++) {
        if (lengths[i] < 0 || lengths[i] > SS_MAX_LEN || E[i] < 0 || E[i] > SS_MAX_E) return false;
        const uint64_t hi = ((uint64_t)(uint32_t)cls[(size_t)i] << 58) | ((uint64_t)chunk[(size_t)i] << 24) |
                            (uint64_t)(SS_MAX_LEN - lengths[i]) >> 1;
        const uint64_t lo = ((uint64_t)((SS_MAX_LEN - lengths[i]) & 1) << 63) |
                            ((uint64_t)(SS_MAX_E - E[i]) << 48) | (uint64_t)i;
        key[(size_t)i] = ((unsigned __int128)hi << 64) | lo;
    }
    std::sort(key.begin(), key.end());
    perm.resize((size_t)n);
    for (int64_t i = 0; i < n; i++) perm[(size_t)i] = (int64_t)(uint64_t)(key[(size_t)i] & (((unsigned __int128)1 << 48) - 1));
    // cut into items of one block-round
    items.clear();
    std::vector<double> cost;
    *est_cost = 0;
    int64_t i = 0;
    while (i < n) {
        const int c = cls[(size_t)perm[(size_t)i]];
        const int lp = shapes[(size_t)c].first, rs = shapes[(size_t)c].second;
        const int per_item = 4 * (64 / lp);
        int64_t j = i;
        int32_t emax = 0;
        double work = 0;
        int64_t mmax = 0;
        while (j < n && j - i < per_item && cls[(size_t)perm[(size_t)j]] == c) {
            const int64_t p = perm[(size_t)j];
            emax = std::max(emax, E[p]);
            mmax = std::max<int64_t>(mmax, lengths[p]);
            j++;
        }
        // a block-round costs its longest pair's columns times the lanes' slices
        work = (double)mmax * (double)rs * (double)(4 * 64) / 64.0;
        PItem it;
        it.first = i;
        it.count = (int32_t)(j - i);
        it.lp = (int16_t)lp;
        it.rs = (int16_t)rs;
        it.emax = emax;
        it.pad = 0;
        items.push_back(it);
        cost.push_back(work);
        *est_cost += work;
        i = j;
    }
    // Largest items first, by cost level (powers of four).  The estimate above
    // cannot see where a walk stops; a pair with a larger threshold tends to
    // walk further before its count exceeds it, so within a level items of
    // several lanes per pair go by threshold (powers of two, largest first).
    // Then by the position of the item's first pair in the input, so that
    // items of different (length, threshold) groups that read the same
    // stretch of the bit stream run at about the same time and share its
    // cache lines (one-lane items, which the kernel stages, rely on that).
    std::vector<size_t> order(items.size());
    std::iota(order.begin(), order.end(), (size_t)0);
    std::vector<int> level(items.size()), elevel(items.size());
    for (size_t k = 0; k < items.size(); k++) {
        int l = 0;
        for (double c = cost[k]; c >= 4.0; c *= 0.25) l++;
        level[k] = l;
        int e = 0;
        if (items[k].lp > 1)
            for (int64_t v = (int64_t)items[k].emax + 1; v > 1; v >>= 1) e++;
        elevel[k] = e;
    }
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        if (level[a] != level[b]) return level[a] > level[b];
        if (elevel[a] != elevel[b]) return elevel[a] > elevel[b];
        return perm[(size_t)items[a].first] < perm[(size_t)items[b].first];
    });
    std::vector<PItem> sorted;
    sorted.reserve(order.size());
    for (size_t k : order) sorted.push_back(items[k]);
    items.swap(sorted);
    return true;
}

int validate_plan_inputs(const int32_t* lengths, const int32_t* E, int64_t n)
{
    if (n < 0) return SS_EINVAL;
    if (n > 0 && (!lengths || !E)) return SS_EINVAL;
    for (int64_t i = 0; i < n; i++) {
        if (lengths[i] < 0 || E[i] < 0) return SS_EINVAL;
        if (lengths[i] > SS_MAX_LEN || E[i] > SS_MAX_E) return SS_ELEN;
    }
    return SS_OK;
}

}  // namespace ss

using namespace ss;

extern "C" int ss_plan_items_host(const int32_t* lengths, const int32_t* E_per_pair, int64_t n_pairs,
                                  int32_t slices_per_lane, int64_t* n_items, int64_t* items, int64_t max_items,
                                  int64_t* perm)
{
    if (!n_items) return SS_EINVAL;
    if (slices_per_lane != 1 && slices_per_lane != 2 && slices_per_lane != 4 && slices_per_lane != 8) return SS_EINVAL;
    int rc = validate_plan_inputs(lengths, E_per_pair, n_pairs);
    if (rc != SS_OK) return rc;
    if (n_pairs == 0) { *n_items = 0; return SS_OK; }
    const int rsmin = plan_min_slices(E_per_pair, n_pairs);
    if (rsmin == 0) return SS_ELEN;
    try {
        std::vector<PItem> it;
        std::vector<int64_t> pm;
        int nc = 0;
        double cost = 0;
        if (!plan_items(lengths, E_per_pair, n_pairs, std::max<int>(slices_per_lane, rsmin), it, pm, &nc, &cost))
            return SS_ELEN;
        *n_items = (int64_t)it.size();
        if (items)
            for (int64_t k = 0; k < std::min<int64_t>(max_items, (int64_t)it.size()); k++) {
                items[5 * k + 0] = it[(size_t)k].first;
                items[5 * k + 1] = it[(size_t)k].count;
                items[5 * k + 2] = it[(size_t)k].lp;
                items[5 * k + 3] = it[(size_t)k].rs;
                items[5 * k + 4] = it[(size_t)k].emax;
            }
        if (perm) std::memcpy(perm, pm.data(), pm.size() * sizeof(int64_t));
    } catch (const std::bad_alloc&) {
        return SS_ENOMEM;
    }
    return SS_OK;
}

