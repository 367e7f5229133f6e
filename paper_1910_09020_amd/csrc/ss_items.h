// One work item of a plan swept by a whole 256-thread block (four wavefronts):
// the item's pairs go to lanes by its shape (lanes per pair, slices per lane),
// one-lane items stage the words that hold their pairs in LDS when they fit,
// and each pair's result word is written through the permutation.  Shared by
// the batched persistent kernel and the device-resident serving loop.
#pragma once
#include <climits>

#include "ss_common.h"
#include "ss_wave.h"

namespace ss {
namespace item_sweep {

// The sweep with the item's shape as template arguments, so that the vote over
// a pair's lanes compiles to straight-line code.  Shapes from wave::shape_for:
// one lane with 1..RSMAX slices, or several lanes with more than RSMAX/2 slices
// each; any other shape takes the generic form (lanes per pair at run time).
template <int RS, int RSMAX, class LD>
__device__ __forceinline__ int sweep_lanes(int lp, const LD& ld, int64_t b0, int m, int Ei, bool ok, int lip,
                                           int emax)
{
    constexpr bool multi = 2 * RS > RSMAX;          // shapes with several lanes per pair
    switch (lp) {
    case 1: return wave::sweep_pair<RS, 1>(ld, b0, m, Ei, ok, 1, lip, emax);
    case 2: if constexpr (multi) return wave::sweep_pair<RS, 2>(ld, b0, m, Ei, ok, 2, lip, emax); break;
    case 4: if constexpr (multi) return wave::sweep_pair<RS, 4>(ld, b0, m, Ei, ok, 4, lip, emax); break;
    case 8: if constexpr (multi) return wave::sweep_pair<RS, 8>(ld, b0, m, Ei, ok, 8, lip, emax); break;
    case 16: if constexpr (multi) return wave::sweep_pair<RS, 16>(ld, b0, m, Ei, ok, 16, lip, emax); break;
    case 32: if constexpr (multi) return wave::sweep_pair<RS, 32>(ld, b0, m, Ei, ok, 32, lip, emax); break;
    case 64: if constexpr (multi) return wave::sweep_pair<RS, 64>(ld, b0, m, Ei, ok, 64, lip, emax); break;
    default: break;
    }
    return wave::sweep_pair<RS, 0>(ld, b0, m, Ei, ok, lp, lip, emax);
}

template <int RSMAX, class LD>
__device__ __forceinline__ int sweep_shape(int rs, int lp, const LD& ld, int64_t b0, int m, int Ei, bool ok, int lip,
                                           int emax)
{
    switch (rs) {
    case 1: return sweep_lanes<1, RSMAX>(lp, ld, b0, m, Ei, ok, lip, emax);
    case 2: if constexpr (RSMAX >= 2) return sweep_lanes<2, RSMAX>(lp, ld, b0, m, Ei, ok, lip, emax); break;
    case 3: if constexpr (RSMAX >= 3) return sweep_lanes<3, RSMAX>(lp, ld, b0, m, Ei, ok, lip, emax); break;
    case 4: if constexpr (RSMAX >= 4) return sweep_lanes<4, RSMAX>(lp, ld, b0, m, Ei, ok, lip, emax); break;
    case 5: if constexpr (RSMAX >= 5) return sweep_lanes<5, RSMAX>(lp, ld, b0, m, Ei, ok, lip, emax); break;
    case 6: if constexpr (RSMAX >= 6) return sweep_lanes<6, RSMAX>(lp, ld, b0, m, Ei, ok, lip, emax); break;
    case 7: if constexpr (RSMAX >= 7) return sweep_lanes<7, RSMAX>(lp, ld, b0, m, Ei, ok, lip, emax); break;
    case 8: if constexpr (RSMAX >= 8) return sweep_lanes<8, RSMAX>(lp, ld, b0, m, Ei, ok, lip, emax); break;
    default: break;
    }
    return 0;       // no such shape is planned for this slice width
}

// One-lane shapes from a stage in LDS.
template <int RSMAX>
__device__ __forceinline__ int sweep_staged(int rs, const wave::StagedPlanes& ld, int64_t b0, int m, int Ei, bool ok,
                                            int emax)
{
    switch (rs) {
    case 1: return wave::sweep_pair<1, 1>(ld, b0, m, Ei, ok, 1, 0, emax);
    case 2: if constexpr (RSMAX >= 2) return wave::sweep_pair<2, 1>(ld, b0, m, Ei, ok, 1, 0, emax); break;
    case 3: if constexpr (RSMAX >= 3) return wave::sweep_pair<3, 1>(ld, b0, m, Ei, ok, 1, 0, emax); break;
    case 4: if constexpr (RSMAX >= 4) return wave::sweep_pair<4, 1>(ld, b0, m, Ei, ok, 1, 0, emax); break;
    case 5: if constexpr (RSMAX >= 5) return wave::sweep_pair<5, 1>(ld, b0, m, Ei, ok, 1, 0, emax); break;
    case 6: if constexpr (RSMAX >= 6) return wave::sweep_pair<6, 1>(ld, b0, m, Ei, ok, 1, 0, emax); break;
    case 7: if constexpr (RSMAX >= 7) return wave::sweep_pair<7, 1>(ld, b0, m, Ei, ok, 1, 0, emax); break;
    case 8: if constexpr (RSMAX >= 8) return wave::sweep_pair<8, 1>(ld, b0, m, Ei, ok, 1, 0, emax); break;
    default: break;
    }
    return 0;
}

// Per-plane capacity of the LDS stage (words): an item of 256 one-lane pairs
// that lie close together in the stream (the planner keeps them in input
// order) spans about 256 m / 32 words per plane.
constexpr int kStageWords = 2048;

// The item [first, first + count) of the permutation, shape (LP lanes per pair,
// rs slices per lane, row layout for threshold emax); every thread of the
// block calls this with the same item.  s_lo, s_hi: 4 entries each of LDS;
// s_stage: 4 * kStageWords words of LDS.
template <int RSMAX>
__device__ __forceinline__ void sweep_item(int64_t first, int count, int LP, int rs, int emax,
                                           const int64_t* __restrict__ perm, const wave::GlobalPlanes& planes,
                                           const int64_t* __restrict__ offsets, const int32_t* __restrict__ lengths,
                                           const int32_t* __restrict__ Epp, uint16_t* __restrict__ out,
                                           long long* s_lo, long long* s_hi, uint32_t* s_stage)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int PW = 64 / LP;
    const int k = wv * PW + lane / LP;
    const bool ok = k < count;
    const int64_t pi = perm[first + (ok ? k : 0)];
    const int m = ok ? lengths[pi] : 0;
    const int Ei = ok ? Epp[pi] : 0;
    const int lip = lane % LP;
    const int64_t b0 = offsets[pi];
    int c;
    if (LP == 1) {
        // one pair per lane: stage the words that hold the block's pairs, when they fit
        long long lo = (ok && m > 0) ? (long long)(b0 >> 5) : LLONG_MAX;
        long long hi = (ok && m > 0) ? (long long)((b0 + m - 1) >> 5) + 1 : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo = min(lo, (long long)__shfl_xor(lo, o));
            hi = max(hi, (long long)__shfl_xor(hi, o));
        }
        if (lane == 0) { s_lo[wv] = lo; s_hi[wv] = hi; }
        __syncthreads();
        lo = min(min(s_lo[0], s_lo[1]), min(s_lo[2], s_lo[3]));
        hi = max(max(s_hi[0], s_hi[1]), max(s_hi[2], s_hi[3]));
        if (hi > lo && hi - lo <= kStageWords) {
            const int nw = (int)(hi - lo);
#pragma unroll
            for (int p = 0; p < 4; p++) {
                const uint32_t* __restrict__ src = p < 2 ? planes.q + p * planes.SWq : planes.r + (p - 2) * planes.SWr;
                const uint64_t SWp = (uint64_t)(p < 2 ? planes.SWq : planes.SWr);
                // words outside the plane (offsets the caller got wrong) read as zero
                for (int i = threadIdx.x; i < nw; i += 256)
                    s_stage[p * kStageWords + i] = (uint64_t)(lo + i) < SWp ? src[lo + i] : 0u;
            }
            __syncthreads();
            const wave::StagedPlanes ld{s_stage, (int64_t)lo, nw, kStageWords};
            c = sweep_staged<RSMAX>(rs, ld, b0, m, Ei, ok, emax);
        } else {
            c = sweep_shape<RSMAX>(rs, LP, planes, b0, m, Ei, ok, lip, emax);
        }
    } else {
        c = sweep_shape<RSMAX>(rs, LP, planes, b0, m, Ei, ok, lip, emax);
    }
    if (ok && lip == 0) out[pi] = wave::result_word(c, Ei);
}

}  // namespace item_sweep
}  // namespace ss
