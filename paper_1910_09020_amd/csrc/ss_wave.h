// Wavefront-cooperative column sweep: the body shared by the standalone kernel
// and the persistent batched kernel.
//
// LP lanes work on one pair; every lane holds up to RS 32-row slices of the
// 2E+1 rows (slice s = lane_in_pair + LP * t holds rows 32s..32s+31, row index
// r = k + Emax for diagonal offset k).  Each column is one step of the greedy
// walk of Section 2.4 read column-wise: a row still free since the checkpoint
// stays alive if its Equation 1 cell is 0; a wavefront ballot tells whether
// any row of the pair is still alive; if none, the column holds the obstacle
// that closes the longest escape segment: count it, and every row is free
// again from the next column (the new checkpoint).  A pair stops counting once
// its count exceeds its threshold (step 4) and reports min(count, E+1).
#pragma once
#include "ss_common.h"

namespace ss {
namespace wave {

// three-input logic (v_bitop3_b32); truth-table index (src0 << 2) | (src1 << 1) | src2
__device__ __forceinline__ uint32_t and_xnor(uint32_t s, uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_bitop3_b32(s, a, b, 0x90);     // s & ~(a ^ b)
}

// 32 bits of a plane starting at absolute stream bit a (zero outside the buffer)
__device__ __forceinline__ uint32_t bits32(const uint32_t* __restrict__ P, int64_t SW, int64_t a)
{
    const int64_t w = a >> 5;                 // arithmetic shift: floor for negative a
    const uint32_t sh = (uint32_t)(a & 31);
    const uint32_t lo = (w >= 0 && w < SW) ? P[w] : 0u;
    const uint32_t hi = (w + 1 >= 0 && w + 1 < SW) ? P[w + 1] : 0u;
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// bits [lo, hi) of a word set (lo, hi clamped to [0, 32])
__device__ __forceinline__ uint32_t span_mask(int lo, int hi)
{
    lo = lo < 0 ? 0 : (lo > 32 ? 32 : lo);
    hi = hi < 0 ? 0 : (hi > 32 ? 32 : hi);
    if (hi <= lo) return 0u;
    const uint32_t up = hi == 32 ? ~0u : ((1u << hi) - 1u);
    const uint32_t dn = (1u << lo) - 1u;      // lo < 32 here
    return up & ~dn;
}

// Shape for a maximum threshold E: lanes per pair and slices per lane, with at
// most RSMAX slices per lane.
__host__ __device__ inline void shape_for(int32_t E, int RSMAX, int* lp, int* rs)
{
    const int SL = (2 * E + 1 + 31) / 32;
    if (SL <= RSMAX) { *lp = 1; *rs = SL; return; }
    int L = 1;
    while ((int64_t)L * RSMAX < SL) L <<= 1;
    *lp = L;
    *rs = (SL + L - 1) / L;
}

// OR of x over the pair's LP lanes (aligned runs of LP lanes; LP a power of
// two, uniform across the wavefront).  Within 16-lane rows by DPP (quad
// permutes, then half-row and row mirrors), across rows by lane shuffles.
__device__ __forceinline__ uint32_t group_or(uint32_t x, int LP)
{
    if (LP >= 2) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    if (LP >= 4) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    if (LP >= 8) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    if (LP >= 16) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false); // row_mirror
    if (LP >= 32) x |= (uint32_t)__shfl_xor((int)x, 16);
    if (LP >= 64) x |= (uint32_t)__shfl_xor((int)x, 32);
    return x;
}

// One 32-column block of the sweep for the calling lane's RS slices.
// MASK: apply the query-range mask (columns whose rows may index outside [0, m)).
// The per-column bookkeeping is lane-mask arithmetic (finm: all ones once the
// pair's walk has ended), so that a column is straight-line vector code.
template <int RS, bool MASK>
__device__ __forceinline__ void sweep_block(uint32_t (&alive)[RS], const uint32_t (&rmask)[RS],
                                            const uint32_t (&q0lo)[RS], const uint32_t (&q0hi)[RS],
                                            const uint32_t (&q1lo)[RS], const uint32_t (&q1hi)[RS], uint32_t rw0,
                                            uint32_t rw1, int jb, int jend, int m, int Ei, int Emax, int LP,
                                            int lip, int& count, uint32_t& finm)
{
    for (int jj = 0; jj < jend; jj++) {
        const int j = jb + jj;
        const uint32_t rb0 = (uint32_t)__builtin_amdgcn_sbfe((int)rw0, jj, 1);   // reference bit j, broadcast
        const uint32_t rb1 = (uint32_t)__builtin_amdgcn_sbfe((int)rw1, jj, 1);
        uint32_t any = 0;
#pragma unroll
        for (int t = 0; t < RS; t++) {
            const uint32_t x0 = __builtin_amdgcn_alignbit(q0hi[t], q0lo[t], jj);
            const uint32_t x1 = __builtin_amdgcn_alignbit(q1hi[t], q1lo[t], jj);
            uint32_t a = and_xnor(and_xnor(alive[t], x0, rb0), x1, rb1);
            if (MASK) {
                const int base = j - Emax + 32 * (lip + LP * t);      // query position of bit 0
                a &= span_mask(-base, m - base);
            }
            alive[t] = a;
            any |= a;
        }
        any = group_or(any, LP);
        // dead column: no row of the pair still free, the walk not ended, j inside the pair
        const uint32_t live = j < m ? ~finm : 0u;
        const uint32_t deadm = any == 0u ? live : 0u;
        count -= (int)deadm;                                                 // +1 on a dead column
#pragma unroll
        for (int t = 0; t < RS; t++)
            alive[t] = __builtin_amdgcn_bitop3_b32(alive[t], rmask[t], deadm, 0xD8);   // deadm ? rmask : alive
        finm |= (count > Ei ? deadm : 0u) | (j + 1 >= m ? ~0u : 0u);
    }
}

// Sweep one pair with the calling lane's share of its rows.  All 64 lanes of
// the wavefront must call this together (it uses wavefront votes), with the
// same LP.
//   b0, m, Ei   : the pair's stream bit offset, length and threshold
//   pair_ok     : false for lanes without a pair (they still vote)
//   LP, lip     : lanes per pair and this lane's index in its pair
//   RS          : slices this lane holds; Emax: row layout threshold
// Returns the count reported by the walk, min(count, Ei+1).
template <int RS, int LPC>
__device__ __forceinline__ int sweep_pair(const uint32_t* __restrict__ pk, int64_t SW, int64_t b0, int m, int Ei,
                                          bool pair_ok, int LP_rt, int lip, int Emax)
{
    const int LP = LPC > 0 ? LPC : LP_rt;
    const uint32_t* __restrict__ Q0 = pk;
    const uint32_t* __restrict__ Q1 = pk + SW;
    const uint32_t* __restrict__ R0 = pk + 2 * SW;
    const uint32_t* __restrict__ R1 = pk + 3 * SW;
    const int NR = 2 * Emax + 1;

    uint32_t alive[RS], rmask[RS], q0lo[RS], q0hi[RS], q1lo[RS], q1hi[RS], n0[RS], n1[RS];
#pragma unroll
    for (int t = 0; t < RS; t++) {
        const int s = lip + LP * t;
        // rows r in [32s, 32s+32) that exist (r < NR) and whose |r - Emax| <= Ei
        const int lo = Emax - Ei - 32 * s, hi = Emax + Ei + 1 - 32 * s;
        rmask[t] = span_mask(lo, hi < NR - 32 * s ? hi : NR - 32 * s);
        alive[t] = rmask[t];
        q0lo[t] = q0hi[t] = q1lo[t] = q1hi[t] = n0[t] = n1[t] = 0u;
    }
    int count = 0;
    uint32_t finm = (!pair_ok || m == 0) ? ~0u : 0u;
    const bool fin = finm != 0u;
    // interior blocks of columns need no query-range mask for any pair of the wavefront
    int mmin = fin ? 0x7FFFFFFF : m;
    int mmax = fin ? 0 : m;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        mmin = min(mmin, __shfl_xor(mmin, o));
        mmax = max(mmax, __shfl_xor(mmax, o));
    }

    // Query window of slice s for block jb: pair-relative positions jb - Emax + 32 s + [0, 64).
    // The window moves by one word per block, so each block loads only the
    // next high word (and the next reference word), one block ahead.
    if (!fin) {
#pragma unroll
        for (int t = 0; t < RS; t++) {
            const int64_t a = b0 - Emax + 32 * (int64_t)(lip + LP * t);
            q0lo[t] = bits32(Q0, SW, a);
            q1lo[t] = bits32(Q1, SW, a);
            n0[t] = bits32(Q0, SW, a + 32);
            n1[t] = bits32(Q1, SW, a + 32);
        }
    }
    uint32_t nr0 = fin ? 0u : bits32(R0, SW, b0), nr1 = fin ? 0u : bits32(R1, SW, b0);
    for (int jb = 0; jb < mmax; jb += 32) {
        if (__all(finm != 0u)) break;
#pragma unroll
        for (int t = 0; t < RS; t++) { q0hi[t] = n0[t]; q1hi[t] = n1[t]; }
        const uint32_t rw0 = nr0, rw1 = nr1;
        if (jb + 32 < mmax && finm == 0u) {
#pragma unroll
            for (int t = 0; t < RS; t++) {
                const int64_t a = b0 + jb + 64 - Emax + 32 * (int64_t)(lip + LP * t);
                n0[t] = bits32(Q0, SW, a);
                n1[t] = bits32(Q1, SW, a);
            }
            nr0 = bits32(R0, SW, b0 + jb + 32);
            nr1 = bits32(R1, SW, b0 + jb + 32);
        }
        const int jend = min(32, mmax - jb);
        if ((jb >= Emax) && (jb + 31 + Emax < mmin))
            sweep_block<RS, false>(alive, rmask, q0lo, q0hi, q1lo, q1hi, rw0, rw1, jb, jend, m, Ei, Emax, LP, lip,
                                   count, finm);
        else
            sweep_block<RS, true>(alive, rmask, q0lo, q0hi, q1lo, q1hi, rw0, rw1, jb, jend, m, Ei, Emax, LP, lip,
                                  count, finm);
#pragma unroll
        for (int t = 0; t < RS; t++) { q0lo[t] = q0hi[t]; q1lo[t] = q1hi[t]; }
    }
    return count > Ei + 1 ? Ei + 1 : count;
}

__device__ __forceinline__ uint16_t result_word(int count, int Ei)
{
    return (uint16_t)((count <= Ei ? 0x8000u : 0u) | (uint32_t)count);
}

}  // namespace wave
}  // namespace ss
