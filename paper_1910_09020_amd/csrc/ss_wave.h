// Wavefront-cooperative column sweep: the body shared by the standalone kernel
// and the persistent batched kernel.
//
// LP lanes work on one pair; every lane holds up to RS 32-row slices of the
// 2E+1 rows (slice s = lane_in_pair + LP * t holds rows 32s..32s+31, row index
// r = k + Emax for diagonal offset k).  Each column is one step of the greedy
// walk of Section 2.4 read column-wise: a row still free since the checkpoint
// stays alive if its Equation 1 cell is 0; an OR over the pair's lanes (lane
// permutes) tells whether any row of the pair is still alive; if none, the
// column holds the obstacle that closes the longest escape segment: count it,
// and every row is free again from the next column (the new checkpoint).  A
// pair stops counting once its count exceeds its threshold (step 4, taken at
// 32-column block boundaries) and reports min(count, E+1).
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

// Word loaders for the sweep: word(p, w) returns word w of plane p (0, 1:
// query; 2, 3: reference), zero outside the plane.
//
// From HBM through buffer loads: the hardware range check returns zero for an
// offset past the plane, and every word index outside [0, SW) (negative ones
// included) is sent to one such offset, so each load is issued
// unconditionally, with no branch around it.  A plane must be smaller than
// 2^30 - 64 words (SS_MAX_STREAM_BASES).
// The query planes (0, 1) and the reference planes (2, 3) may live in two
// buffers of their own sizes (each side packed by itself), or in one buffer of
// four planes of SW words (four()).
struct GlobalPlanes {
    const uint32_t* q;       // plane p = 0, 1 at q + p * SWq
    const uint32_t* r;       // plane p = 2, 3 at r + (p - 2) * SWr
    int64_t SWq, SWr;
    __device__ __forceinline__ static GlobalPlanes four(const uint32_t* pk, int64_t SW)
    {
        return GlobalPlanes{pk, pk + 2 * SW, SW, SW};
    }
    __device__ __forceinline__ uint32_t word(int p, int w) const
    {
        const int64_t SW = p < 2 ? SWq : SWr;
        const uint32_t* base = p < 2 ? q + p * SWq : r + (p - 2) * SWr;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint32_t*>(base), (short)0, (int)(uint32_t)(SW * 4), 0x00020000);
        const uint32_t off = (uint32_t)w < (uint32_t)SW ? (uint32_t)w << 2 : 0xFFFFFFF0u;
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    }
};

// Words [lo, lo + nw) of each plane staged in LDS (plane p at st + p * cap);
// words outside read as zero.  Every bit that can change a result lies inside
// some pair's own [b0, b0 + m), so a stage that covers those spans of the
// pairs being swept gives the same results as the global loader.
struct StagedPlanes {
    const uint32_t* st;
    int64_t lo;
    int nw, cap;
    __device__ __forceinline__ uint32_t word(int p, int w) const
    {
        const int i = (int)(w - lo);
        return (unsigned)i < (unsigned)nw ? st[p * cap + i] : 0u;
    }
};

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
// permutes, then half-row and row mirrors), across rows by the permlane swaps
// (rows 0<->1 and 2<->3, then the two halves), all vector ALU operations.
__device__ __forceinline__ uint32_t group_or(uint32_t x, int LP)
{
    if (LP >= 2) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    if (LP >= 4) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    if (LP >= 8) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    if (LP >= 16) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false); // row_mirror
    if (LP >= 32) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        x = r[0] | r[1];
    }
    if (LP >= 64) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        x = r[0] | r[1];
    }
    return x;
}

// A lane's share of one pair's sweep.  Slice t of the lane holds rows
// 32 s .. 32 s + 31 with s = lane_in_pair + LP t; within a 32-column block
// starting at column jb, bit p of the 64-bit windows (hi:lo) of slice t stands
// for query position jb - Emax + 32 s + p (pair-relative), so that column
// jb + c reads bits [c, c + 32): row r = 32 s + p meets query position
// j + r - Emax, as Equation 1 places the diagonals.
template <int RS>
struct Share {
    uint32_t alive[RS];     // rows free since the checkpoint
    uint32_t rmask[RS];     // rows of the pair: |r - Emax| <= E_pair and r < 2 Emax + 1
    uint32_t nfin;          // all ones while the walk goes on, 0 once it has ended
    int slack;              // E_pair - obstacles counted
};

// Block windows: query planes, the validity plane (query position in [0, m)),
// and the block's 32 reference bits.
template <int RS>
struct Win {
    uint32_t q0lo[RS], q0hi[RS], q1lo[RS], q1hi[RS], vlo[RS], vhi[RS];
    uint32_t r0, r1;
};

// v_bitop3 truth table: src2 ? src1 : src0
constexpr int kSelect = 0xD8;

// One column of the walk at window shift sh.  MASK: AND each row with the
// validity plane (rows whose query position falls outside [0, m) hold
// obstacles); END: the pair's last column may lie in this block (column j).
// A column where none of the pair's rows is still free holds the obstacle
// that ends the longest escape segment: count it while the walk goes on and
// free every row of the pair again from the next column.  The stop once the
// count exceeds the threshold is taken at block boundaries: counting a few
// columns further changes neither min(count, E+1) nor the decision.
template <int RS, int LPC, bool MASK, bool END>
__device__ __forceinline__ void column(Share<RS>& S, const Win<RS>& W, int sh, int LP_rt, int j, int m)
{
    const int LP = LPC > 0 ? LPC : LP_rt;
    const uint32_t rb0 = (uint32_t)__builtin_amdgcn_sbfe((int)W.r0, sh, 1);   // reference bit, broadcast
    const uint32_t rb1 = (uint32_t)__builtin_amdgcn_sbfe((int)W.r1, sh, 1);
    uint32_t any = 0;
#pragma unroll
    for (int t = 0; t < RS; t++) {
        const uint32_t x0 = __builtin_amdgcn_alignbit(W.q0hi[t], W.q0lo[t], sh);
        const uint32_t x1 = __builtin_amdgcn_alignbit(W.q1hi[t], W.q1lo[t], sh);
        uint32_t a = and_xnor(and_xnor(S.alive[t], x0, rb0), x1, rb1);
        if (MASK) a &= __builtin_amdgcn_alignbit(W.vhi[t], W.vlo[t], sh);
        S.alive[t] = a;
        any |= a;
    }
    any = group_or(any, LP);
    const uint32_t deadm = any == 0u ? S.nfin : 0u;
    S.slack += (int)deadm;                                               // -1 on a counted obstacle
    if (END) S.nfin = j + 1 >= m ? 0u : S.nfin;
#pragma unroll
    for (int t = 0; t < RS; t++) S.alive[t] = __builtin_amdgcn_bitop3_b32(S.alive[t], S.rmask[t], deadm, kSelect);
}

// Move every window of a block by 16 bit positions.
template <int RS, bool MASK>
__device__ __forceinline__ void advance16(Win<RS>& W)
{
#pragma unroll
    for (int t = 0; t < RS; t++) {
        W.q0lo[t] = __builtin_amdgcn_alignbit(W.q0hi[t], W.q0lo[t], 16);
        W.q0hi[t] >>= 16;
        W.q1lo[t] = __builtin_amdgcn_alignbit(W.q1hi[t], W.q1lo[t], 16);
        W.q1hi[t] >>= 16;
        if (MASK) {
            W.vlo[t] = __builtin_amdgcn_alignbit(W.vhi[t], W.vlo[t], 16);
            W.vhi[t] >>= 16;
        }
    }
    W.r0 >>= 16;
    W.r1 >>= 16;
}

// A full block of 32 columns as two passes of one 16-column body with
// immediate shifts.
template <int RS, int LPC, bool MASK>
__device__ __forceinline__ void block_full(Share<RS>& S, Win<RS> W, int LP)
{
#pragma nounroll
    for (int h = 0; h < 2; h++) {
#pragma unroll
        for (int c = 0; c < 16; c++) column<RS, LPC, MASK, false>(S, W, c, LP, 0, 0);
        if (h == 0) advance16<RS, MASK>(W);
    }
}

// A block in which a pair's walk may end: jend columns (uniform), masked, with
// the end-of-pair test on every column.
template <int RS, int LPC>
__device__ __forceinline__ void block_end(Share<RS>& S, const Win<RS>& W, int LP, int jb, int jend, int m)
{
    for (int c = 0; c < jend; c++) column<RS, LPC, true, true>(S, W, c, LP, jb + c, m);
}

// Sweep one pair with the calling lane's share of its rows.  All 64 lanes of
// the wavefront must call this together (it uses wavefront votes and lane
// permutes), with the same LP.
//   ld          : window loader (GlobalPlanes or StagedPlanes)
//   bq, br      : stream bit offsets of the pair's query and reference
//   m           : columns walked (the reference's length for pairs of equal
//                 length; see columns_walked for pairs of unequal length)
//   nq          : the query's length (cells whose query position falls outside
//                 [0, nq) are obstacles, the fourth case of Equation 1)
//   Ei          : the pair's threshold
//   pair_ok     : false for lanes without a pair (they still take part)
//   LP, lip     : lanes per pair and this lane's index in its pair
//   RS          : slices this lane holds; Emax: row layout threshold
// Returns the count reported by the walk, min(count, Ei+1).
template <int RS, int LPC, class LD>
__device__ __forceinline__ int sweep_pair2(const LD& ld, int64_t bq, int64_t br, int m, int nq, int Ei, bool pair_ok,
                                           int LP_rt, int lip, int Emax)
{
    const int LP = LPC > 0 ? LPC : LP_rt;
    const int NR = 2 * Emax + 1;

    Share<RS> S;
    Win<RS> W;
    uint32_t n0[RS], n1[RS];
#pragma unroll
    for (int t = 0; t < RS; t++) {
        const int s = lip + LP * t;
        // rows r in [32s, 32s+32) that exist (r < NR) and whose |r - Emax| <= Ei
        const int lo = Emax - Ei - 32 * s, hi = Emax + Ei + 1 - 32 * s;
        S.rmask[t] = span_mask(lo, hi < NR - 32 * s ? hi : NR - 32 * s);
        S.alive[t] = S.rmask[t];
        W.vlo[t] = W.vhi[t] = 0u;
    }
    S.nfin = (!pair_ok || m == 0) ? 0u : ~0u;
    S.slack = pair_ok ? Ei : 0;
    int mmax = S.nfin != 0u ? m : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mmax = max(mmax, __shfl_xor(mmax, o));

    // Window words.  Slice t's query window at block jb starts at stream bit
    // bq - Emax + 32 s + jb, i.e. at bit shq of word wq + s + jb/32; the
    // reference bits of block jb start at bit shr of word wr + jb/32.  The
    // window moves by one word per block, so each block loads one new word
    // per plane and slice (and per reference plane), one block ahead, and
    // keeps the last one (c0, c1, cr0, cr1) for the next funnel shift.
    const int64_t aq = bq - Emax;
    const int wq = (int)(aq >> 5), wr = (int)(br >> 5);       // arithmetic shift: floor
    const uint32_t shq = (uint32_t)(aq & 31), shr = (uint32_t)(br & 31);
    uint32_t c0[RS], c1[RS];
#pragma unroll
    for (int t = 0; t < RS; t++) {
        const int w = wq + lip + LP * t;
        const uint32_t a0 = ld.word(0, w), b0w = ld.word(0, w + 1), d0 = ld.word(0, w + 2);
        const uint32_t a1 = ld.word(1, w), b1w = ld.word(1, w + 1), d1 = ld.word(1, w + 2);
        W.q0lo[t] = __builtin_amdgcn_alignbit(b0w, a0, shq);
        W.q1lo[t] = __builtin_amdgcn_alignbit(b1w, a1, shq);
        n0[t] = __builtin_amdgcn_alignbit(d0, b0w, shq);
        n1[t] = __builtin_amdgcn_alignbit(d1, b1w, shq);
        c0[t] = d0;
        c1[t] = d1;
    }
    uint32_t cr0 = ld.word(2, wr + 1), cr1 = ld.word(3, wr + 1);
    uint32_t nr0 = __builtin_amdgcn_alignbit(cr0, ld.word(2, wr), shr);
    uint32_t nr1 = __builtin_amdgcn_alignbit(cr1, ld.word(3, wr), shr);
    for (int jb = 0; jb < mmax; jb += 32) {
        S.nfin = S.slack < 0 ? 0u : S.nfin;                             // the count exceeds the threshold: stop
        if (!__any(S.nfin != 0u)) break;
#pragma unroll
        for (int t = 0; t < RS; t++) { W.q0hi[t] = n0[t]; W.q1hi[t] = n1[t]; }
        W.r0 = nr0;
        W.r1 = nr1;
        if (jb + 32 < mmax) {
            const int k = jb >> 5;
#pragma unroll
            for (int t = 0; t < RS; t++) {
                const int w = wq + lip + LP * t + k + 3;
                const uint32_t x0 = ld.word(0, w), x1 = ld.word(1, w);
                n0[t] = __builtin_amdgcn_alignbit(x0, c0[t], shq);
                n1[t] = __builtin_amdgcn_alignbit(x1, c1[t], shq);
                c0[t] = x0;
                c1[t] = x1;
            }
            const uint32_t y0 = ld.word(2, wr + k + 2), y1 = ld.word(3, wr + k + 2);
            nr0 = __builtin_amdgcn_alignbit(y0, cr0, shr);
            nr1 = __builtin_amdgcn_alignbit(y1, cr1, shr);
            cr0 = y0;
            cr1 = y1;
        }
        // block kind, uniform over the wavefront: a walking pair ends here;
        // some row may meet a query position outside [0, nq); neither
        const bool end = __any(S.nfin != 0u && m <= jb + 32);
        const bool mask = end || jb < Emax || __any(S.nfin != 0u && nq <= jb + 31 + Emax);
        if (mask) {
#pragma unroll
            for (int t = 0; t < RS; t++) {
                const int base = jb - Emax + 32 * (lip + LP * t);      // query position of window bit 0
                W.vlo[t] = span_mask(-base, nq - base);
                W.vhi[t] = span_mask(-base - 32, nq - base - 32);
            }
        }
        if (end)
            block_end<RS, LPC>(S, W, LP, jb, min(32, mmax - jb), m);
        else if (mask)
            block_full<RS, LPC, true>(S, W, LP);
        else
            block_full<RS, LPC, false>(S, W, LP);
#pragma unroll
        for (int t = 0; t < RS; t++) { W.q0lo[t] = W.q0hi[t]; W.q1lo[t] = W.q1hi[t]; }
    }
    const int count = Ei - S.slack;
    return count > Ei + 1 ? Ei + 1 : count;
}

// Pairs of equal length m: query and reference at the same stream offset.
template <int RS, int LPC, class LD>
__device__ __forceinline__ int sweep_pair(const LD& ld, int64_t b0, int m, int Ei, bool pair_ok, int LP_rt, int lip,
                                          int Emax)
{
    return sweep_pair2<RS, LPC>(ld, b0, b0, m, m, Ei, pair_ok, LP_rt, lip, Emax);
}

// Columns walked for a reference of m bases and a query of n (unequal lengths,
// the note of Section 2.4 between steps 4 and 5): the maze over the longer
// sequence holds a comparison of two existing characters only in columns
// 1 .. min(m, n + E) (none when n = 0); the obstacles the walk meets beyond
// them are the trailing ones caused by the fourth case of Equation 1, which
// are deducted before the decision, so the walk stops there.  For m = n this
// is m.
__host__ __device__ __forceinline__ int columns_walked(int m, int n, int E)
{
    if (n <= 0 || m <= 0) return 0;
    return (int64_t)n + E < (int64_t)m ? n + E : m;
}

__device__ __forceinline__ uint16_t result_word(int count, int Ei)
{
    return (uint16_t)((count <= Ei ? 0x8000u : 0u) | (uint32_t)count);
}

}  // namespace wave
}  // namespace ss
