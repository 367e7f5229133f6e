// Lane-sliced column-sweep kernel template (included by the per-threshold units).
//
// Layout: bit s of every 32-bit word belongs to pair 32*g + s ("group" g, one
// group per lane).  A lane therefore advances 32 pairs by one maze column with
// each bitwise instruction.
//
// The sweep is the greedy walk of Section 2.4 read column by column.  For each
// pair and row k (diagonal offset k in [-E, E], Equation 1) the state bit S_k
// says "row k has been free from the current checkpoint up to the previous
// column".  At column j:
//     a_k  = S_k AND Z[k, j] == 0          (Equation 1 cell, all four cases)
//     dead = no a_k set                    (every row has met its first obstacle:
//                                           column j is the obstacle closing the
//                                           longest escape segment of step 2)
//     count += dead,  S_k = a_k OR dead    (step 3: the next column is the new
//                                           checkpoint, every row free again)
// A run that is still alive after column m-1 reaches the destination and is not
// counted; an obstacle exactly at column m-1 is.  The count is kept as a
// saturating thermometer (t_l = count >= l, l = 1..E+1), which reproduces the
// stop of step 4 (count = E+1 for rejected pairs) without any early exit.
#pragma once
#include "ss_common.h"

namespace ss {
namespace sliced {

// ---------------------------------------------------------------- sweep state
// Three-input logic on gfx950 (v_bitop3_b32); the truth-table index is
// (src0 << 2) | (src1 << 1) | src2.
__device__ __forceinline__ uint32_t and_xnor(uint32_t s, uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_bitop3_b32(s, a, b, 0x90);     // s & ~(a ^ b)
}
__device__ __forceinline__ uint32_t or_not(uint32_t a, uint32_t y)
{
    return __builtin_amdgcn_bitop3_b32(a, y, y, 0xF3);     // a | ~y
}
__device__ __forceinline__ uint32_t or_and_not(uint32_t t, uint32_t p, uint32_t y)
{
    return __builtin_amdgcn_bitop3_b32(t, p, y, 0xF4);     // t | (p & ~y)
}

template <int E>
struct SweepState {
    static constexpr int NR = 2 * E + 1;
    uint32_t S[NR];        // row k = r - E free since the checkpoint (one bit per pair)
    uint32_t T[E + 1];     // T[l-1]: count >= l

    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int r = 0; r < NR; r++) S[r] = ~0u;
#pragma unroll
        for (int l = 0; l <= E; l++) T[l] = 0u;
    }

    // S[r] holds a_r for the column just processed; any = OR of them.
    __device__ __forceinline__ void close_column(uint32_t any)
    {
#pragma unroll
        for (int l = E; l >= 1; l--) T[l] = or_and_not(T[l], T[l - 1], any);
        T[0] = or_not(T[0], any);
#pragma unroll
        for (int r = 0; r < NR; r++) S[r] = or_not(S[r], any);
    }

    // One column: q0/q1 give the query words at position j + (r - E).
    // VALID(r) is false for rows whose query index is outside [0, m).
    template <class Q0, class Q1, class VALID>
    __device__ __forceinline__ void column(uint32_t r0, uint32_t r1, Q0&& q0, Q1&& q1, VALID&& valid)
    {
        uint32_t any = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            uint32_t a = and_xnor(and_xnor(S[r], r0, q0(r)), r1, q1(r));
            if (!valid(r)) a = 0;
            S[r] = a;
            any |= a;
        }
        close_column(any);
    }
};

__device__ __forceinline__ uint32_t comp(const uint4& v, int t)
{
    return t == 0 ? v.x : (t == 1 ? v.y : (t == 2 ? v.z : v.w));
}

__device__ __forceinline__ constexpr int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Interior chunk loop variants.
enum { MAIN_CIRC = 0, MAIN_SHIFT4 = 1 };

// Column-sweep kernel.  Chunks whose columns see a query index outside [0, m)
// (the first EC and the last few) run through a checked path; interior chunks
// run unchecked with the query window held in registers:
//   MAIN_CIRC  : slot = chunk mod W with the loop unrolled W chunks, so every
//                register index is static and the window never moves;
//   MAIN_SHIFT4: four chunks per step, the window shifts by four chunks.
template <int E, int MODE>
__global__ __launch_bounds__(256) void k_sliced(const uint32_t* __restrict__ pk, int64_t G, int m,
                                                int64_t n_pairs, uint16_t* __restrict__ out)
{
    constexpr int NR = 2 * E + 1;
    constexpr int B = kChunk;
    constexpr int EC = (E + B - 1) / B;
    constexpr int W = 2 * EC + 1;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int nch = (m + B - 1) / B;
    const int64_t cstride = G * B;
    const int64_t pstride = (int64_t)nch * cstride;
    const uint32_t* __restrict__ base = pk + g * B;

    auto ld = [&](int plane, int c) -> uint4 {
        return *reinterpret_cast<const uint4*>(base + plane * pstride + (int64_t)c * cstride);
    };
    auto put = [](uint32_t (&d)[B], const uint4& v) { d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w; };
    auto zero = [](uint32_t (&d)[B]) { d[0] = 0; d[1] = 0; d[2] = 0; d[3] = 0; };

    SweepState<E> st;
    st.init();

    // ---- checked chunks [cbeg, cend): window slot i holds chunk c0 - EC + i
    auto checked_range = [&](int cbeg, int cend) {
        if (cbeg >= cend) return;
        uint32_t w0[W][B], w1[W][B];
#pragma unroll
        for (int i = 0; i < W - 1; i++) {
            const int c = cbeg - EC + i;
            if (c >= 0 && c < nch) { put(w0[i], ld(0, c)); put(w1[i], ld(1, c)); }
            else { zero(w0[i]); zero(w1[i]); }
        }
        for (int c0 = cbeg; c0 < cend; c0++) {
            const int cn = c0 + EC;
            if (cn < nch) { put(w0[W - 1], ld(0, cn)); put(w1[W - 1], ld(1, cn)); }
            else { zero(w0[W - 1]); zero(w1[W - 1]); }
            const uint4 rr0 = ld(2, c0), rr1 = ld(3, c0);
#pragma unroll
            for (int t = 0; t < B; t++) {
                const int j = B * c0 + t;
                if (j >= m) break;
                st.column(comp(rr0, t), comp(rr1, t),
                          [&](int r) { const int o = t + r - E, d = floordiv(o, B); return w0[EC + d][o - d * B]; },
                          [&](int r) { const int o = t + r - E, d = floordiv(o, B); return w1[EC + d][o - d * B]; },
                          [&](int r) { const int pos = j + r - E; return pos >= 0 && pos < m; });
            }
#pragma unroll
            for (int i = 0; i < W - 1; i++) {
#pragma unroll
                for (int e = 0; e < B; e++) { w0[i][e] = w0[i + 1][e]; w1[i][e] = w1[i + 1][e]; }
            }
        }
    };

    const int head_end = min(EC, nch);
    checked_range(0, head_end);

    // interior chunks c in [EC, ct) never touch a query index outside [0, m)
    const int ct = (m - B - E >= 0) ? (m - B - E) / B + 1 : 0;
    auto always = [](int) { return true; };
    if (ct > EC) {
        if constexpr (MODE == MAIN_CIRC) {
            uint32_t q0w[W][B], q1w[W][B];
#pragma unroll
            for (int c = 0; c < 2 * EC; c++) { put(q0w[c % W], ld(0, c)); put(q1w[c % W], ld(1, c)); }
            for (int cb = 0; cb < ct; cb += W) {
#pragma unroll
                for (int u = 0; u < W; u++) {
                    const int c0 = cb + u;
                    if (c0 >= EC && c0 < ct) {
                        if (c0 + EC < nch) { put(q0w[(u + EC) % W], ld(0, c0 + EC)); put(q1w[(u + EC) % W], ld(1, c0 + EC)); }
                        const uint4 rr0 = ld(2, c0), rr1 = ld(3, c0);
#pragma unroll
                        for (int t = 0; t < B; t++) {
                            st.column(comp(rr0, t), comp(rr1, t),
                                      [&](int r) { const int o = t + r - E, d = floordiv(o, B); return q0w[(u + d + 2 * W) % W][o - d * B]; },
                                      [&](int r) { const int o = t + r - E, d = floordiv(o, B); return q1w[(u + d + 2 * W) % W][o - d * B]; },
                                      always);
                        }
                    }
                }
            }
        } else {
            constexpr int U = 4;
            constexpr int NW = 2 * EC + U;          // slot i holds chunk cb - EC + i
            uint32_t q0w[NW][B], q1w[NW][B];
#pragma unroll
            for (int i = 0; i < 2 * EC; i++) { put(q0w[i], ld(0, i)); put(q1w[i], ld(1, i)); }
            for (int cb = EC; cb < ct; cb += U) {
                uint4 rr0[U], rr1[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int cn = cb + EC + u;
                    if (cn < nch) { put(q0w[2 * EC + u], ld(0, cn)); put(q1w[2 * EC + u], ld(1, cn)); }
                    if (cb + u < ct) { rr0[u] = ld(2, cb + u); rr1[u] = ld(3, cb + u); }
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    if (cb + u < ct) {
#pragma unroll
                        for (int t = 0; t < B; t++) {
                            st.column(comp(rr0[u], t), comp(rr1[u], t),
                                      [&](int r) { const int o = t + r - E, d = floordiv(o, B); return q0w[EC + u + d][o - d * B]; },
                                      [&](int r) { const int o = t + r - E, d = floordiv(o, B); return q1w[EC + u + d][o - d * B]; },
                                      always);
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < 2 * EC; i++) {
#pragma unroll
                    for (int e = 0; e < B; e++) { q0w[i][e] = q0w[i + U][e]; q1w[i][e] = q1w[i + U][e]; }
                }
            }
        }
    }
    checked_range(max(EC, ct), nch);

    // ---- decide and write (step 5): thermometer -> binary digits, one word per pair
    constexpr int NB = (E + 1) < 2 ? 1 : (E + 1) < 4 ? 2 : (E + 1) < 8 ? 3 : (E + 1) < 16 ? 4 : (E + 1) < 32 ? 5 : 6;
    uint32_t dig[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        uint32_t x = 0;
#pragma unroll
        for (int i = 1; (i << b) <= E + 1; i++) x ^= st.T[(i << b) - 1];
        dig[b] = x;
    }
    const uint32_t acc = ~st.T[E];
    const int64_t p0 = g * 32;
    uint32_t res[16];
#pragma unroll
    for (int s2 = 0; s2 < 16; s2++) {
        uint32_t v[2];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int s = 2 * s2 + h;
            uint32_t x = ((acc >> s) & 1u) << 15;
#pragma unroll
            for (int b = 0; b < NB; b++) x |= ((dig[b] >> s) & 1u) << b;
            v[h] = x;
        }
        res[s2] = v[0] | (v[1] << 16);
    }
    if (p0 + 32 <= n_pairs) {
        uint4* o = reinterpret_cast<uint4*>(out + p0);
#pragma unroll
        for (int q = 0; q < 4; q++) o[q] = make_uint4(res[4 * q], res[4 * q + 1], res[4 * q + 2], res[4 * q + 3]);
    } else {
#pragma unroll
        for (int s = 0; s < 32; s++)
            if (p0 + s < n_pairs) out[p0 + s] = (uint16_t)(res[s >> 1] >> (16 * (s & 1)));
    }
}

template <int E>
hipError_t launch_sliced_E(const uint32_t* packed, int64_t n_pairs, int32_t m, uint16_t* out, hipStream_t s)
{
    const int64_t G = cdiv(n_pairs, 32);
    const int threads = 256;
    const int64_t blocks = cdiv(G, threads);
    constexpr int mode = E <= 10 ? MAIN_CIRC : MAIN_SHIFT4;
    hipLaunchKernelGGL((k_sliced<E, mode>), dim3((unsigned)blocks), dim3(threads), 0, s, packed, G, m, n_pairs, out);
    return hipGetLastError();
}

template <int... Es>
struct SlicedTable {
    static hipError_t run(int E, const uint32_t* packed, int64_t n, int32_t m, uint16_t* out, hipStream_t s)
    {
        hipError_t r = hipErrorInvalidValue;
        ((E == Es ? (r = launch_sliced_E<Es>(packed, n, m, out, s), 0) : 0), ...);
        return r;
    }
};


}  // namespace sliced
}  // namespace ss
