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
#include <algorithm>
#include "ss_sliced_ops.h"

namespace ss {
namespace sliced {

// ---------------------------------------------------------------- sweep state
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

    // a new checkpoint without an obstacle: every row free again (a sub-maze boundary)
    __device__ __forceinline__ void restart()
    {
#pragma unroll
        for (int r = 0; r < NR; r++) S[r] = ~0u;
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

    // One column: q0(r)/q1(r) give the query words at position j + (r - E).
    // MASKED: vm(r) is all ones for rows whose query index lies in [0, m) and
    // zero for the others (their cells are obstacles, the fourth case of
    // Equation 1).
    template <bool MASKED, class Q0, class Q1, class VM>
    __device__ __forceinline__ void column(uint32_t r0, uint32_t r1, Q0&& q0, Q1&& q1, VM&& vm)
    {
        uint32_t any = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            uint32_t a = and_xnor(and_xnor(S[r], r0, q0(r)), r1, q1(r));
            if constexpr (MASKED) a &= vm(r);
            S[r] = a;
            any |= a;
        }
        close_column(any);
    }
};


// Window loop variants.
enum { MAIN_CIRC = 0, MAIN_SHIFT4 = 1 };
// Thresholds that sweep with one window over the whole pair, its loads running
// a chunk ahead; the others take the three-part sweep (sweep_group_seams) with
// four-chunk steps.  Chosen per E from measurements on 30 M x 100 bp and
// 10 M x 250 bp, one window against three parts: E = 8..10 6-15% faster,
// E = 11 and 12 up to 8% and 5% slower, E = 13..16 5-8% faster, E = 18 and 20
// three times slower (from E = 17 the window's ring is 12 chunks and the
// registers pass 240 VGPRs).
constexpr bool single_window(int E) { return E <= 10 || (E >= 13 && E <= 16); }

// Column sweep of group g (pairs 32g .. 32g+31); writes the group's results.
// ld(plane, c) returns the four words of chunk c of a plane (Q0, Q1, R0, R1)
// of this group.  Every chunk of every plane is loaded exactly once: one query
// window runs over the whole pair (chunks outside [0, nch) read as zero), and
// each chunk's columns run either plain or masked.  A chunk is masked when one
// of its rows meets a query index outside [0, m) (the first EC chunks and
// those from ct on); its cells outside [0, m) are cleared.  m is the same for
// every lane, so the choice, and each cell's validity, is uniform.
// The window is circular: slot = chunk mod W with the loop unrolled W chunks,
// so every register index is static and the window never moves.
template <int E, int MODE, bool SUB = false, class LD>
__device__ __forceinline__ void sweep_group(LD&& ld, int m, int64_t g, int64_t n_pairs,
                                            uint16_t* __restrict__ out, int sub_width = 0)
{
    // SUB: Snake-on-Chip's decomposition (Section 2.5): at every multiple of
    // sub_width the walk restarts from a new checkpoint, so each sub-maze of
    // sub_width columns is solved on its own and the counts add up
    int next_sub = SUB ? sub_width : 0x7FFFFFFF;
    constexpr int B = kChunk;
    constexpr int EC = (E + B - 1) / B;
    const int nch = (m + B - 1) / B;
    // chunks c in [EC, ct) never touch a query index outside [0, m)
    const int ct = (m - B - E >= 0) ? (m - B - E) / B + 1 : 0;
    auto put = [](uint32_t (&d)[B], const uint4& v) { d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w; };
    SweepState<E> st;
    st.init();

    // the four columns of chunk c0; w0(o), w1(o): query words at position 4 c0 + o
    auto run_chunk = [&](int c0, bool masked, const uint4& rr0, const uint4& rr1, auto&& w0, auto&& w1) {
        if (!masked) {
#pragma unroll
            for (int t = 0; t < B; t++) {
                if (SUB && B * c0 + t == next_sub) { st.restart(); next_sub += sub_width; }
                st.template column<false>(comp(rr0, t), comp(rr1, t), [&](int r) { return w0(t + r - E); },
                                          [&](int r) { return w1(t + r - E); }, [](int) { return ~0u; });
            }
        } else {
            // the validity of a cell depends only on its column and row (the same
            // for every lane), so it is a scalar condition
#pragma unroll
            for (int t = 0; t < B; t++) {
                const int j = B * c0 + t;
                if (j >= m) break;
                if (SUB && j == next_sub) { st.restart(); next_sub += sub_width; }
                st.template column<true>(comp(rr0, t), comp(rr1, t), [&](int r) { return w0(t + r - E); },
                                         [&](int r) { return w1(t + r - E); },
                                         [&](int r) { return (unsigned)(j + r - E) < (unsigned)m ? ~0u : 0u; });
            }
        }
    };

    static_assert(MODE == MAIN_CIRC, "one window: the circular form");
    // The loads run one chunk ahead of the columns.  Chunk c0's columns read
    // query chunks c0-EC .. c0+EC and reference chunk c0; before they start,
    // query chunk c0+EC+1 and reference chunk c0+1 are issued, so a wavefront
    // always has a chunk in flight while it computes (issued in the same step
    // and consumed at once, every chunk would wait out a full memory latency).
    // In the steady loop every step issues the same four loads with no
    // condition, so the compiler's wait for the data of chunk c0 counts
    // exactly the four younger loads instead of draining them all; the last
    // chunks, whose prefetches would fall past the end, run after it.
    // Slots of chunks outside [0, nch) are only ever read by masked columns,
    // which clear those cells: they start at zero and are not refilled.
    constexpr int W = 2 * EC + 2;               // even: chunk parity is static in the unrolled loops
    uint32_t q0w[W][B], q1w[W][B];              // slot (c mod W) holds query chunk c
    uint4 rf0[2], rf1[2];                       // reference chunk c in [c & 1]
#pragma unroll
    for (int i = 0; i < W; i++) {
#pragma unroll
        for (int e = 0; e < B; e++) { q0w[i][e] = 0u; q1w[i][e] = 0u; }
    }
    auto load_q = [&](int slot, int c) {
        put(q0w[slot], ld(0, c));
        put(q1w[slot], ld(1, c));
    };
#pragma unroll
    for (int c = 0; c <= EC; c++)
        if (c < nch) load_q(c % W, c);
    if (nch > 0) {                              // m = 0: nothing to read (the planes may be absent)
        rf0[0] = ld(2, 0);
        rf1[0] = ld(3, 0);
    }
    // chunk c0 at unrolled position u (c0 = u mod W)
    auto columns = [&](int c0, int u) {
        auto w0 = [&](int o) { const int d = floordiv(o, B); return q0w[(u + d + 2 * W) % W][o - d * B]; };
        auto w1 = [&](int o) { const int d = floordiv(o, B); return q1w[(u + d + 2 * W) % W][o - d * B]; };
        run_chunk(c0, !(c0 >= EC && c0 < ct), rf0[u & 1], rf1[u & 1], w0, w1);
    };
    const int nsteady = nch - EC - 1;           // chunks whose next query and reference chunks exist
    int cb = 0;
    for (; cb + W <= nsteady; cb += W) {
#pragma unroll
        for (int u = 0; u < W; u++) {
            const int c0 = cb + u;
            load_q((u + EC + 1) % W, c0 + EC + 1);
            rf0[(u + 1) & 1] = ld(2, c0 + 1);
            rf1[(u + 1) & 1] = ld(3, c0 + 1);
            columns(c0, u);
        }
    }
    // fewer than W + EC + 1 chunks remain
#pragma unroll
    for (int u = 0; u < W + EC + 1; u++) {
        const int c0 = cb + u;
        if (c0 < nch) {
            if (c0 + EC + 1 < nch) load_q((u + EC + 1) % W, c0 + EC + 1);
            if (c0 + 1 < nch) {
                rf0[(u + 1) & 1] = ld(2, c0 + 1);
                rf1[(u + 1) & 1] = ld(3, c0 + 1);
            }
            columns(c0, u);
        }
    }

    write_group<E>(st.T, g, n_pairs, out);
}

// The same sweep in three parts, for thresholds whose window is large: the
// chunks whose columns see a query index outside [0, m) (the first EC and the
// last few) run through a checked loop with a window of its own, reloading the
// few chunks it shares with the interior, where that register-lean form is
// faster than the single window above; interior chunks run unchecked, four
// per step (MAIN_SHIFT4: their loads issued together, the window shifting by
// four chunks).
template <int E, int MODE, bool SUB = false, class LD>
__device__ __forceinline__ void sweep_group_seams(LD&& ld, int m, int64_t g, int64_t n_pairs,
                                            uint16_t* __restrict__ out, int sub_width = 0)
{
    // SUB: Snake-on-Chip's decomposition (Section 2.5): at every multiple of
    // sub_width the walk restarts from a new checkpoint, so each sub-maze of
    // sub_width columns is solved on its own and the counts add up
    int next_sub = SUB ? sub_width : 0x7FFFFFFF;
    constexpr int B = kChunk;
    constexpr int EC = (E + B - 1) / B;
    constexpr int W = 2 * EC + 1;
    const int nch = (m + B - 1) / B;
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
                if (SUB && j == next_sub) { st.restart(); next_sub += sub_width; }
                st.template column<true>(comp(rr0, t), comp(rr1, t),
                          [&](int r) { const int o = t + r - E, d = floordiv(o, B); return w0[EC + d][o - d * B]; },
                          [&](int r) { const int o = t + r - E, d = floordiv(o, B); return w1[EC + d][o - d * B]; },
                          [&](int r) { return (unsigned)(j + r - E) < (unsigned)m ? ~0u : 0u; });
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
    auto always = [](int) { return ~0u; };
    if (ct > EC) {
        static_assert(MODE == MAIN_SHIFT4, "three parts: four chunks per step");
        {
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
                            if (SUB && B * (cb + u) + t == next_sub) { st.restart(); next_sub += sub_width; }
                            st.template column<false>(comp(rr0[u], t), comp(rr1[u], t),
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

    write_group<E>(st.T, g, n_pairs, out);
}

// The sweep kernel: one group per lane, one layout block per wavefront.  Every
// word is read once, so the loads are marked non-temporal (the measured read
// rate of this access pattern rises from 5.8 to 6.3 TB/s with the hint).
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
template <int E, int MODE, bool SUB>
__global__ __launch_bounds__(256) void k_sliced(const uint32_t* __restrict__ pk, int64_t G, int m,
                                                int64_t n_pairs, uint16_t* __restrict__ out, int sub_width)
{
    static_assert(kSlicedBlock == 64, "one layout block per wavefront");
    // the wavefront's layout block, in scalar registers (256 threads: four wavefronts per block)
    const int64_t gb = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int64_t g = gb * kSlicedBlock + lane;
    if (g >= G) return;
    const int nch = (m + kChunk - 1) / kChunk;
    const int64_t Gb = sliced_block_groups(gb * kSlicedBlock, G);
    const v4u* __restrict__ base =
        reinterpret_cast<const v4u*>(pk) + sliced_block_base(gb * kSlicedBlock, nch) + lane;
    auto ld = [&](int plane, int c) -> uint4 {
        const v4u x = __builtin_nontemporal_load(base + ((int64_t)plane * nch + c) * Gb);
        return make_uint4(x.x, x.y, x.z, x.w);
    };
    if constexpr (single_window(E))
        sweep_group<E, MODE, SUB>(ld, m, g, n_pairs, out, sub_width);
    else
        sweep_group_seams<E, MODE, SUB>(ld, m, g, n_pairs, out, sub_width);
}

template <int E>
hipError_t launch_sliced_E(const uint32_t* packed, int64_t n_pairs, int32_t m, int sub_width, uint16_t* out,
                           hipStream_t s)
{
    const int64_t G = cdiv(n_pairs, 32);
    const int threads = 256;
    const int64_t blocks = cdiv(G, threads);
    constexpr int mode = single_window(E) ? MAIN_CIRC : MAIN_SHIFT4;
    if (sub_width > 0 && sub_width < m)
        hipLaunchKernelGGL((k_sliced<E, mode, true>), dim3((unsigned)blocks), dim3(threads), 0, s, packed, G, m,
                           n_pairs, out, sub_width);
    else
        hipLaunchKernelGGL((k_sliced<E, mode, false>), dim3((unsigned)blocks), dim3(threads), 0, s, packed, G, m,
                           n_pairs, out, 0);
    return hipGetLastError();
}

template <int... Es>
struct SlicedTable {
    static hipError_t run(int E, const uint32_t* packed, int64_t n, int32_t m, int sub_width, uint16_t* out,
                          hipStream_t s)
    {
        hipError_t r = hipErrorInvalidValue;
        ((E == Es ? (r = launch_sliced_E<Es>(packed, n, m, sub_width, out, s), 0) : 0), ...);
        return r;
    }
};


}  // namespace sliced
}  // namespace ss
