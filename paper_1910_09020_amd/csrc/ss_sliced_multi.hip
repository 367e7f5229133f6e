// Several thresholds in one pass over the lane-sliced planes.
//
// The walk of Section 2.4 at threshold E uses the 2E+1 rows of offsets -E..E;
// its checkpoints depend on E, so every threshold keeps its own row states and
// count (one SweepState each), but all of them read the same loaded words: the
// query window of the largest threshold covers every smaller one's offsets.  A
// chunk runs unmasked only when the largest threshold's rows all stay inside
// [0, m), which holds for every smaller one as well; in a masked chunk each
// state masks its own rows.  The planes are read once per pass instead of once
// per threshold, and the VALU work is the sum of the thresholds' own.
#include "ss_sliced_kernel.h"

namespace ss {
namespace sliced {

// One SweepState per threshold Es... (ascending); results of the k-th go to
// out + k * out_stride.
template <int... Es>
struct MultiState;

template <>
struct MultiState<> {
    __device__ __forceinline__ void init() {}
    template <bool MASKED, class W0, class W1>
    __device__ __forceinline__ void column(uint32_t, uint32_t, const W0&, const W1&, int, int, int)
    {
    }
    __device__ __forceinline__ void write(int64_t, int64_t, uint16_t* __restrict__, int64_t) {}
};

template <int E, int... Rest>
struct MultiState<E, Rest...> {
    SweepState<E> st;
    MultiState<Rest...> rest;

    __device__ __forceinline__ void init()
    {
        st.init();
        rest.init();
    }
    // column t of the chunk (position j); w0(o), w1(o): query words at offset o from the chunk start
    template <bool MASKED, class W0, class W1>
    __device__ __forceinline__ void column(uint32_t r0, uint32_t r1, const W0& w0, const W1& w1, int t, int j,
                                           int m)
    {
        st.template column<MASKED>(r0, r1, [&](int r) { return w0(t + r - E); },
                                   [&](int r) { return w1(t + r - E); },
                                   [&](int r) { return (unsigned)(j + r - E) < (unsigned)m ? ~0u : 0u; });
        rest.template column<MASKED>(r0, r1, w0, w1, t, j, m);
    }
    __device__ __forceinline__ void write(int64_t g, int64_t n_pairs, uint16_t* __restrict__ out, int64_t stride)
    {
        write_group<E>(st.T, g, n_pairs, out);
        rest.write(g, n_pairs, out + stride, stride);
    }
};

template <int... Es>
constexpr int max_of()
{
    int r = 0;
    ((r = Es > r ? Es : r), ...);
    return r;
}

// The single-window sweep of sweep_group with one state per threshold.
template <int... Es, class LD>
__device__ __forceinline__ void sweep_group_multi(LD&& ld, int m, int64_t g, int64_t n_pairs,
                                                  uint16_t* __restrict__ out, int64_t out_stride)
{
    constexpr int EM = max_of<Es...>();
    constexpr int B = kChunk;
    constexpr int EC = (EM + B - 1) / B;
    const int nch = (m + B - 1) / B;
    const int ct = (m - B - EM >= 0) ? (m - B - EM) / B + 1 : 0;   // chunks [EC, ct) stay inside [0, m)
    auto put = [](uint32_t (&d)[B], const uint4& v) { d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w; };
    MultiState<Es...> st;
    st.init();

    auto run_chunk = [&](int c0, bool masked, const uint4& rr0, const uint4& rr1, auto&& w0, auto&& w1) {
        if (!masked) {
#pragma unroll
            for (int t = 0; t < B; t++) st.template column<false>(comp(rr0, t), comp(rr1, t), w0, w1, t, 0, m);
        } else {
#pragma unroll
            for (int t = 0; t < B; t++) {
                const int j = B * c0 + t;
                if (j >= m) break;
                st.template column<true>(comp(rr0, t), comp(rr1, t), w0, w1, t, j, m);
            }
        }
    };

    // the window and the loads run exactly as in sweep_group (one chunk ahead, a steady loop with no
    // condition on its loads, then the remainder)
    constexpr int W = 2 * EC + 2;
    uint32_t q0w[W][B], q1w[W][B];
    uint4 rf0[2], rf1[2];
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
    if (nch > 0) {
        rf0[0] = ld(2, 0);
        rf1[0] = ld(3, 0);
    }
    auto columns = [&](int c0, int u) {
        auto w0 = [&](int o) { const int d = floordiv(o, B); return q0w[(u + d + 2 * W) % W][o - d * B]; };
        auto w1 = [&](int o) { const int d = floordiv(o, B); return q1w[(u + d + 2 * W) % W][o - d * B]; };
        run_chunk(c0, !(c0 >= EC && c0 < ct), rf0[u & 1], rf1[u & 1], w0, w1);
    };
    const int nsteady = nch - EC - 1;
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
    st.write(g, n_pairs, out, out_stride);
}

template <int... Es>
__global__ __launch_bounds__(256) void k_sliced_multi(const uint32_t* __restrict__ pk, int64_t G, int m,
                                                      int64_t n_pairs, uint16_t* __restrict__ out,
                                                      int64_t out_stride)
{
    static_assert(kSlicedBlock == 64, "one layout block per wavefront");
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
    sweep_group_multi<Es...>(ld, m, g, n_pairs, out, out_stride);
}

template <int... Es>
hipError_t launch_multi(const uint32_t* packed, int64_t n_pairs, int32_t m, uint16_t* out, int64_t out_stride,
                        hipStream_t s)
{
    const int64_t G = cdiv(n_pairs, 32);
    const int64_t blocks = cdiv(G, 256);
    hipLaunchKernelGGL((k_sliced_multi<Es...>), dim3((unsigned)blocks), dim3(256), 0, s, packed, G, m, n_pairs, out,
                       out_stride);
    return hipGetLastError();
}

}  // namespace sliced

// Thresholds that share a pass: runs of consecutive thresholds whose states and window fit the
// registers of one kernel at three or two wavefronts per SIMD.  Measured on 30 M x 100 bp against
// one pass per threshold: E = 0..4 (150 VGPRs) 0.42 ms against 1.37 ms, E = 5..7 (220 VGPRs)
// 0.47 ms against 0.84 ms; E = 8, 9 together (253 VGPRs) took 0.75 ms against 0.58 ms, so from
// E = 8 every threshold takes its own pass.  sliced_multi_span(E): how many thresholds from E one
// pass takes (0: none starts at E).
int sliced_multi_span(int E_first)
{
    return E_first == 0 ? 5 : E_first == 5 ? 3 : 0;
}

hipError_t launch_sliced_multi_group(int E_first, const uint32_t* packed, int64_t n_pairs, int32_t m, uint16_t* out,
                                     int64_t out_stride, hipStream_t s)
{
    if (n_pairs == 0) return hipSuccess;
    switch (E_first) {
    case 0: return sliced::launch_multi<0, 1, 2, 3, 4>(packed, n_pairs, m, out, out_stride, s);
    case 5: return sliced::launch_multi<5, 6, 7>(packed, n_pairs, m, out, out_stride, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ss
