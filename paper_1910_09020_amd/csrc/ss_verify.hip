// Verification step that a pre-alignment filter precedes: the exact edit
// distance (unit-cost Levenshtein distance) of the pairs the filter accepts,
// and the compaction of their indices.
//
// Edit distance by Myers' bit-vector algorithm (G. Myers, "A fast bit-vector
// algorithm for approximate string matching based on dynamic programming",
// J. ACM 46(3), 1999), in the form that computes the global distance D[m][n]:
// the vertical difference vectors Pv/Mv of one DP column are kept as bit masks
// over the query positions, and every reference character updates them with a
// handful of word operations; the horizontal difference entering the top row
// is +1 in every column (D[0][j] = j), and the score follows the bottom row.
// One pair per lane; W 32-bit words cover a query of up to 32 W positions,
// with the additions and shifts carried from word to word.
#include "ss_wave.h"

namespace ss {
namespace {

template <int W>
__global__ __launch_bounds__(256) void k_verify(const uint32_t* __restrict__ pk, int64_t SW,
                                                const int64_t* __restrict__ offsets,
                                                const int32_t* __restrict__ lengths,
                                                const int64_t* __restrict__ index, int64_t n,
                                                int32_t* __restrict__ ed_out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t p = index ? index[k] : k;
    const int m = lengths[p];
    const int64_t b0 = offsets[p];
    const uint32_t* __restrict__ Q0 = pk;
    const uint32_t* __restrict__ Q1 = pk + SW;
    const uint32_t* __restrict__ R0 = pk + 2 * SW;
    const uint32_t* __restrict__ R1 = pk + 3 * SW;

    // query planes of this pair, position i at bit i % 32 of word i / 32 (bits past m are never read
    // back: carries and shifts only move information upwards)
    uint32_t q0[W], q1[W], pv[W], mv[W];
#pragma unroll
    for (int w = 0; w < W; w++) {
        q0[w] = wave::bits32(Q0, SW, b0 + 32 * w);
        q1[w] = wave::bits32(Q1, SW, b0 + 32 * w);
        pv[w] = ~0u;
        mv[w] = 0u;
    }
    const int lw = (m - 1) >> 5, lb = (m - 1) & 31;     // word and bit of the last query position
    int score = m;
    for (int jb = 0; jb < m; jb += 32) {
        const uint32_t rw0 = wave::bits32(R0, SW, b0 + jb), rw1 = wave::bits32(R1, SW, b0 + jb);
        const int jend = m - jb < 32 ? m - jb : 32;
        for (int jj = 0; jj < jend; jj++) {
            // reference character j as two all-ones/all-zeros masks
            const uint32_t rb0 = (uint32_t)__builtin_amdgcn_sbfe((int)rw0, jj, 1);
            const uint32_t rb1 = (uint32_t)__builtin_amdgcn_sbfe((int)rw1, jj, 1);
            uint32_t carry = 0, ph_in = 1u, mh_in = 0u;
#pragma unroll
            for (int w = 0; w < W; w++) {
                // Eq: query positions equal to the reference character
                const uint32_t eq = wave::and_xnor(wave::and_xnor(~0u, q0[w], rb0), q1[w], rb1);
                const uint32_t xv = eq | mv[w];
                const uint64_t s = (uint64_t)(eq & pv[w]) + pv[w] + carry;
                carry = (uint32_t)(s >> 32);
                const uint32_t xh = ((uint32_t)s ^ pv[w]) | eq;
                const uint32_t ph = mv[w] | ~(xh | pv[w]);
                const uint32_t mh = pv[w] & xh;
                if (w == lw) score += (int)((ph >> lb) & 1u) - (int)((mh >> lb) & 1u);
                const uint32_t phs = (ph << 1) | ph_in, mhs = (mh << 1) | mh_in;
                ph_in = ph >> 31;
                mh_in = mh >> 31;
                pv[w] = mhs | ~(xv | phs);
                mv[w] = phs & xv;
            }
        }
    }
    ed_out[k] = score;
}

__global__ void k_zero_count(unsigned long long* count) { *count = 0ull; }

// Indices of accepted pairs (result bit 15 set).  A block takes 4096 results
// (16 per thread, in order), counts them with wavefront ballots and one LDS
// scan over its four waves, takes its output range with a single atomic and
// writes the indices in order; the blocks' ranges come in arrival order.
constexpr int kSelPer = 16;
__global__ __launch_bounds__(256) void k_select(const uint16_t* __restrict__ res, int64_t n,
                                                int64_t* __restrict__ idx, unsigned long long* __restrict__ count)
{
    __shared__ unsigned long long s_base;
    __shared__ int s_wave[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + t) * kSelPer;
    uint32_t bits = 0;
#pragma unroll
    for (int e = 0; e < kSelPer; e++) {
        const int64_t i = i0 + e;
        if (i < n && (res[i] & 0x8000u)) bits |= 1u << e;
    }
    const int mine = __popc(bits);
    // inclusive scan of mine over the wavefront
    int x = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wv] = x;
    __syncthreads();
    if (t == 0) {
        const int tot = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
        s_base = tot ? atomicAdd(count, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    int before = x - mine;
    for (int w = 0; w < wv; w++) before += s_wave[w];
    unsigned long long o = s_base + (unsigned long long)before;
    while (bits) {
        const int e = __builtin_ctz(bits);
        bits &= bits - 1u;
        idx[o++] = i0 + e;
    }
}

}  // namespace

template <int W>
static void launch_verify_W(dim3 grid, hipStream_t s, const uint32_t* packed, int64_t SW, const int64_t* offsets,
                            const int32_t* lengths, const int64_t* index, int64_t n, int32_t* ed_out)
{
    hipLaunchKernelGGL(k_verify<W>, grid, dim3(256), 0, s, packed, SW, offsets, lengths, index, n, ed_out);
}

hipError_t launch_verify(const uint32_t* packed, int64_t stream_words, const int64_t* offsets, const int32_t* lengths,
                         const int64_t* index, int64_t n, int32_t max_len, int32_t* ed_out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)cdiv(n, 256));
    if (max_len <= 32) launch_verify_W<1>(grid, s, packed, stream_words, offsets, lengths, index, n, ed_out);
    else if (max_len <= 64) launch_verify_W<2>(grid, s, packed, stream_words, offsets, lengths, index, n, ed_out);
    else if (max_len <= 128) launch_verify_W<4>(grid, s, packed, stream_words, offsets, lengths, index, n, ed_out);
    else launch_verify_W<8>(grid, s, packed, stream_words, offsets, lengths, index, n, ed_out);
    return hipGetLastError();
}

hipError_t launch_select(const uint16_t* results, int64_t n, int64_t* index_out, unsigned long long* count,
                         hipStream_t s)
{
    // the counter is cleared by a kernel (no memset node if the caller captures the stream)
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, count);
    if (n > 0)
        hipLaunchKernelGGL(k_select, dim3((unsigned)cdiv(n, 256 * kSelPer)), dim3(256), 0, s, results, n, index_out,
                           count);
    return hipGetLastError();
}

}  // namespace ss
