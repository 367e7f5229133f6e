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
// Up to 256 positions: one pair per lane; W 32-bit words cover a query of up
// to 32 W positions, with the additions and shifts carried from word to word.
// Longer pairs: one pair per wavefront, lane L holding query positions
// [32 W L, 32 W (L + 1)); the carries of the addition cross lanes through one
// carry-lookahead step over the wavefront (each lane's segment either
// generates a carry, propagates one, or neither: with G and P those lanes' bit
// masks, the lanes that receive a carry are (G + (G | P)) ^ P), and the
// one-position shifts cross lanes through a shuffle.
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

// One pair per wavefront (four per block), query positions [32 W L, 32 W (L + 1))
// on lane L: pairs of up to 2048 W positions.
template <int W>
__global__ __launch_bounds__(256) void k_verify_wave(const uint32_t* __restrict__ pk, int64_t SW,
                                                     const int64_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ lengths,
                                                     const int64_t* __restrict__ index, int64_t n,
                                                     int32_t* __restrict__ ed_out)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t k = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (k >= n) return;                                  // the whole wavefront
    const int64_t p = index ? index[k] : k;
    const int m = __builtin_amdgcn_readfirstlane(lengths[p]);
    const int64_t b0 = offsets[p];
    const uint32_t* __restrict__ Q0 = pk;
    const uint32_t* __restrict__ Q1 = pk + SW;
    const uint32_t* __restrict__ R0 = pk + 2 * SW;
    const uint32_t* __restrict__ R1 = pk + 3 * SW;
    if (m == 0 || m > 2048 * W) {
        // (a pair longer than the caller's max_len is reported as -1)
        if (lane == 0) ed_out[k] = m == 0 ? 0 : -1;
        return;
    }
    // this lane's query positions (positions at or past m read as any value: carries and shifts
    // only move information upwards, and the score is read at position m - 1)
    uint32_t q0[W], q1[W], pv[W], mv[W];
#pragma unroll
    for (int w = 0; w < W; w++) {
        const int64_t at = b0 + 32 * ((int64_t)W * lane + w);
        q0[w] = wave::bits32(Q0, SW, at);
        q1[w] = wave::bits32(Q1, SW, at);
        pv[w] = ~0u;
        mv[w] = 0u;
    }
    const int last = m - 1;
    const int l_lane = last / (32 * W), l_word = (last >> 5) % W, l_bit = last & 31;
    int score = m;
    for (int jb = 0; jb < m; jb += 32) {
        const uint32_t rw0 = __builtin_amdgcn_readfirstlane(wave::bits32(R0, SW, b0 + jb));
        const uint32_t rw1 = __builtin_amdgcn_readfirstlane(wave::bits32(R1, SW, b0 + jb));
        const int jend = m - jb < 32 ? m - jb : 32;
        for (int jj = 0; jj < jend; jj++) {
            const uint32_t rb0 = (uint32_t)__builtin_amdgcn_sbfe((int)rw0, jj, 1);
            const uint32_t rb1 = (uint32_t)__builtin_amdgcn_sbfe((int)rw1, jj, 1);
            // (Eq & Pv) + Pv over this lane's segment with no carry in
            uint32_t eq[W], sum[W], carry = 0, ones = ~0u;
#pragma unroll
            for (int w = 0; w < W; w++) {
                eq[w] = wave::and_xnor(wave::and_xnor(~0u, q0[w], rb0), q1[w], rb1);
                const uint64_t s = (uint64_t)(eq[w] & pv[w]) + pv[w] + carry;
                sum[w] = (uint32_t)s;
                carry = (uint32_t)(s >> 32);
                ones &= sum[w];
            }
            // carry lookahead over the lanes (a segment that generates cannot also be all ones)
            const uint64_t G = __ballot(carry != 0u);
            const uint64_t P = __ballot(ones == ~0u);
            uint32_t cin = (uint32_t)((((G + (G | P)) ^ P) >> lane) & 1ull);
            // the pass with the carry in, then the rest of the column step
            uint32_t ph[W], mh[W];
#pragma unroll
            for (int w = 0; w < W; w++) {
                const uint32_t sw = sum[w] + cin;
                cin = sw < cin ? 1u : 0u;
                const uint32_t xh = (sw ^ pv[w]) | eq[w];
                ph[w] = mv[w] | ~(xh | pv[w]);
                mh[w] = pv[w] & xh;
            }
            // the bottom row's horizontal difference
            uint32_t dp = 0, dm = 0;
#pragma unroll
            for (int w = 0; w < W; w++) {
                if (w == l_word) {
                    dp = (ph[w] >> l_bit) & 1u;
                    dm = (mh[w] >> l_bit) & 1u;
                }
            }
            score += (int)__builtin_amdgcn_readlane(dp, l_lane) - (int)__builtin_amdgcn_readlane(dm, l_lane);
            // shift up by one position: lane 0 takes +1 (D[0][j] = j) and 0; others the previous lane's top bits
            const uint32_t ph_top = __shfl_up(ph[W - 1] >> 31, 1), mh_top = __shfl_up(mh[W - 1] >> 31, 1);
            uint32_t ph_in = lane == 0 ? 1u : ph_top, mh_in = lane == 0 ? 0u : mh_top;
#pragma unroll
            for (int w = 0; w < W; w++) {
                const uint32_t xv = eq[w] | mv[w];
                const uint32_t phs = (ph[w] << 1) | ph_in, mhs = (mh[w] << 1) | mh_in;
                ph_in = ph[w] >> 31;
                mh_in = mh[w] >> 31;
                pv[w] = mhs | ~(xv | phs);
                mv[w] = phs & xv;
            }
        }
    }
    if (lane == 0) ed_out[k] = score;
}

// Banded form, one pair per wavefront: the edit distance when it is at most the
// pair's threshold Ep, else Ep + 1, in time proportional to m * Ep instead of
// m * m.  The wavefront holds a window of 32-position words of the query (lane
// L: words W L .. W L + W - 1), bottom position lo.  Every 32 columns, when the
// window's bottom word lies wholly below the band |i - j| <= Ep for the coming
// columns, it is dropped: its vertical deltas are added to the value B of the
// row under the window, the other words move down one word, and a new word
// enters at the top with vertical deltas +1.  Within a column, the row under
// the window is taken to grow by 1 (its horizontal delta is +1, entered as the
// bottom shift-in as for row 0 of the full form).  Every value so assumed is at
// least the true one (a row never exceeds the row below it plus one, nor its
// left neighbour plus one), so computed values are never below the true ones,
// and every cell on an optimal path of cost <= Ep (which stays within Ep / 2 of
// the diagonal) is computed from exact neighbours: D[m][m] is exact when it is
// <= Ep.  At the end D[m][m] = B + the vertical deltas of the window's rows up
// to m.  The window needs 2048 W >= 2 Ep + 65 positions.
template <int W>
__global__ __launch_bounds__(256) void k_verify_band(const uint32_t* __restrict__ pk, int64_t SW,
                                                     const int64_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ lengths,
                                                     const int32_t* __restrict__ Epp, int32_t E,
                                                     const int64_t* __restrict__ index, int64_t n,
                                                     int32_t* __restrict__ ed_out)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t k = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (k >= n) return;                                  // the whole wavefront
    const int64_t p = index ? index[k] : k;
    const int m = __builtin_amdgcn_readfirstlane(lengths[p]);
    const int Ep = __builtin_amdgcn_readfirstlane(Epp ? Epp[p] : E);
    const int64_t b0 = offsets[p];
    const uint32_t* __restrict__ Q0 = pk;
    const uint32_t* __restrict__ Q1 = pk + SW;
    const uint32_t* __restrict__ R0 = pk + 2 * SW;
    const uint32_t* __restrict__ R1 = pk + 3 * SW;
    if (2 * (int64_t)Ep + 65 > 2048 * W) {
        if (lane == 0) ed_out[k] = -1;                   // the window cannot hold this threshold's band
        return;
    }
    uint32_t q0[W], q1[W], pv[W], mv[W];
    int lo = 0;                                          // query position of the window's bottom row
    auto load_query = [&]() {
#pragma unroll
        for (int w = 0; w < W; w++) {
            const int64_t at = b0 + lo + 32 * ((int64_t)W * lane + w);
            q0[w] = wave::bits32(Q0, SW, at);
            q1[w] = wave::bits32(Q1, SW, at);
        }
    };
    load_query();
#pragma unroll
    for (int w = 0; w < W; w++) {
        pv[w] = ~0u;
        mv[w] = 0u;
    }
    int B = 0;                                           // D of the row under the window, this column
    for (int jb = 0; jb < m; jb += 32) {
        if (lo + 32 <= jb - Ep) {
            // drop the bottom word (lane 0, word 0): its rows' vertical deltas go into B
            B += __builtin_amdgcn_readlane(__popc(pv[0]) - __popc(mv[0]), 0);
            const uint32_t pn = __shfl_down(pv[0], 1), mn = __shfl_down(mv[0], 1);
#pragma unroll
            for (int w = 0; w + 1 < W; w++) {
                pv[w] = pv[w + 1];
                mv[w] = mv[w + 1];
            }
            pv[W - 1] = lane == 63 ? ~0u : pn;
            mv[W - 1] = lane == 63 ? 0u : mn;
            lo += 32;
            load_query();
        }
        const uint32_t rw0 = __builtin_amdgcn_readfirstlane(wave::bits32(R0, SW, b0 + jb));
        const uint32_t rw1 = __builtin_amdgcn_readfirstlane(wave::bits32(R1, SW, b0 + jb));
        const int jend = m - jb < 32 ? m - jb : 32;
        for (int jj = 0; jj < jend; jj++) {
            const uint32_t rb0 = (uint32_t)__builtin_amdgcn_sbfe((int)rw0, jj, 1);
            const uint32_t rb1 = (uint32_t)__builtin_amdgcn_sbfe((int)rw1, jj, 1);
            uint32_t eq[W], sum[W], carry = 0, ones = ~0u;
#pragma unroll
            for (int w = 0; w < W; w++) {
                eq[w] = wave::and_xnor(wave::and_xnor(~0u, q0[w], rb0), q1[w], rb1);
                const uint64_t s = (uint64_t)(eq[w] & pv[w]) + pv[w] + carry;
                sum[w] = (uint32_t)s;
                carry = (uint32_t)(s >> 32);
                ones &= sum[w];
            }
            const uint64_t G = __ballot(carry != 0u);
            const uint64_t P = __ballot(ones == ~0u);
            uint32_t cin = (uint32_t)((((G + (G | P)) ^ P) >> lane) & 1ull);
            uint32_t ph[W], mh[W];
#pragma unroll
            for (int w = 0; w < W; w++) {
                const uint32_t sw = sum[w] + cin;
                cin = sw < cin ? 1u : 0u;
                const uint32_t xh = (sw ^ pv[w]) | eq[w];
                ph[w] = mv[w] | ~(xh | pv[w]);
                mh[w] = pv[w] & xh;
            }
            const uint32_t ph_top = __shfl_up(ph[W - 1] >> 31, 1), mh_top = __shfl_up(mh[W - 1] >> 31, 1);
            uint32_t ph_in = lane == 0 ? 1u : ph_top, mh_in = lane == 0 ? 0u : mh_top;
#pragma unroll
            for (int w = 0; w < W; w++) {
                const uint32_t xv = eq[w] | mv[w];
                const uint32_t phs = (ph[w] << 1) | ph_in, mhs = (mh[w] << 1) | mh_in;
                ph_in = ph[w] >> 31;
                mh_in = mh[w] >> 31;
                pv[w] = mhs | ~(xv | phs);
                mv[w] = phs & xv;
            }
            B += 1;
        }
    }
    // D[m][m]: B plus the vertical deltas of the window's rows below position m
    int part = 0;
#pragma unroll
    for (int w = 0; w < W; w++) {
        const int first = lo + 32 * (W * lane + w);
        const int keep = m - first;                      // positions of this word below m
        const uint32_t mask = keep >= 32 ? ~0u : (keep <= 0 ? 0u : ((1u << keep) - 1u));
        part += __popc(pv[w] & mask) - __popc(mv[w] & mask);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o);
    const int D = B + part;
    if (lane == 0) ed_out[k] = D <= Ep ? D : Ep + 1;
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

template <int W>
static void launch_verify_wave_W(hipStream_t s, const uint32_t* packed, int64_t SW, const int64_t* offsets,
                                 const int32_t* lengths, const int64_t* index, int64_t n, int32_t* ed_out)
{
    hipLaunchKernelGGL(k_verify_wave<W>, dim3((unsigned)cdiv(n, 4)), dim3(256), 0, s, packed, SW, offsets, lengths,
                       index, n, ed_out);
}

hipError_t launch_verify(const uint32_t* packed, int64_t stream_words, const int64_t* offsets, const int32_t* lengths,
                         const int64_t* index, int64_t n, int32_t max_len, int32_t* ed_out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)cdiv(n, 256));
    if (max_len > 256) {
        // one pair per wavefront: 2048 positions per word of each lane
        const int64_t SW = stream_words;
        if (max_len <= 2048) launch_verify_wave_W<1>(s, packed, SW, offsets, lengths, index, n, ed_out);
        else if (max_len <= 4096) launch_verify_wave_W<2>(s, packed, SW, offsets, lengths, index, n, ed_out);
        else if (max_len <= 8192) launch_verify_wave_W<4>(s, packed, SW, offsets, lengths, index, n, ed_out);
        else if (max_len <= 16384) launch_verify_wave_W<8>(s, packed, SW, offsets, lengths, index, n, ed_out);
        else if (max_len <= 32768) launch_verify_wave_W<16>(s, packed, SW, offsets, lengths, index, n, ed_out);
        else launch_verify_wave_W<32>(s, packed, SW, offsets, lengths, index, n, ed_out);
        return hipGetLastError();
    }
    if (max_len <= 32) launch_verify_W<1>(grid, s, packed, stream_words, offsets, lengths, index, n, ed_out);
    else if (max_len <= 64) launch_verify_W<2>(grid, s, packed, stream_words, offsets, lengths, index, n, ed_out);
    else if (max_len <= 128) launch_verify_W<4>(grid, s, packed, stream_words, offsets, lengths, index, n, ed_out);
    else launch_verify_W<8>(grid, s, packed, stream_words, offsets, lengths, index, n, ed_out);
    return hipGetLastError();
}

template <int W>
static void launch_band_W(hipStream_t s, const uint32_t* packed, int64_t SW, const int64_t* offsets,
                          const int32_t* lengths, const int32_t* Epp, int32_t E, const int64_t* index, int64_t n,
                          int32_t* ed_out)
{
    hipLaunchKernelGGL(k_verify_band<W>, dim3((unsigned)cdiv(n, 4)), dim3(256), 0, s, packed, SW, offsets, lengths,
                       Epp, E, index, n, ed_out);
}

hipError_t launch_verify_banded(const uint32_t* packed, int64_t stream_words, const int64_t* offsets,
                                const int32_t* lengths, const int32_t* Epp, int32_t E, const int64_t* index,
                                int64_t n, int32_t* ed_out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t need = 2 * (int64_t)E + 65;             // window positions for the largest threshold
    const int64_t SW = stream_words;
    if (need <= 2048) launch_band_W<1>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
    else if (need <= 2 * 2048) launch_band_W<2>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
    else if (need <= 3 * 2048) launch_band_W<3>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
    else if (need <= 4 * 2048) launch_band_W<4>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
    else if (need <= 5 * 2048) launch_band_W<5>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
    else if (need <= 6 * 2048) launch_band_W<6>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
    else if (need <= 8 * 2048) launch_band_W<8>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
    else if (need <= 12 * 2048) launch_band_W<12>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
    else launch_band_W<16>(s, packed, SW, offsets, lengths, Epp, E, index, n, ed_out);
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
