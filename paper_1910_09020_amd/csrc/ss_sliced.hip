// Lane-sliced encoder and the threshold dispatch of the column-sweep kernel.
//
// Layout: bit s of every 32-bit word belongs to pair 32*g + s ("group" g, one
// group per lane of the sweep kernel).  The encoder transposes 32 pairs at a
// time with wavefront ballots: one ballot per (plane, position) gives the word
// of 32 pairs for each half of the wavefront.
#include "ss_common.h"

namespace ss {
namespace {

__device__ __forceinline__ uint32_t base_code(uint32_t b) { return ((b >> 1) ^ (b >> 2)) & 3u; }

// 1 when b is one of A C G T a c g t
__device__ __forceinline__ uint32_t base_ok(uint32_t b)
{
    const uint32_t v = (b | 0x20u) - 0x61u;          // 'a' -> 0, 'c' -> 2, 'g' -> 6, 't' -> 19
    return (v < 20u) ? ((0x80045u >> v) & 1u) : 0u;
}

// ---------------------------------------------------------------- encoder
// One 64-lane block per group; lanes 0..31 handle chunk c, lanes 32..63 chunk
// c+1 of the same 32 pairs.  Each ballot transposes one base position of 32
// pairs (per plane) into one word per half-wave.
__global__ __launch_bounds__(64) void k_pack_sliced(const uint8_t* __restrict__ reads,
                                                    const uint8_t* __restrict__ refs,
                                                    const int64_t* __restrict__ offsets,
                                                    const int64_t* __restrict__ index, int64_t n_pairs,
                                                    int m, int64_t G, uint32_t* __restrict__ packed,
                                                    uint32_t* __restrict__ err)
{
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int s = lane & 31, h = lane >> 5;
    const int64_t slot = g * 32 + s;
    const bool have = slot < n_pairs;
    int64_t off = 0;
    if (have) {
        const int64_t pi = index ? index[slot] : slot;
        off = offsets ? offsets[pi] : pi * (int64_t)m;
    }
    const int nch = (m + kChunk - 1) / kChunk;
    uint32_t bad = 0;
    uint4* out4 = reinterpret_cast<uint4*>(packed);
    for (int c2 = 0; c2 < nch; c2 += 2) {
        const int c = c2 + h;
        uint64_t bq0[kChunk], bq1[kChunk], br0[kChunk], br1[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; t++) {
            const int j = kChunk * c + t;
            uint32_t qb = 'A', rb = 'A';
            if (have && j < m) {
                qb = reads[off + j];
                rb = refs[off + j];
                bad |= (base_ok(qb) & base_ok(rb)) ^ 1u;
            }
            const uint32_t qc = base_code(qb), rc = base_code(rb);
            bq0[t] = __ballot(qc & 1u);
            bq1[t] = __ballot(qc >> 1);
            br0[t] = __ballot(rc & 1u);
            br1[t] = __ballot(rc >> 1);
        }
        if (lane < 8) {
            const int p = lane & 3, hh = lane >> 2;
            const int cc = c2 + hh;
            if (cc < nch) {
                uint32_t w[kChunk];
#pragma unroll
                for (int t = 0; t < kChunk; t++) {
                    const uint64_t b = p == 0 ? bq0[t] : (p == 1 ? bq1[t] : (p == 2 ? br0[t] : br1[t]));
                    w[t] = (uint32_t)(b >> (32 * hh));
                }
                out4[((int64_t)p * nch + cc) * G + g] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    if (bad && err) atomicOr(err, 1u);
}

}  // namespace

hipError_t launch_sliced_lo(int E, const uint32_t* packed, int64_t n, int32_t m, uint16_t* out, hipStream_t s);
hipError_t launch_sliced_mid(int E, const uint32_t* packed, int64_t n, int32_t m, uint16_t* out, hipStream_t s);
hipError_t launch_sliced_hi(int E, const uint32_t* packed, int64_t n, int32_t m, uint16_t* out, hipStream_t s);

hipError_t launch_pack_sliced(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets,
                              const int64_t* index, int64_t n_pairs, int32_t m, uint32_t* packed,
                              uint32_t* err, hipStream_t s)
{
    const int64_t G = cdiv(n_pairs, 32);
    if (G == 0 || m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_sliced, dim3((unsigned)G), dim3(64), 0, s, reads, refs, offsets, index, n_pairs, m,
                       G, packed, err);
    return hipGetLastError();
}

hipError_t launch_sliced(const uint32_t* packed, int64_t n_pairs, int32_t m, int32_t E, uint16_t* out,
                         hipStream_t s)
{
    if (n_pairs == 0) return hipSuccess;
    if (E < 0 || E > kMaxESliced) return hipErrorInvalidValue;
    if (E <= 10) return launch_sliced_lo(E, packed, n_pairs, m, out, s);
    if (E <= 20) return launch_sliced_mid(E, packed, n_pairs, m, out, s);
    return launch_sliced_hi(E, packed, n_pairs, m, out, s);
}

}  // namespace ss
