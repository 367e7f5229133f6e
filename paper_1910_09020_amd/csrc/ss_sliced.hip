// Lane-sliced encoder and the threshold dispatch of the column-sweep kernel.
//
// Layout: bit s of every 32-bit word belongs to pair 32*g + s ("group" g, one
// group per lane of the sweep kernel).  The encoder transposes 32 pairs at a
// time with wavefront ballots: one ballot per (plane, position) gives the word
// of 32 pairs for each half of the wavefront.
#include <algorithm>

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

// ---------------------------------------------------------------- tiled encoder
// One 256-thread block encodes GB consecutive groups (32*GB pair slots).
// Phase 1 copies the slots' bases into LDS as 2-bit codes (one byte per base,
// rows padded to whole dwords, one pad dword per group so that the phase-2
// reads of different groups fall in different banks) and validates every
// byte: a byte b is one of ACGTacgt exactly when (b & 0xDF) equals the letter
// its code stands for, looked up with a byte permute.  Phase 2: one thread per
// (group, chunk of four positions) folds the 32 slots' code dwords into the
// four words of each plane.
__device__ __forceinline__ uint32_t codes4(uint32_t x, uint32_t& bad)
{
    const uint32_t cc = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
    const uint32_t letter = __builtin_amdgcn_perm(0u, 0x54474341u, cc);   // 'A','C','G','T' by code
    bad |= (x & 0xDFDFDFDFu) ^ letter;
    return cc;
}

__global__ __launch_bounds__(256) void k_pack_tile(const uint8_t* __restrict__ reads,
                                                   const uint8_t* __restrict__ refs,
                                                   const int64_t* __restrict__ offsets,
                                                   const int64_t* __restrict__ index, int64_t n_pairs, int m,
                                                   int64_t G, int GB, int fast, uint32_t* __restrict__ packed,
                                                   uint32_t* __restrict__ err)
{
    extern __shared__ uint32_t lds[];
    const int mw = (m + 3) >> 2;              // dwords per slot row
    const int gs = 32 * mw + 1;               // dwords per group
    const int nch = mw;
    const int64_t g0 = (int64_t)blockIdx.x * GB;
    const int64_t s0 = g0 * 32;
    const int np = (int)min((int64_t)32 * GB, n_pairs - s0);
    const int t = threadIdx.x;
    uint32_t bad = 0;
    uint4* __restrict__ out4 = reinterpret_cast<uint4*>(packed);
    // fast path: slots s0.. are pairs s0.. stored back to back, m % 4 == 0, the
    // block's first byte is 16-byte aligned and the block holds at most
    // 256 * kQ 16-byte loads per side.  Every load of both sides is issued
    // before any is consumed, to keep enough bytes in flight.
    constexpr int kQ = 8;
    const int ndw = np * mw;
    const int nq = ndw >> 2;
    // dw / mw by multiply-high, exact for dw < 2^16 and 2 <= mw < 2^16 (the
    // reciprocal of mw = 1 does not fit 32 bits: that case divides by itself)
    const uint32_t rmw = mw > 1 ? 0xFFFFFFFFu / (uint32_t)mw + 1u : 0u;
    auto row_of = [&](int dw) { return mw > 1 ? (int)__umulhi((uint32_t)dw, rmw) : dw; };
    uint4 v[2][kQ];
    if (fast) {
#pragma unroll
        for (int sd = 0; sd < 2; sd++) {
            const uint4* __restrict__ s128 = reinterpret_cast<const uint4*>((sd ? refs : reads) + s0 * (int64_t)m);
#pragma unroll
            for (int k = 0; k < kQ; k++) {
                const int q = t + 256 * k;
                if (q < nq) v[sd][k] = s128[q];
            }
        }
    }
#pragma unroll
    for (int side = 0; side < 2; side++) {
        const uint8_t* __restrict__ src = side ? refs : reads;
        if (fast) {
#pragma unroll
            for (int k = 0; k < kQ; k++) {
                const int q = t + 256 * k;
                if (q < nq) {
                    const uint32_t d[4] = {v[side][k].x, v[side][k].y, v[side][k].z, v[side][k].w};
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const int dw = 4 * q + e;
                        const int p = row_of(dw), col = dw - p * mw;
                        lds[(p >> 5) * gs + (p & 31) * mw + col] = codes4(d[e], bad);
                    }
                }
            }
            const uint32_t* __restrict__ s32 = reinterpret_cast<const uint32_t*>(src + s0 * (int64_t)m);
            for (int dw = 4 * nq + t; dw < ndw; dw += 256) {
                const int p = row_of(dw), col = dw - p * mw;
                lds[(p >> 5) * gs + (p & 31) * mw + col] = codes4(s32[dw], bad);
            }
        } else {
            uint8_t* lb = reinterpret_cast<uint8_t*>(lds);
            const int nb = np * m;
            for (int i = t; i < nb; i += 256) {
                const int p = i / m, col = i - p * m;
                const int64_t slot = s0 + p;
                const int64_t pi = index ? index[slot] : slot;
                const int64_t off = offsets ? offsets[pi] : pi * (int64_t)m;
                uint32_t bb = 0;
                const uint32_t c = codes4((uint32_t)src[off + col] | 0x41414100u, bb);   // pad the other lanes with 'A'
                bad |= bb;
                lb[4 * ((p >> 5) * gs + (p & 31) * mw) + col] = (uint8_t)(c & 3u);
            }
        }
        __syncthreads();
        for (int task = t; task < GB * nch; task += 256) {
            const int gl = task % GB, c = task / GB;
            if (g0 + gl >= G) continue;
            uint32_t lo[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u};
            const uint32_t* __restrict__ row = lds + gl * gs + c;
#pragma unroll
            for (int s = 0; s < 32; s++) {
                const uint32_t cc = row[s * mw];
                lo[s >> 3] |= (cc & 0x01010101u) << (s & 7);
                hi[s >> 3] |= ((cc >> 1) & 0x01010101u) << (s & 7);
            }
            uint32_t wl[4], wh[4];
#pragma unroll
            for (int tt = 0; tt < 4; tt++) {
                // word of position 4c+tt: byte q = slots 8q..8q+7
                const uint32_t sel01 = (uint32_t)tt | ((uint32_t)(tt + 4) << 8) | 0x0C0C0000u;
                const uint32_t sel23 = 0x00000C0Cu | ((uint32_t)tt << 16) | ((uint32_t)(tt + 4) << 24);
                wl[tt] = __builtin_amdgcn_perm(lo[1], lo[0], sel01) | __builtin_amdgcn_perm(lo[3], lo[2], sel23);
                wh[tt] = __builtin_amdgcn_perm(hi[1], hi[0], sel01) | __builtin_amdgcn_perm(hi[3], hi[2], sel23);
            }
            out4[((int64_t)(2 * side) * nch + c) * G + g0 + gl] = make_uint4(wl[0], wl[1], wl[2], wl[3]);
            out4[((int64_t)(2 * side + 1) * nch + c) * G + g0 + gl] = make_uint4(wh[0], wh[1], wh[2], wh[3]);
        }
        __syncthreads();
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
    const int64_t mw = cdiv(m, 4);
    const int64_t group_bytes = (32 * mw + 1) * 4;
    if (group_bytes <= 65536) {
        // tiled path: GB groups per block, LDS <= 32 KiB when possible
        int GB = (int)std::max<int64_t>(1, std::min<int64_t>(8, 32768 / group_bytes));
        // the streaming path: at most 8 sixteen-byte loads per thread and side
        const bool fast = index == nullptr && m % 4 == 0 && (int64_t)GB * mw <= 256 &&
                          ((((uintptr_t)reads | (uintptr_t)refs) & 15u) == 0);
        // the fast path needs pair i at byte i*m
        const bool contiguous = offsets == nullptr;
        const size_t shmem = (size_t)GB * group_bytes;
        hipLaunchKernelGGL(k_pack_tile, dim3((unsigned)cdiv(G, GB)), dim3(256), shmem, s, reads, refs, offsets, index,
                           n_pairs, m, G, GB, (fast && contiguous) ? 1 : 0, packed, err);
        return hipGetLastError();
    }
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
