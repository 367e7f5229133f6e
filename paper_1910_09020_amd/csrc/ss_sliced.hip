// Lane-sliced encoder and the threshold dispatch of the column-sweep kernel.
//
// Layout: bit s of every 32-bit word belongs to pair 32*g + s ("group" g, one
// group per lane of the sweep kernel).  The encoder transposes 32 pairs at a
// time with wavefront ballots: one ballot per (plane, position) gives the word
// of 32 pairs for each half of the wavefront.
#include <algorithm>

#include "ss_common.h"
#include "ss_sliced_ops.h"
#include "ss_tile.h"

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
                out4[sliced_block_base(g, nch) + ((int64_t)p * nch + cc) * sliced_block_groups(g, G) +
                     g % kSlicedBlock] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    if (bad && err) atomicOr(err, 1u);
}

// ---------------------------------------------------------------- tiled encoder
// One 256-thread block encodes GB consecutive groups into the packed buffer.
__global__ __launch_bounds__(256) void k_pack_tile(const uint8_t* __restrict__ reads,
                                                   const uint8_t* __restrict__ refs,
                                                   const int64_t* __restrict__ offsets,
                                                   const int64_t* __restrict__ index, int64_t n_pairs, int m,
                                                   int64_t G, int GB, int fast, uint32_t* __restrict__ packed,
                                                   uint32_t* __restrict__ err)
{
    extern __shared__ uint32_t lds[];
    const int64_t g0 = (int64_t)blockIdx.x * GB;
    uint32_t bad = 0;
    // GB divides kSlicedBlock, so the block's groups share one layout block
    const int64_t nch = (m + kChunk - 1) / kChunk;
    tile::load_encode_groups(reads, refs, offsets, index, n_pairs, m, g0, GB, fast, lds,
                             reinterpret_cast<uint4*>(packed) + sliced_block_base(g0, nch),
                             sliced_block_groups(g0, G), g0 % kSlicedBlock, bad);
    if (tile::invalid(bad) && err) atomicOr(err, 1u);
}

}  // namespace

hipError_t launch_sliced_lo(int E, const uint32_t* packed, int64_t n, int32_t m, int sub_width, uint16_t* out,
                           hipStream_t s);
hipError_t launch_sliced_mid(int E, const uint32_t* packed, int64_t n, int32_t m, int sub_width, uint16_t* out,
                           hipStream_t s);
hipError_t launch_sliced_hi(int E, const uint32_t* packed, int64_t n, int32_t m, int sub_width, uint16_t* out,
                           hipStream_t s);
hipError_t launch_fused_lo(int E, const uint8_t* reads, const uint8_t* refs, int64_t n, int32_t m, int T, int GB,
                          int U, int fast, size_t shmem, uint16_t* out, uint32_t* err, hipStream_t s);
hipError_t launch_fused_mid(int E, const uint8_t* reads, const uint8_t* refs, int64_t n, int32_t m, int T, int GB,
                           int U, int fast, size_t shmem, uint16_t* out, uint32_t* err, hipStream_t s);

hipError_t launch_pack_sliced(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets,
                              const int64_t* index, int64_t n_pairs, int32_t m, uint32_t* packed,
                              uint32_t* err, hipStream_t s)
{
    const int64_t G = cdiv(n_pairs, 32);
    if (G == 0 || m == 0) return hipSuccess;
    const int64_t mw = cdiv(m, 4);
    const int64_t group_bytes = (int64_t)tile::stage_dwords(m) * 4;
    if (group_bytes <= 65536) {
        // tiled path: GB groups per block, LDS <= 32 KiB when possible
        int GB = 8;
        while (GB > 1 && GB * group_bytes > 32768) GB >>= 1;
        // the streaming paths need pair i at byte i*m from 16-byte aligned bases
        const bool contiguous = index == nullptr && offsets == nullptr &&
                                ((((uintptr_t)reads | (uintptr_t)refs) & 15u) == 0);
        const size_t shmem = (size_t)GB * group_bytes;
        hipLaunchKernelGGL(k_pack_tile, dim3((unsigned)cdiv(G, GB)), dim3(256), shmem, s, reads, refs, offsets, index,
                           n_pairs, m, G, GB, tile::fast_mode(m, GB, contiguous), packed, err);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_pack_sliced, dim3((unsigned)G), dim3(64), 0, s, reads, refs, offsets, index, n_pairs, m,
                       G, packed, err);
    return hipGetLastError();
}

hipError_t launch_sliced(const uint32_t* packed, int64_t n_pairs, int32_t m, int32_t E, uint16_t* out,
                         hipStream_t s, int sub_width)
{
    if (n_pairs == 0) return hipSuccess;
    if (E < 0 || E > kMaxESliced) return hipErrorInvalidValue;
    if (E <= 10) return launch_sliced_lo(E, packed, n_pairs, m, sub_width, out, s);
    if (E <= 20) return launch_sliced_mid(E, packed, n_pairs, m, sub_width, out, s);
    return launch_sliced_hi(E, packed, n_pairs, m, sub_width, out, s);
}

// Tile shape of the fused kernel: T groups per tile buffer (two of them), in
// wave mode the sweep's column words, and 16 bytes of counters; U > 0 groups
// per unit when each encoding wavefront encodes by itself (contiguous pairs
// whose U groups fit its loads), else U = 0 and GB groups staged at a time by
// the three together.  Returns the LDS bytes per block, or 0 when no shape
// fits.
int fused_tile_cap(int64_t n_pairs)
{
    // the automatic tile leaves no CU without a tile: at most G / CUs groups per tile
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess || cus <= 0)
        return 256;
    const int64_t G = cdiv(n_pairs, 32);
    return (int)std::max<int64_t>(1, std::min<int64_t>(256, G / cus));
}

size_t fused_shape(int32_t m, int tile_groups, bool contiguous, int* T_out, int* GB_out, int* U_out, int max_t)
{
    const int64_t stage_b = (int64_t)tile::stage_dwords(m) * 4;
    const int64_t buf_b = 16ll * tile::fused_group_chunks(m);   // one group in one tile buffer
    // T: the given tile, else the largest step multiple that keeps two blocks per CU
    // (a multiple of 16 from 16 on: the sweeping wave's groups per pass), else one
    auto pick = [&](int step, auto&& lds_for) -> int {
        if (tile_groups > 0)
            return (tile_groups % step == 0 && lds_for(tile_groups) <= kMaxFusedLds) ? tile_groups : 0;
        for (int blocks = 2; blocks >= 1; blocks--) {
            int T = 0;
            for (int t = step; t <= std::min(256, std::max(max_t, step)); t += step)
                if ((t < 16 || t % 16 == 0) && blocks * lds_for(t) <= kMaxFusedLds) T = t;
            if (T > 0) return T;
        }
        return 0;
    };
    for (int U = 2; U >= 1 && contiguous && m > 0; U >>= 1) {
        if (tile::fast_mode(m, U, true, tile::kWaveQ, 64) == 0) continue;
        const int64_t sw = 3 * ((U * stage_b + 15) & ~(int64_t)15);
        auto lds_w = [&](int64_t T) { return sw + 2 * T * buf_b + 4ll * tile::fused_dead_words(m) + 16; };
        const int T = pick(U, lds_w);
        if (T > 0) {
            *T_out = T;
            *GB_out = U;
            *U_out = U;
            return (size_t)lds_w(T);
        }
    }
    // staging groups: the most whose bytes the encoding threads' loads cover (so the
    // streaming path applies), and whose staging fits 32 KiB
    int GB = 8;
    while (GB > 1 &&
           (GB * stage_b > 32768 || tile::fast_mode(m, GB, true, tile::kFusedQ, tile::kFusedThreads) == 0))
        GB >>= 1;
    if (tile_groups > 0)
        while (GB > 1 && tile_groups % GB != 0) GB >>= 1;
    auto lds_b = [&](int64_t T) { return ((GB * stage_b + 15) & ~(int64_t)15) + 2 * T * buf_b + 16; };
    const int T = pick(GB, lds_b);
    if (T == 0) return 0;
    *T_out = T;
    *GB_out = GB;
    *U_out = 0;
    return (size_t)lds_b(T);
}

hipError_t launch_fused(const uint8_t* reads, const uint8_t* refs, int64_t n_pairs, int32_t m, int32_t E,
                        int tile_groups, uint16_t* out, uint32_t* err, hipStream_t s)
{
    if (n_pairs == 0) return hipSuccess;
    if (E < 0 || E > kMaxEFused) return hipErrorInvalidValue;
    const bool contiguous = (((uintptr_t)reads | (uintptr_t)refs) & 15u) == 0;
    int T = 0, GB = 0, U = 0;
    const size_t shmem = fused_shape(m, tile_groups, contiguous, &T, &GB, &U, fused_tile_cap(n_pairs));
    if (shmem == 0) return hipErrorInvalidValue;
    const int fast = U > 0 ? tile::fast_mode(m, U, true, tile::kWaveQ, 64)
                           : tile::fast_mode(m, GB, contiguous, tile::kFusedQ, tile::kFusedThreads);
    if (E <= 5) return launch_fused_lo(E, reads, refs, n_pairs, m, T, GB, U, fast, shmem, out, err, s);
    return launch_fused_mid(E, reads, refs, n_pairs, m, T, GB, U, fast, shmem, out, err, s);
}

}  // namespace ss
