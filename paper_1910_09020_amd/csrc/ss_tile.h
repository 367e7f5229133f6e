// Tiled encoder body shared by the standalone encoder and the fused
// encode-and-sweep kernel.
//
// NT threads of a block (256 in the standalone encoder, fewer in the fused
// kernel, where one wavefront sweeps) encode GB consecutive groups of 32 pair
// slots into the lane-sliced layout (bit s of a word belongs to slot
// 32*g + s).  Phase 1 copies the slots' bases into LDS staging as codes (one
// byte per base, the code's low bit at bit 0 and its high bit at bit 4; rows
// padded to whole dwords, four pad dwords per group: 16-byte stores stay
// aligned, and the 32 phase-2 reads of a half-wave, 8 groups x 4 chunks, fall
// in 32 different banks) and validates every byte: a byte b is one of ACGTacgt
// exactly when (b & 0xDF) equals the letter its code stands for.  Phase 2: one
// thread per (group, chunk of four positions) folds the 32 slots' code dwords
// into the four words of each plane: shifting slot s's dword left by s % 4 puts
// four slots' low bits in the low nibble of each byte and their high bits in
// the high nibble, and byte permutes take the nibbles to the words.
#pragma once
#include "ss_common.h"

namespace ss {
namespace tile {

// dwords of LDS staging per group of 32 slots of length m
__host__ __device__ inline int stage_dwords(int m) { return 32 * ((m + 3) >> 2) + 4; }

// Codes of the four bytes of x (A 0, C 1, G 2, T 3, either case), each in its
// byte with the low bit at bit 0 and the high bit at bit 4.  Bits 1 and 2 of a
// letter tell the four apart (A 0, C 2, T 4, G 6) and select, by byte permute,
// both the code and the letter itself; bad accumulates x ^ letter, which for a
// valid byte differs at most in the case bit (see invalid).
__device__ __forceinline__ uint32_t codes4(uint32_t x, uint32_t& bad)
{
    const uint32_t sel = x & 0x06060606u;
    const uint32_t cc = __builtin_amdgcn_perm(0x00100011u, 0x00010000u, sel);      // A 00, C 01, T 11, G 10 (hex)
    const uint32_t letter = __builtin_amdgcn_perm(0x00470054u, 0x00430041u, sel);  // 'A', 'C', 'T', 'G'
    bad |= x ^ letter;
    return cc;
}

// true when some byte that went through codes4 was not one of ACGTacgt
__device__ __forceinline__ bool invalid(uint32_t bad) { return (bad & 0xDFDFDFDFu) != 0u; }

constexpr int kQ = 8;      // 16-byte loads per thread and side on the standalone encoder's fast path
constexpr int kFusedThreads = 192;  // encoding threads of a fused block (waves 0..2; wave 3 sweeps)
constexpr int kFusedQ = 9;         // their 16-byte loads per thread and side (192 * 9 * 16 B >= 8 groups of 100 bp)
constexpr int kWaveQ = 7;          // 16-byte loads per lane and side when one wavefront encodes alone (64 * 7 * 16 B >= 2 groups of 100 bp)
// uint4 words of one group in a fused tile buffer: the four planes of
// ceil(m/4) chunks one after another (group-major, so the positions of a plane
// are consecutive words), plus one uint4 of padding that spreads consecutive
// groups over the LDS banks
__host__ __device__ inline int fused_group_chunks(int m) { return 4 * ((m + 3) >> 2) + 1; }
// words of the fused sweep's column store in wave mode: 16 groups (a pass of the
// sweeping wavefront at four lanes per group) of m words, at an odd stride
__host__ __device__ inline int fused_dead_words(int m) { return 16 * (m | 1); }

// Encoder mode for GB groups of pairs of length m stored back to back from
// 16-byte aligned bases (contiguous), else 0: 1 when m % 4 == 0 and each side
// of the GB groups fits nt * kq sixteen-byte loads (nt encoding threads), 2
// when m % 4 != 0 and the raw bytes fit them as well.
__host__ __device__ inline int fast_mode(int m, int GB, bool contiguous, int kq = kQ, int nt = 256)
{
    if (!contiguous || m <= 0) return 0;
    const int64_t bytes = 32ll * GB * (m % 4 == 0 ? m : 4 * ((m + 3) / 4));
    if (bytes > (int64_t)nt * kq * 16) return 0;
    return m % 4 == 0 ? 1 : 2;
}

// Fast path: the 16-byte loads of groups g0 .. g0+GB-1, both sides, by NT
// threads (thread tid of them takes loads tid, tid + NT, ...).  Raw buffer loads over exactly the
// groups' bytes: the hardware range check returns zero for a load past the
// end instead of touching memory, so every load is issued unconditionally
// (straight-line code keeps all of them in flight together, and a caller can
// issue the next groups' loads before consuming these).  present == false
// issues loads over an empty range (nothing is read).
template <int KQ = kQ, int NT = 256>
__device__ __forceinline__ void load_groups(const uint8_t* __restrict__ reads, const uint8_t* __restrict__ refs,
                                            int64_t n_pairs, int m, int64_t g0, int GB, bool present,
                                            uint4 (&v)[2][KQ], int tid = (int)threadIdx.x)
{
    const int64_t s0 = g0 * 32;
    const int np = present ? (int)min((int64_t)32 * GB, n_pairs - s0) : 0;
    const int nbytes = np > 0 ? np * m : 0;
#pragma unroll
    for (int sd = 0; sd < 2; sd++) {
        const uint8_t* base = (sd ? refs : reads) + (present ? s0 * (int64_t)m : 0);
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base), (short)0, nbytes, 0x00020000);
#pragma unroll
        for (int k = 0; k < KQ; k++)
            v[sd][k] = __builtin_bit_cast(
                uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * (tid + NT * k), 0, 0));
    }
}

// the barrier of a whole block
struct BlockBarrier {
    __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

// for NT = 64 (one wavefront encodes): its LDS accesses before, in order before
// those after (no other wavefront takes part)
struct WaveSync {
    __device__ __forceinline__ void operator()() const
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
};

// Encode groups g0 .. g0+GB-1 (those that hold a slot below n_pairs); GB is a
// power of two.  Slot i reads pair index[i] (or i) at offsets[pair] (or
// pair * m).  The words of (plane p, chunk c, local group gl) go to
// out4[(p * nch + c) * ostride + (obase + gl) * gstride] (out4 may point to
// global memory or to LDS).  stage: GB * stage_dwords(m) dwords of LDS, 16-byte
// aligned.  NT threads (tid 0 .. NT-1) do the work.
// fast (see fast_mode): 0 = any slots, byte loads; 1 or 2 = slots are pairs
// stored back to back from a 16-byte aligned byte (index and offsets null)
// and v holds load_groups' loads of these groups; 1 when m % 4 == 0 (codes
// staged per slot row), 2 otherwise (raw bytes staged in source order, read
// back per slot and chunk with a byte-align).  It synchronises the encoding
// threads four times through bar (by default the block barrier, in which every
// thread of the block takes part).
template <int KQ = kQ, int NT = 256, class BAR = BlockBarrier>
__device__ __forceinline__ void encode_groups(const uint8_t* __restrict__ reads, const uint8_t* __restrict__ refs,
                                              const int64_t* __restrict__ offsets,
                                              const int64_t* __restrict__ index, int64_t n_pairs, int m,
                                              int64_t g0, int GB, int fast, const uint4 (&v)[2][KQ],
                                              uint32_t* __restrict__ stage, uint4* __restrict__ out4,
                                              int64_t ostride, int64_t obase, uint32_t& bad,
                                              int64_t gstride = 1, const BAR& bar = BAR(),
                                              int tid = (int)threadIdx.x)
{
    const int mw = (m + 3) >> 2;              // dwords per slot row
    const int gs = 32 * mw + 4;               // dwords per group
    const int nch = mw;
    const int64_t s0 = g0 * 32;
    const int np = (int)min((int64_t)32 * GB, n_pairs - s0);
    const int lgb = 31 - __builtin_clz((unsigned)GB);
    const int t = tid;
    const int ndw = np * mw;
    const int nq = ndw >> 2;
    // Staging index of source dword dw (slot p = dw / mw, column dw % mw):
    // (p / 32) * gs + (p % 32) * mw + dw % mw = dw + 4 * (dw / (32 * mw)).  The
    // four dwords of a 16-byte load share their group (32 * mw is a multiple
    // of 4), so one quotient q / (8 * mw) serves all four and they go out as
    // one aligned 16-byte store.  Quotients by multiply-high with
    // ceil(2^32 / d): exact while x * d < 2^32 (here x < 2^13 and d <= 2^13
    // on the fast path, x < 2^11 for q).
    const uint32_t d16 = 8u * (uint32_t)(mw > 0 ? mw : 1), d4 = 4u * d16;
    const uint32_t r16 = 0xFFFFFFFFu / d16 + 1u, r4 = 0xFFFFFFFFu / d4 + 1u;
#pragma unroll
    for (int side = 0; side < 2; side++) {
        const uint8_t* __restrict__ src = side ? refs : reads;
        if (fast == 2) {
            // raw bytes in source order; the bytes past the last whole 16 one at a time
            const int nb = np * m, nq16 = nb >> 4;
#pragma unroll
            for (int k = 0; k < KQ; k++) {
                const int q = t + NT * k;
                if (q < nq16) reinterpret_cast<uint4*>(stage)[q] = v[side][k];
            }
            const uint8_t* __restrict__ sb = src + s0 * (int64_t)m;
            for (int i = 16 * nq16 + t; i < nb; i += NT) reinterpret_cast<uint8_t*>(stage)[i] = sb[i];
        } else if (fast) {
#pragma unroll
            for (int k = 0; k < KQ; k++) {
                const int q = t + NT * k;
                if (q < nq) {
                    uint4* __restrict__ dst = reinterpret_cast<uint4*>(stage) + q + (int)__umulhi((uint32_t)q, r16);
                    *dst = make_uint4(codes4(v[side][k].x, bad), codes4(v[side][k].y, bad),
                                      codes4(v[side][k].z, bad), codes4(v[side][k].w, bad));
                }
            }
            const uint32_t* __restrict__ s32 = reinterpret_cast<const uint32_t*>(src + s0 * (int64_t)m);
            for (int dw = 4 * nq + t; dw < ndw; dw += NT)
                stage[dw + 4 * (int)__umulhi((uint32_t)dw, r4)] = codes4(s32[dw], bad);
        } else {
            uint8_t* lb = reinterpret_cast<uint8_t*>(stage);
            const int nb = np * m;
            for (int i = t; i < nb; i += NT) {
                const int p = i / m, col = i - p * m;
                const int64_t slot = s0 + p;
                const int64_t pi = index ? index[slot] : slot;
                const int64_t off = offsets ? offsets[pi] : pi * (int64_t)m;
                uint32_t bb = 0;
                const uint32_t c = codes4((uint32_t)src[off + col] | 0x41414100u, bb);   // pad the other lanes with 'A'
                bad |= bb;
                lb[4 * ((p >> 5) * gs + (p & 31) * mw) + col] = (uint8_t)(c & 0x11u);
            }
        }
        bar();
        for (int task = t; task < GB * nch; task += NT) {
            const int gl = task & (GB - 1), c = task >> lgb;
            if (32 * gl >= np) continue;
            // acc[s / 4] byte t: bit s % 4 the low and bit 4 + s % 4 the high code
            // bit of slot s at position 4c + t
            uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
            if (fast == 2) {
                // positions 4c..4c+3 of slot p start at byte p*m + 4c; bytes past m
                // and slots past the batch read as 'A' (validated and coded once, here)
                const int keepb = m - 4 * c;
                const uint32_t keep = keepb >= 4 ? 0xFFFFFFFFu : ((1u << (8 * keepb)) - 1u);
                int off = 32 * gl * m + 4 * c;
#pragma unroll
                for (int s = 0; s < 32; s++) {
                    const uint32_t w0 = stage[off >> 2], w1 = stage[(off >> 2) + 1];
                    uint32_t x = __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)(off & 3));
                    x = (32 * gl + s < np) ? ((x & keep) | (0x41414141u & ~keep)) : 0x41414141u;
                    acc[s >> 2] |= codes4(x, bad) << (s & 3);
                    off += m;
                }
            } else {
                // staged codes; slots without a pair (the batch's last group) hold stale
                // bytes, whose bits would reach other slots through the shifts: skipped
                const uint32_t* __restrict__ row = stage + gl * gs + c;
                const int ns = np - 32 * gl;
                if (ns >= 32) {
#pragma unroll
                    for (int s = 0; s < 32; s++) acc[s >> 2] |= row[s * mw] << (s & 3);
                } else {
#pragma unroll
                    for (int s = 0; s < 32; s++)
                        if (s < ns) acc[s >> 2] |= row[s * mw] << (s & 3);
                }
            }
            // lo[q] / hi[q] byte t: the low / high code bits of slots 8q .. 8q+7
            uint32_t lo[4], hi[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                lo[q] = (acc[2 * q] & 0x0F0F0F0Fu) | ((acc[2 * q + 1] << 4) & 0xF0F0F0F0u);
                hi[q] = ((acc[2 * q] >> 4) & 0x0F0F0F0Fu) | (acc[2 * q + 1] & 0xF0F0F0F0u);
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
            out4[((int64_t)(2 * side) * nch + c) * ostride + (obase + gl) * gstride] = make_uint4(wl[0], wl[1], wl[2], wl[3]);
            out4[((int64_t)(2 * side + 1) * nch + c) * ostride + (obase + gl) * gstride] = make_uint4(wh[0], wh[1], wh[2], wh[3]);
        }
        bar();
    }
}

// load_groups + encode_groups
__device__ __forceinline__ void load_encode_groups(const uint8_t* __restrict__ reads,
                                                   const uint8_t* __restrict__ refs,
                                                   const int64_t* __restrict__ offsets,
                                                   const int64_t* __restrict__ index, int64_t n_pairs, int m,
                                                   int64_t g0, int GB, int fast, uint32_t* __restrict__ stage,
                                                   uint4* __restrict__ out4, int64_t ostride, int64_t obase,
                                                   uint32_t& bad)
{
    uint4 v[2][kQ];
    load_groups(reads, refs, n_pairs, m, g0, GB, fast != 0, v);
    encode_groups(reads, refs, offsets, index, n_pairs, m, g0, GB, fast, v, stage, out4, ostride, obase, bad);
}

}  // namespace tile
}  // namespace ss
