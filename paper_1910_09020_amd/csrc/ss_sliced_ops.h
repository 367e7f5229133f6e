// Bit-sliced helpers shared by the lane-sliced column sweep (ss_sliced_kernel.h)
// and the fused encode-and-sweep kernel (ss_fused.h): three-input logic, the
// decision and result words of a group of 32 pairs.
#pragma once
#include "ss_common.h"

namespace ss {

// Lane-sliced layout in device memory.  Groups of 32 pairs come in blocks of
// kSlicedBlock groups (the groups one wavefront of the sweep takes); block b
// holds the words of its Gb = min(kSlicedBlock, G - kSlicedBlock * b) groups
// contiguously, plane-major, then chunk, then group: the 16-byte word of
// (plane p, chunk c, group g) is uint4 number
//     kSlicedBlock * 4 * nch * b + (p * nch + c) * Gb + (g - kSlicedBlock * b),
// so that each wavefront's loads sweep one contiguous stretch of memory.
constexpr int kSlicedBlock = 64;
__host__ __device__ inline int64_t sliced_block_base(int64_t g, int64_t nch)
{
    return (g / kSlicedBlock) * kSlicedBlock * 4 * nch;
}
__host__ __device__ inline int64_t sliced_block_groups(int64_t g, int64_t G)
{
    const int64_t b0 = g - g % kSlicedBlock;
    return G - b0 < kSlicedBlock ? G - b0 : kSlicedBlock;
}

namespace sliced {

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

__device__ __forceinline__ uint32_t comp(const uint4& v, int t)
{
    return t == 0 ? v.x : (t == 1 ? v.y : (t == 2 ? v.z : v.w));
}

__device__ __forceinline__ constexpr int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Write the 32 results of group g: acc (bit s: pair 32g+s accepted) and the
// count's binary digits dig; one 16-bit word per pair (bit 15 accept, low bits
// the count).
template <int NB>
__device__ __forceinline__ void write_digits(const uint32_t (&dig)[NB], uint32_t acc, int64_t g, int64_t n_pairs,
                                             uint16_t* __restrict__ out)
{
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

// Decide and write (step 5) for the 32 pairs of group g from the thermometer
// T (T[l-1]: count >= l): accept = count <= E, count in binary digits; one
// 16-bit word per pair (bit 15 accept, low bits the count).
template <int E>
__device__ __forceinline__ void write_group(const uint32_t (&T)[E + 1], int64_t g, int64_t n_pairs,
                                            uint16_t* __restrict__ out)
{
    constexpr int NB = (E + 1) < 2 ? 1 : (E + 1) < 4 ? 2 : (E + 1) < 8 ? 3 : (E + 1) < 16 ? 4 : (E + 1) < 32 ? 5 : 6;
    uint32_t dig[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        uint32_t x = 0;
#pragma unroll
        for (int i = 1; (i << b) <= E + 1; i++) x ^= T[(i << b) - 1];
        dig[b] = x;
    }
    write_digits<NB>(dig, ~T[E], g, n_pairs, out);
}
}  // namespace sliced
}  // namespace ss
