// Bit-stream encoder of one output word: 32 bases of the concatenated batch
// (word w holds bases 32w .. 32w + 31) into planes Q0, Q1 (and R0, R1), code
// A=0 C=1 G=2 T=3, plane 0 = low bit, any other byte flagged.  Shared by the
// stream encoder kernel and the device-resident serving loop.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {
namespace stream_pack {

// Four ASCII bytes -> low/high code bits in the low 4 bits of each result.
__device__ __forceinline__ void code4(uint32_t x, uint32_t& lo, uint32_t& hi, uint32_t& bad)
{
    const uint32_t c = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
    const uint32_t p0 = c & 0x01010101u, p1 = (c >> 1) & 0x01010101u;
    lo = ((p0 * 0x00204081u) >> 21) & 0xFu;
    hi = ((p1 * 0x00204081u) >> 21) & 0xFu;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const uint32_t v = (((x >> (8 * k)) & 0xFFu) | 0x20u) - 0x61u;
        bad |= (v < 20u) ? (((0x80045u >> v) & 1u) ^ 1u) : 1u;
    }
}

// Word w of a plane of SW words (TWO: reads and refs into Q0, Q1, R0, R1;
// otherwise reads into two planes); words at or past the last base are zero.
// aligned: reads (and refs) are 16-byte aligned, so full words load as uint4.
// Returns nonzero when one of the word's bytes is not a base.
template <bool TWO>
__device__ __forceinline__ uint32_t pack_word(const uint8_t* __restrict__ reads, const uint8_t* __restrict__ refs,
                                              int64_t total, int64_t SW, int aligned, uint32_t* __restrict__ packed,
                                              int64_t w)
{
    uint32_t q0 = 0, q1 = 0, r0 = 0, r1 = 0, bad = 0;
    const int64_t b = w * 32;
    if (b < total) {
        const int64_t nb = total - b < 32 ? total - b : 32;
        if (nb == 32 && aligned) {
            const uint4* a4 = reinterpret_cast<const uint4*>(reads + b);
            uint4 a[2] = {a4[0], a4[1]};
            uint32_t xa[8] = {a[0].x, a[0].y, a[0].z, a[0].w, a[1].x, a[1].y, a[1].z, a[1].w};
#pragma unroll
            for (int k = 0; k < 8; k++) {
                uint32_t lo, hi;
                code4(xa[k], lo, hi, bad);
                q0 |= lo << (4 * k);
                q1 |= hi << (4 * k);
            }
            if constexpr (TWO) {
                const uint4* f4 = reinterpret_cast<const uint4*>(refs + b);
                uint4 f[2] = {f4[0], f4[1]};
                uint32_t xf[8] = {f[0].x, f[0].y, f[0].z, f[0].w, f[1].x, f[1].y, f[1].z, f[1].w};
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    uint32_t lo, hi;
                    code4(xf[k], lo, hi, bad);
                    r0 |= lo << (4 * k);
                    r1 |= hi << (4 * k);
                }
            }
        } else {
            for (int k = 0; k < nb; k++) {
                uint32_t lo, hi, bb = 0;
                const uint32_t xa = reads[b + k];
                code4(xa, lo, hi, bb);
                q0 |= (lo & 1u) << k;
                q1 |= (hi & 1u) << k;
                // code4 judged three zero bytes too; only the low byte counts
                const uint32_t va = (xa | 0x20u) - 0x61u;
                bad |= (va < 20u) ? (((0x80045u >> va) & 1u) ^ 1u) : 1u;
                if constexpr (TWO) {
                    const uint32_t xf = refs[b + k];
                    code4(xf, lo, hi, bb);
                    r0 |= (lo & 1u) << k;
                    r1 |= (hi & 1u) << k;
                    const uint32_t vf = (xf | 0x20u) - 0x61u;
                    bad |= (vf < 20u) ? (((0x80045u >> vf) & 1u) ^ 1u) : 1u;
                }
            }
        }
    }
    packed[w] = q0;
    packed[SW + w] = q1;
    if constexpr (TWO) {
        packed[2 * SW + w] = r0;
        packed[3 * SW + w] = r1;
    }
    return bad;
}

}  // namespace stream_pack
}  // namespace ss
