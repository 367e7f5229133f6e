// Bit-stream encoder, one-pair-per-lane filter and wavefront-cooperative filter.
//
// Bit-stream layout: four planes (Q0, Q1, R0, R1) of the concatenated batch;
// base b is bit b%32 of word b/32 of its plane, code A=0 C=1 G=2 T=3 (plane 0 =
// low bit).  Every plane carries two zero guard words at its end.
#include "ss_pack_ops.h"
#include "ss_wave.h"

namespace ss {
namespace {

// three-input logic (v_bitop3_b32); truth-table index (src0 << 2) | (src1 << 1) | src2
#define SS_BITOP3(a, b, c, imm) __builtin_amdgcn_bitop3_b32((a), (b), (c), (imm))

// --------------------------------------------------------------- encoder
// TWO: reads and refs into planes Q0, Q1, R0, R1; otherwise one side (reads)
// into two planes.
template <bool TWO>
__global__ __launch_bounds__(256) void k_pack_stream(const uint8_t* __restrict__ reads,
                                                     const uint8_t* __restrict__ refs, int64_t total,
                                                     int64_t SW, int aligned, uint32_t* __restrict__ packed,
                                                     uint32_t* __restrict__ err)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= SW) return;
    const uint32_t bad = stream_pack::pack_word<TWO>(reads, refs, total, SW, aligned, packed, w);
    if (bad && err) atomicOr(err, 1u);
}

using wave::bits32;
using wave::span_mask;

// --------------------------------------------------------------- one pair per lane
// Each lane holds one pair.  Word by word (32 columns, the same word for every
// lane of the wave), the lane builds its 2E+1 rows of Equation 1 as mismatch
// masks and runs the walk of Section 2.4 inside the word with the borrow
// trick: for a checkpoint at bit b, (M - 2^b) & ~M marks the free cells of the
// row from b up to its first obstacle, so the OR over rows is the longest
// escape segment; a borrow that runs off bit 31 carries the segment into the
// next word (one carry bit per row).
template <int E, bool VAR_E>
__global__ __launch_bounds__(256) void k_plain(const uint32_t* __restrict__ qpk, int64_t SWq,
                                               const uint32_t* __restrict__ rpk, int64_t SWr,
                                               const int64_t* __restrict__ offsets,
                                               const int32_t* __restrict__ lengths,
                                               const int32_t* __restrict__ Epp, int64_t n,
                                               uint16_t* __restrict__ out)
{
    constexpr int NR = 2 * E + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool lane_ok = i < n;
    const int64_t ii = lane_ok ? i : 0;
    const int m = lane_ok ? lengths[ii] : 0;
    const int Ei = VAR_E ? Epp[ii] : E;
    const int64_t b0 = offsets[ii];
    const uint32_t* __restrict__ Q0 = qpk;
    const uint32_t* __restrict__ Q1 = qpk + SWq;
    const uint32_t* __restrict__ R0 = rpk;
    const uint32_t* __restrict__ R1 = rpk + SWr;
    auto qword = [&](const uint32_t* P, int u) { return bits32(P, SWq, b0 + 32 * (int64_t)u); };
    auto rword = [&](const uint32_t* P, int u) { return bits32(P, SWr, b0 + 32 * (int64_t)u); };
    auto vword = [&](int u) { return span_mask(0 - 32 * u, m - 32 * u); };   // query positions inside [0, m)

    const int W = (m + 31) >> 5;
    bool done = !lane_ok || m == 0;
    int nobs = 0, p = 0;
    uint32_t cin[NR], D[NR], M[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) { cin[r] = 0u; D[r] = 0u; M[r] = ~0u; }
    uint32_t qp0 = 0, qp1 = 0, vp = 0;
    uint32_t qc0 = done ? 0u : qword(Q0, 0), qc1 = done ? 0u : qword(Q1, 0), vc = vword(0);

    for (int w = 0;; w++) {
        const bool act0 = !done && w < W;
        if (!__any(act0)) break;
        uint32_t qn0 = 0, qn1 = 0, r0 = 0, r1 = 0;
        if (act0) {
            qn0 = qword(Q0, w + 1);
            qn1 = qword(Q1, w + 1);
            r0 = rword(R0, w);
            r1 = rword(R1, w);
        }
        const uint32_t vn = vword(w + 1);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const int k = r - E;
            uint32_t a0, a1, v;
            if (k >= 0) {
                a0 = __builtin_amdgcn_alignbit(qn0, qc0, k);
                a1 = __builtin_amdgcn_alignbit(qn1, qc1, k);
                v = __builtin_amdgcn_alignbit(vn, vc, k);
            } else {
                a0 = __builtin_amdgcn_alignbit(qc0, qp0, 32 + k);
                a1 = __builtin_amdgcn_alignbit(qc1, qp1, 32 + k);
                v = __builtin_amdgcn_alignbit(vc, vp, 32 + k);
            }
            const uint32_t mm = SS_BITOP3(r0, a0, v, 0x7D);          // (r0 ^ a0) | ~v
            uint32_t row = SS_BITOP3(mm, r1, a1, 0xF6);              // mm | (r1 ^ a1)
            if (VAR_E && (k > Ei || -k > Ei)) row = ~0u;
            M[r] = row;
        }
        bool act = act0;
        uint32_t bitp = (act && (p >> 5) == w) ? (1u << (p & 31)) : 0u;
        uint32_t U = 0;
        if (act) {
#pragma unroll
            for (int r = 0; r < NR; r++) {
                D[r] = M[r] - (bitp | cin[r]);
                U |= D[r] & ~M[r];
            }
        }
        for (;;) {
            if (act) {
                if (U >> 31) {
                    act = false;                            // segment continues into the next word
                } else {
                    const int sb = bitp ? (int)__builtin_ctz(bitp) : 0;
                    const int reach = U ? 32 - (int)__builtin_clz(U) : sb;
                    const int rabs = 32 * w + reach;
                    if (rabs >= m) {
                        done = true;                        // the segment reaches the destination
                        act = false;
                    } else {
                        nobs++;
                        p = rabs + 1;
                        if (nobs > Ei) { done = true; act = false; }
                        else if (p >= 32 * (w + 1)) act = false;
                        else bitp = 1u << (p & 31);
                    }
                }
            }
            if (!__any(act)) break;
            if (act) {
                U = 0;
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    D[r] = M[r] - bitp;
                    U |= D[r] & ~M[r];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; r++) cin[r] = (D[r] & ~M[r]) >> 31;
        qp0 = qc0; qp1 = qc1; vp = vc;
        qc0 = qn0; qc1 = qn1; vc = vn;
    }
    if (lane_ok) out[i] = (uint16_t)((nobs <= Ei ? 0x8000u : 0u) | (uint32_t)nobs);
}

// --------------------------------------------------------------- wavefront-cooperative
// Standalone launch of the sweep in ss_wave.h: LP lanes per pair, RS slices per
// lane, pairs in input order (64 / LP pairs per wavefront).  The query of pair
// i is qlen[i] bases from stream bit qoff[i] of the query planes, its
// reference rlen[i] bases from bit roff[i] of the reference planes;
// with equal lengths the walk covers every column, otherwise the columns that
// hold a comparison of two existing characters (wave::columns_walked).
template <int LP, int RS>
__global__ __launch_bounds__(256) void k_wave(wave::GlobalPlanes planes, const int64_t* __restrict__ qoff,
                                              const int32_t* __restrict__ qlen, const int64_t* __restrict__ roff,
                                              const int32_t* __restrict__ rlen, const int32_t* __restrict__ Epp,
                                              int64_t n, int Emax, uint16_t* __restrict__ out)
{
    constexpr int PW = 64 / LP;
    const int lane = threadIdx.x & 63;
    const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int grp = lane / LP, lip = lane % LP;
    const int64_t pi = wv * PW + grp;
    const bool pair_ok = pi < n;
    const int64_t pc = pair_ok ? pi : 0;
    const int nq = pair_ok ? qlen[pc] : 0;
    const int m = pair_ok ? rlen[pc] : 0;
    const int Ei = Epp ? Epp[pc] : Emax;
    const int mw = wave::columns_walked(m, nq, Ei);
    const int c = wave::sweep_pair2<RS, LP>(planes, qoff[pc], roff[pc], mw, nq, Ei, pair_ok, LP, lip, Emax);
    if (pair_ok && lip == 0) out[pi] = wave::result_word(c, Ei);
}

__global__ __launch_bounds__(256) void k_unpack(const uint16_t* __restrict__ res, int64_t n,
                                                uint8_t* __restrict__ accept, int32_t* __restrict__ edits)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = res[i];
    if (accept) accept[i] = (uint8_t)(v >> 15);
    if (edits) edits[i] = (int32_t)(v & 0x7FFFu);
}

template <int E>
hipError_t launch_plain_E(const uint32_t* qpk, int64_t SWq, const uint32_t* rpk, int64_t SWr, const int64_t* off,
                          const int32_t* len, const int32_t* Epp, int64_t n, uint16_t* out, hipStream_t s)
{
    const int threads = 256;
    const unsigned blocks = (unsigned)cdiv(n, threads);
    if (Epp)
        hipLaunchKernelGGL((k_plain<E, true>), dim3(blocks), dim3(threads), 0, s, qpk, SWq, rpk, SWr, off, len, Epp,
                           n, out);
    else
        hipLaunchKernelGGL((k_plain<E, false>), dim3(blocks), dim3(threads), 0, s, qpk, SWq, rpk, SWr, off, len, Epp,
                           n, out);
    return hipGetLastError();
}

template <int... Es>
struct PlainTable {
    static hipError_t run(int E, const uint32_t* qpk, int64_t SWq, const uint32_t* rpk, int64_t SWr,
                          const int64_t* off, const int32_t* len, const int32_t* Epp, int64_t n, uint16_t* out,
                          hipStream_t s)
    {
        hipError_t r = hipErrorInvalidValue;
        ((E == Es ? (r = launch_plain_E<Es>(qpk, SWq, rpk, SWr, off, len, Epp, n, out, s), 0) : 0), ...);
        return r;
    }
};

struct WaveArgs {
    wave::GlobalPlanes planes;
    const int64_t* qoff;
    const int32_t* qlen;
    const int64_t* roff;
    const int32_t* rlen;
    const int32_t* Epp;
    int64_t n;
    int E;
    uint16_t* out;
};

template <int LP, int RS>
hipError_t launch_wave_LR(const WaveArgs& a, hipStream_t s)
{
    constexpr int PW = 64 / LP;
    const int64_t waves = cdiv(a.n, PW);
    const int threads = 256;
    const unsigned blocks = (unsigned)cdiv(waves * 64, threads);
    hipLaunchKernelGGL((k_wave<LP, RS>), dim3(blocks), dim3(threads), 0, s, a.planes, a.qoff, a.qlen, a.roff, a.rlen,
                       a.Epp, a.n, a.E, a.out);
    return hipGetLastError();
}

template <int RS>
hipError_t launch_wave_R(int LP, const WaveArgs& a, hipStream_t s)
{
    switch (LP) {
    case 1: return launch_wave_LR<1, RS>(a, s);
    case 2: return launch_wave_LR<2, RS>(a, s);
    case 4: return launch_wave_LR<4, RS>(a, s);
    case 8: return launch_wave_LR<8, RS>(a, s);
    case 16: return launch_wave_LR<16, RS>(a, s);
    case 32: return launch_wave_LR<32, RS>(a, s);
    case 64: return launch_wave_LR<64, RS>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_wave_args(const WaveArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    int LP, RS;
    wave_shape(a.E, &LP, &RS);
    switch (RS) {
    case 1: return launch_wave_R<1>(LP, a, s);
    case 2: return launch_wave_R<2>(LP, a, s);
    case 4: return launch_wave_R<4>(LP, a, s);
    case 8: return launch_wave_R<8>(LP, a, s);
    case 16: return launch_wave_R<16>(LP, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

void wave_shape(int32_t E, int* lanes_per_pair, int* slices_per_lane)
{
    // standalone launches use power-of-two slices per lane, up to 16
    const int SL = (int)cdiv(2 * (int64_t)E + 1, 32);
    int RS = 1;
    while (RS < SL && RS < 16) RS <<= 1;
    int LP = 1;
    while ((int64_t)LP * RS < SL) LP <<= 1;
    *lanes_per_pair = LP;
    *slices_per_lane = RS;
}

hipError_t launch_pack_stream(const uint8_t* reads, const uint8_t* refs, int64_t total_bases, uint32_t* packed,
                              uint32_t* err, hipStream_t s)
{
    const int64_t SW = cdiv(total_bases, 32) + 2;
    const int aligned = ((((uintptr_t)reads) | ((uintptr_t)refs)) & 15u) == 0;
    const int threads = 256;
    hipLaunchKernelGGL(k_pack_stream<true>, dim3((unsigned)cdiv(SW, threads)), dim3(threads), 0, s, reads, refs,
                       total_bases, SW, aligned, packed, err);
    return hipGetLastError();
}

hipError_t launch_pack_side(const uint8_t* ascii, int64_t total_bases, uint32_t* packed, uint32_t* err, hipStream_t s)
{
    const int64_t SW = cdiv(total_bases, 32) + 2;
    const int aligned = (((uintptr_t)ascii) & 15u) == 0;
    const int threads = 256;
    hipLaunchKernelGGL(k_pack_stream<false>, dim3((unsigned)cdiv(SW, threads)), dim3(threads), 0, s, ascii,
                       (const uint8_t*)nullptr, total_bases, SW, aligned, packed, err);
    return hipGetLastError();
}

hipError_t launch_plain(const uint32_t* packed, int64_t stream_words, const int64_t* offsets,
                        const int32_t* lengths, const int32_t* Epp, int64_t n, int32_t E, uint16_t* out,
                        hipStream_t s)
{
    if (n == 0) return hipSuccess;
    return launch_plain_sides(packed, stream_words, packed + 2 * stream_words, stream_words, offsets, lengths, Epp,
                              n, E, out, s);
}

hipError_t launch_plain_sides(const uint32_t* qpk, int64_t q_words, const uint32_t* rpk, int64_t r_words,
                              const int64_t* offsets, const int32_t* lengths, const int32_t* Epp, int64_t n,
                              int32_t E, uint16_t* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    using Tab = PlainTable<0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23,
                           24, 25, 26, 27, 28, 29, 30, 31>;
    return Tab::run(E, qpk, q_words, rpk, r_words, offsets, lengths, Epp, n, out, s);
}

hipError_t launch_wave(const uint32_t* packed, int64_t stream_words, const int64_t* offsets,
                       const int32_t* lengths, const int32_t* Epp, int64_t n, int32_t E, uint16_t* out,
                       hipStream_t s)
{
    const WaveArgs a{wave::GlobalPlanes{packed, packed + 2 * stream_words, stream_words, stream_words},
                     offsets, lengths, offsets, lengths, Epp, n, E, out};
    return launch_wave_args(a, s);
}

hipError_t launch_wave_sides(const uint32_t* qpk, int64_t q_words, const uint32_t* rpk, int64_t r_words,
                             const int64_t* qoff, const int32_t* qlen, const int64_t* roff, const int32_t* rlen,
                             const int32_t* Epp, int64_t n, int32_t E, uint16_t* out, hipStream_t s)
{
    const WaveArgs a{wave::GlobalPlanes{qpk, rpk, q_words, r_words}, qoff, qlen, roff, rlen, Epp, n, E, out};
    return launch_wave_args(a, s);
}

hipError_t launch_unpack(const uint16_t* res, int64_t n, uint8_t* accept, int32_t* edits, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, res, n, accept, edits);
    return hipGetLastError();
}

}  // namespace ss
