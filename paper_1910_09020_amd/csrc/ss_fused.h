// Fused encode-and-sweep kernel (the one-call path for E <= 10): the encoder of
// ss_tile.h writes each tile of pairs into on-chip memory, where the column
// sweep of Section 2.4 runs on it; the packed encoding never reaches device
// memory.
#pragma once
#include <algorithm>
#include "ss_sliced_ops.h"
#include "ss_tile.h"

namespace ss {
namespace sliced {

// ---------------------------------------------------------------- fused kernel
// Roles in a fused block of 256 threads: waves 0..2 encode, wave 3 sweeps.
constexpr int kFusedEnc = tile::kFusedThreads;
constexpr int kFusedEncQ = tile::kFusedQ;

// Lanes that sweep one group: for E > 0 the 2E+1 rows are split over a quad's
// lanes, so the 16 groups of a 100 bp tile fill the sweeping wavefront and a
// lane runs about 18 instructions per column (at E = 5) instead of 44.
constexpr int fused_lanes(int E) { return E == 0 ? 1 : 4; }
constexpr int kFusedCPI = 2;   // chunks per item of the sweep (one LDS round trip per item)

// OR of x over the LPG consecutive lanes of one group (LPG = 1, 2 or 4; the
// lanes of a group lie in one quad)
template <int LPG>
__device__ __forceinline__ uint32_t quad_or(uint32_t x)
{
    if (LPG >= 2) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    if (LPG >= 4) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    return x;
}

// Column sweep of one group held in LDS in the group-major layout (word P of
// plane p at gp[p * 4 * nch + P]; planes Q0, Q1, R0, R1) by LPG lanes, CPI
// chunks of four columns per call, so that a sweep can be cut into pieces.
// Lane h of the group takes SL = ceil((2E+1) / LPG) of the rows, diagonal
// offsets sh - E .. sh - E + SL - 1 with sh = min(h * SL, 2E + 1 - SL) (the last
// lane may repeat rows of the one before it, which leaves the OR over rows
// unchanged); its slot i at column j compares reference position j with query
// position j + vb + i, vb = sh - E.  A column's "some row is free" is the OR
// over the group's lanes of each lane's own OR, so every lane keeps the same
// count (the thermometer Tm, as in SweepState).
// Bit-sliced counts in ND binary digits (digit d of count s is bit s of word d),
// each count at most S; ND is the bit width of S.
constexpr int count_digits(int S) { return S < 2 ? 1 : 1 + count_digits(S >> 1); }

// count == S (for a count <= S, the AND of the digits S has set)
template <int S, int ND>
__device__ __forceinline__ uint32_t sat_eq(const uint32_t (&c)[ND])
{
    uint32_t r = ~0u;
#pragma unroll
    for (int d = 0; d < ND; d++)
        if ((S >> d) & 1) r &= c[d];
    return r;
}

// count + 1 where inc is set (counts below S only: the caller masks inc)
template <int ND>
__device__ __forceinline__ void digits_inc(uint32_t (&c)[ND], uint32_t inc)
{
#pragma unroll
    for (int d = 0; d < ND; d++) {
        const uint32_t k = c[d] & inc;
        c[d] ^= inc;
        inc = k;
    }
}

// min(a + b, S) for counts a, b <= S
template <int S, int ND>
__device__ __forceinline__ void sat_add(uint32_t (&a)[ND], const uint32_t (&b)[ND])
{
    uint32_t sum[ND];
    uint32_t k = 0u;                      // carry into digit d
#pragma unroll
    for (int d = 0; d < ND; d++) {
        sum[d] = a[d] ^ b[d] ^ k;
        k = __builtin_amdgcn_bitop3_b32(a[d], b[d], k, 0xE8);   // majority
    }
    // ge: the (ND+1)-digit sum (k sum) >= S, from the low digit up
    uint32_t ge = ~0u;
#pragma unroll
    for (int d = 0; d < ND; d++) ge = ((S >> d) & 1) ? (sum[d] & ge) : (sum[d] | ge);
    ge |= k;
#pragma unroll
    for (int d = 0; d < ND; d++) a[d] = ((S >> d) & 1) ? (sum[d] | ge) : (sum[d] & ~ge);
}

template <int E, int LPG, int CPI, bool DB = false>
struct TileSweep {
    static constexpr int NR = 2 * E + 1;
    static constexpr int SL = (NR + LPG - 1) / LPG;
    static constexpr int B = kChunk;
    static constexpr int NC = B * CPI;        // columns per call
    static constexpr int NQ = SL + NC - 1;    // query words they read, per lane and plane
    static constexpr int EC = (E + B - 1) / B;
    // DB: instead of a thermometer updated by every lane at every column, each
    // column's OR word goes to dead[j] in LDS, and at the end the group's LPG
    // lanes count a share of the columns each (binary digits saturating at
    // E + 1) and add the shares up through DPP (finish)
    static_assert(!DB || LPG == 4, "counted words: four lanes per group");
    uint32_t S[SL];
    uint32_t Tm[DB ? 1 : E + 1];
    uint32_t* dead = nullptr;                 // DB: this group's column words

    __device__ __forceinline__ static int first_query(int h) { return min(h * SL, NR - SL) - E; }

    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int i = 0; i < SL; i++) S[i] = ~0u;
#pragma unroll
        for (int l = 0; l < (DB ? 1 : E + 1); l++) Tm[l] = 0u;
    }

    template <bool CHK>
    __device__ __forceinline__ void columns(const uint32_t (&w0)[NQ], const uint32_t (&w1)[NQ],
                                            const uint4 (&rr0)[CPI], const uint4 (&rr1)[CPI], int j0, int vb, int m)
    {
        // CHK: vm[x] = ~0 when window position x (query position j0 + vb + x) is in [0, m)
        uint32_t vm[CHK ? NQ : 1];
        if constexpr (CHK) {
#pragma unroll
            for (int x = 0; x < NQ; x++) vm[x] = (unsigned)(j0 + vb + x) < (unsigned)m ? ~0u : 0u;
        }
#pragma unroll
        for (int t = 0; t < NC; t++) {
            const int j = j0 + t;
            if (CHK && j >= m) break;
            const uint32_t r0 = comp(rr0[t / B], t % B), r1 = comp(rr1[t / B], t % B);
            uint32_t any = 0;
#pragma unroll
            for (int i = 0; i < SL; i++) {
                uint32_t a = and_xnor(and_xnor(S[i], r0, w0[t + i]), r1, w1[t + i]);
                if constexpr (CHK) a &= vm[t + i];
                S[i] = a;
                any |= a;
            }
            any = quad_or<LPG>(any);
            if constexpr (DB) {
                dead[j] = any;                // the group's lanes store the same word
            } else {
#pragma unroll
                for (int l = E; l >= 1; l--) Tm[l] = or_and_not(Tm[l], Tm[l - 1], any);
                Tm[0] = or_not(Tm[0], any);
            }
#pragma unroll
            for (int i = 0; i < SL; i++) S[i] = or_not(S[i], any);
        }
    }

    // decide and write (step 5) for group g after its last column; every lane of
    // the group calls it, lane 0 writes
    __device__ __forceinline__ void finish(int h, int m, int64_t g, int64_t n_pairs, uint16_t* __restrict__ out)
    {
        if constexpr (DB) {
            constexpr int SAT = E + 1;
            constexpr int ND = count_digits(SAT);
            tile::WaveSync()();               // the column words stored above, before they are read
            uint32_t c[ND];                   // count of columns with no row free, saturating at E + 1
#pragma unroll
            for (int d = 0; d < ND; d++) c[d] = 0u;
            const int q = (m + LPG - 1) / LPG;
            const int j1 = min(m, (h + 1) * q);
            for (int j = h * q; j < j1; j++) digits_inc<ND>(c, ~dead[j] & ~sat_eq<SAT, ND>(c));
            uint32_t o[ND];
#pragma unroll
            for (int d = 0; d < ND; d++) o[d] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c[d], 0xB1, 0xF, 0xF, false);
            sat_add<SAT, ND>(c, o);
#pragma unroll
            for (int d = 0; d < ND; d++) o[d] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c[d], 0x4E, 0xF, 0xF, false);
            sat_add<SAT, ND>(c, o);
            tile::WaveSync()();               // the reads above, before the group's next columns are stored
            if (h == 0) write_digits<ND>(c, ~sat_eq<SAT, ND>(c), g, n_pairs, out);
        } else {
            if (h == 0) write_group<E>(Tm, g, n_pairs, out);
        }
    }

    // the words of chunks c .. c+CPI-1: reference words (chunks past nch read the
    // last chunk; those columns are not run) and the lane's query window,
    // positions 4c + vb .. 4c + vb + NQ - 1.  Positions outside [0, m) are read
    // for rows that are masked: from at most E words before the group's planes
    // (the previous group, or the staging before the first buffer) to at most
    // 4 * CPI + E words past the end of a plane (still inside the group's planes)
    struct Words {
        uint4 rr0[CPI], rr1[CPI];
        uint32_t w0[NQ], w1[NQ];
    };
    __device__ __forceinline__ static void load(Words& W, const uint32_t* __restrict__ gp, int nch, int vb, int c)
    {
        const uint4* __restrict__ gp4 = reinterpret_cast<const uint4*>(gp);
#pragma unroll
        for (int k = 0; k < CPI; k++) {
            const int ck = min(c + k, nch - 1);
            W.rr0[k] = gp4[2 * nch + ck];
            W.rr1[k] = gp4[3 * nch + ck];
        }
        const uint32_t* __restrict__ q0 = gp + 4 * c + vb;
        const uint32_t* __restrict__ q1 = q0 + 4 * nch;
#pragma unroll
        for (int x = 0; x < NQ; x++) { W.w0[x] = q0[x]; W.w1[x] = q1[x]; }
    }

    // columns 4c .. 4c+NC-1 (those below m); interior: every row of every lane
    // reads a query position in [0, m) and every chunk is below nch
    __device__ __forceinline__ void compute(const Words& W, int m, int vb, int c, bool interior)
    {
        if (interior) columns<false>(W.w0, W.w1, W.rr0, W.rr1, 4 * c, vb, m);
        else columns<true>(W.w0, W.w1, W.rr0, W.rr1, 4 * c, vb, m);
    }

    __device__ __forceinline__ void chunks(const uint32_t* __restrict__ gp, int nch, int m, int vb, int c,
                                           bool interior)
    {
        Words W;
        load(W, gp, nch, vb, c);
        compute(W, m, vb, c, interior);
    }
};

// ---- synchronisation inside a fused block, through counters in LDS
enum { kCtrDone0 = 0, kCtrDone1 = 1, kCtrSwept = 2, kFusedCtrs = 4 };   // 16 bytes after the tile buffers
constexpr uint32_t kSpinLimit = 1u << 22;                           // ~0.1 s of polling

// wait until *p >= v (every lane reads the same word); a wait that outlives
// kSpinLimit polls ORs bit 1 into err and gives up, so that a broken count can
// not hang the device
__device__ __forceinline__ void wait_at_least(const uint32_t* p, uint32_t v, uint32_t* err)
{
    for (uint32_t k = 0; __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < v; k++) {
        if (k == kSpinLimit) {
            if (err && (threadIdx.x & 63) == 0) atomicOr(err, 2u);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// one count per wavefront, after its earlier LDS reads and writes have completed
__device__ __forceinline__ void arrive(uint32_t* p)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Fused encode and sweep.  Tiles of T consecutive groups are dealt to the
// blocks round-robin (persistent blocks).  Waves 0..2 encode tiles from the
// ASCII pairs (stored back to back, pair i at byte i*m) into two LDS tile
// buffers (group-major lane-sliced layout) in turn, while wave 3 sweeps the
// previous tile from the other buffer.  The packed encoding never reaches HBM.
// Two register buffers take turns in every encoding wave: the loads of its next
// groups are in flight while the current ones are encoded.
//
// Wave mode (WAVE, U > 0; pairs of up to a few hundred bases stored from 16-byte
// aligned bases): each encoding wave encodes units of U groups by itself, with
// staging of its own, so the encoders never wait for each other; wave w takes
// the block's units w, w+3, ... (T / U units per tile, in tile order).  They
// meet the sweeping wave through counters in LDS: per tile buffer, units
// encoded into it, and tiles swept.  The sweep of tile i waits until the
// buffer of tile i has counted all units of its tiles up to i; the encoding of
// a unit of tile i, which overwrites the buffer of tile i-2, waits for
// "swept > i-2"; so does a unit without groups (past the batch's last group),
// which encodes nothing but still counts.  (No unit of tile i+2 can count
// before tile i is swept, so the per-buffer count reaches tile i's target only
// when tile i is complete.)
// Every wait on a counter is bounded (see wait_at_least).
//
// Block mode (not WAVE): the three waves encode GB groups at a time together,
// passing four block barriers per GB groups, and the sweeping wave takes part in
// every one: while tile i is encoded (4 * steps(i) barriers) it sweeps tile
// i-1, its work cut into as many pieces as there are barriers, one piece
// before each.  Tile i-1's last words were written before the barrier that
// ends its encoding, and its buffer is written again only for tile i+1, after
// the barrier that ends tile i's encoding, by which the sweep has finished; the
// last tile is swept after the encoders are done, without barriers.
//
// LDS: the staging (wave mode: three regions of U * stage_dwords(m) dwords;
// block mode: GB * stage_dwords(m) dwords), two buffers of
// T * tile::fused_group_chunks(m) uint4, in wave mode the sweep's column words
// (tile::fused_dead_words(m)), then the counters.
template <int E, bool WAVE>
__global__ __launch_bounds__(256) void k_fused(const uint8_t* __restrict__ reads, const uint8_t* __restrict__ refs,
                                               int64_t n_pairs, int m, int T, int GB, int U, int fast,
                                               uint16_t* __restrict__ out, uint32_t* __restrict__ err)
{
    extern __shared__ uint32_t lds[];
    const int nch = (m + kChunk - 1) / kChunk;
    const int GS = tile::fused_group_chunks(m);
    const int64_t G = (n_pairs + 31) / 32;
    const int64_t ntiles = (G + T - 1) / T;
    const int wave_stage = WAVE ? (U * tile::stage_dwords(m) + 3) & ~3 : 0;
    const int stage_w = WAVE ? 3 * wave_stage : (GB * tile::stage_dwords(m) + 3) & ~3;
    uint4* __restrict__ buf0 = reinterpret_cast<uint4*>(lds + stage_w);
    uint32_t* __restrict__ deadbuf = reinterpret_cast<uint32_t*>(buf0 + 2 * (int64_t)T * GS);
    uint32_t* __restrict__ ctr = deadbuf + (WAVE ? tile::fused_dead_words(m) : 0);
    const int64_t t0 = blockIdx.x;
    if (t0 >= ntiles) return;
    const int64_t nmine = (ntiles - t0 + gridDim.x - 1) / gridDim.x;   // tiles of this block
    auto tile_of = [&](int64_t i) { return t0 + i * (int64_t)gridDim.x; };
    auto tile_groups = [&](int64_t t) { return (int)min<int64_t>(T, G - t * T); };
    auto steps_of = [&](int64_t i) { return (tile_groups(tile_of(i)) + GB - 1) / GB; };
    auto buffer = [&](int64_t i) { return buf0 + (i & 1) * (int64_t)T * GS; };
    if (threadIdx.x < kFusedCtrs) ctr[threadIdx.x] = 0u;
    __syncthreads();
    const int upt = WAVE ? T / U : 0;      // units per tile (wave mode)

    if (threadIdx.x < kFusedEnc) {
        uint32_t bad = 0;
        if constexpr (WAVE) {
            __builtin_assume(fast == 1 || fast == 2);     // wave mode is chosen only for the streaming loads
            const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
            uint32_t* __restrict__ stage = lds + w * wave_stage;
            const int64_t total = nmine * upt;
            // unit k: groups k % upt * U .. +U-1 of the block's tile k / upt (none past the batch)
            auto unit_groups = [&](int64_t k) -> int {
                if (k >= total) return 0;
                const int64_t i = k / upt;
                return min(U, tile_groups(tile_of(i)) - (int)(k - i * upt) * U);
            };
            auto unit_g0 = [&](int64_t k) {
                const int64_t i = k / upt;
                return tile_of(i) * T + (k - i * upt) * U;
            };
            int64_t k = w;
            auto step = [&](const uint4 (&cur)[2][tile::kWaveQ], uint4 (&nxt)[2][tile::kWaveQ]) -> bool {
                const int64_t kn = k + 3;
                tile::load_groups<tile::kWaveQ, 64>(reads, refs, n_pairs, m, unit_g0(kn), U,
                                                    fast && unit_groups(kn) > 0, nxt, lane);
                const int64_t i = k / upt;
                const int u = (int)(k - i * upt);
                // every unit of tile i >= 2 waits for the sweep of the buffer's previous tile, also one
                // without groups (past the batch's last group): it still counts toward the buffer's done
                // count, and counted early it could complete tile i - 2's target before that tile is
                // encoded (a CPU model of this schedule finds such interleavings)
                if (i >= 2) wait_at_least(ctr + kCtrSwept, (uint32_t)(i - 1), err);
                if (unit_groups(k) > 0) {
                    tile::encode_groups<tile::kWaveQ, 64>(reads, refs, nullptr, nullptr, n_pairs, m, unit_g0(k), U,
                                                          fast, cur, stage, buffer(i), 1, u * U, bad, GS,
                                                          tile::WaveSync(), lane);
                }
                arrive(ctr + kCtrDone0 + (i & 1));
                k = kn;
                return k < total;
            };
            if (k < total) {
                uint4 va[2][tile::kWaveQ], vb[2][tile::kWaveQ];
                tile::load_groups<tile::kWaveQ, 64>(reads, refs, n_pairs, m, unit_g0(k), U,
                                                    fast && unit_groups(k) > 0, va, lane);
                for (;;) {
                    if (!step(va, vb)) break;
                    if (!step(vb, va)) break;
                }
            }
        } else {
            int64_t i = 0;               // tile index (of this block) and step in it
            int s = 0;
            // one step: encode the current GB groups from cur while the next groups'
            // loads (possibly of the block's next tile) run; false when the block is done
            auto step = [&](const uint4 (&cur)[2][kFusedEncQ], uint4 (&nxt)[2][kFusedEncQ]) -> bool {
                int64_t in = i;
                int sn = s + 1;
                if (sn >= steps_of(i)) { sn = 0; in++; }
                tile::load_groups<kFusedEncQ, kFusedEnc>(reads, refs, n_pairs, m, tile_of(in) * T + sn * GB, GB,
                                                         fast && in < nmine, nxt);
                tile::encode_groups<kFusedEncQ, kFusedEnc>(reads, refs, nullptr, nullptr, n_pairs, m,
                                                           tile_of(i) * T + s * GB, GB, fast, cur, lds, buffer(i), 1,
                                                           s * GB, bad, GS);
                i = in;
                s = sn;
                return i < nmine;
            };
            uint4 va[2][kFusedEncQ], vb[2][kFusedEncQ];
            tile::load_groups<kFusedEncQ, kFusedEnc>(reads, refs, n_pairs, m, t0 * T, GB, fast != 0, va);
            for (;;) {
                if (!step(va, vb)) break;
                if (!step(vb, va)) break;
            }
        }
        if (tile::invalid(bad) && err) atomicOr(err, 1u);
    } else {
        constexpr int LPG = fused_lanes(E);
        constexpr int GPP = 64 / LPG;                    // groups per pass of the wave
        constexpr int CPI = kFusedCPI;                   // chunks per call
        constexpr bool DB = WAVE && E >= 3;              // column words counted at the end (wave mode)
        using SW = TileSweep<E, LPG, CPI, DB>;
        const int lane = threadIdx.x - kFusedEnc;
        const int h = lane % LPG, gq = lane / LPG;
        const int vb = SW::first_query(h);
        const int ct = (m - kChunk - E >= 0) ? (m - kChunk - E) / kChunk + 1 : 0;   // interior chunks [EC, ct)
        SW sw;
        // the sweep of group gl of tile tp from buffer tb, chunks c .. c+CPI-1
        if constexpr (DB) sw.dead = deadbuf + gq * (m | 1);
        auto sweep_item = [&](const uint32_t* __restrict__ tb, int64_t tp, int gl, int c) {
            if (c == 0) sw.init();
            if (c < nch)
                sw.chunks(tb + (int64_t)gl * GS * 4, nch, m, vb, c, c >= SW::EC && c + CPI <= ct);
            if (c + CPI >= nch) sw.finish(h, m, tp * T + gl, n_pairs, out);
        };
        if constexpr (WAVE) {
            for (int64_t i = 0; i < nmine; i++) {
                wait_at_least(ctr + kCtrDone0 + (i & 1), (uint32_t)(upt * (i / 2 + 1)), err);
                const int64_t tp = tile_of(i);
                const int tg = tile_groups(tp);
                const uint32_t* __restrict__ tb = reinterpret_cast<const uint32_t*>(buffer(i));
                for (int g0 = 0; g0 < tg; g0 += GPP) {
                    const int gl = g0 + gq;
                    if (gl < tg) {
                        // the next item's words are loaded while this item's columns run
                        const uint32_t* __restrict__ gp = tb + (int64_t)gl * GS * 4;
                        auto inner = [&](int c) { return c >= SW::EC && c + CPI <= ct; };
                        sw.init();
                        if (nch > 0) {
                            typename SW::Words wa, wb;
                            SW::load(wa, gp, nch, vb, 0);
                            for (int c = 0;; c += 2 * CPI) {
                                if (c + CPI < nch) SW::load(wb, gp, nch, vb, c + CPI);
                                sw.compute(wa, m, vb, c, inner(c));
                                if (c + CPI >= nch) break;
                                if (c + 2 * CPI < nch) SW::load(wa, gp, nch, vb, c + 2 * CPI);
                                sw.compute(wb, m, vb, c + CPI, inner(c + CPI));
                                if (c + 2 * CPI >= nch) break;
                            }
                        }
                        sw.finish(h, m, tp * T + gl, n_pairs, out);
                    }
                }
                arrive(ctr + kCtrSwept);
            }
        } else {
            const int nci = nch > 0 ? (nch + CPI - 1) / CPI : 1;    // items per group (m = 0: the write alone)
            for (int64_t i = 0; i <= nmine; i++) {
                const int nint = i < nmine ? 4 * steps_of(i) : 0;     // barriers of tile i's encoding
                if (i == 0) {
                    for (int b = 0; b < nint; b++) __syncthreads();
                    continue;
                }
                const int64_t tp = tile_of(i - 1);
                const int tg = tile_groups(tp);
                const uint32_t* __restrict__ tb = reinterpret_cast<const uint32_t*>(buffer(i - 1));
                const int work = ((tg + GPP - 1) / GPP) * nci;       // (pass, item) pairs
                int it = 0, pass = 0, c = 0;
                const int npiece = nint > 0 ? nint : 1;
                for (int b = 0; b < npiece; b++) {
                    // equal pieces (weighting them towards either phase of the encoding measured slower)
                    const int end = nint > 0 ? (int)((int64_t)work * (b + 1) / nint) : work;
                    for (; it < end; it++) {
                        const int gl = pass * GPP + gq;
                        if (gl < tg) sweep_item(tb, tp, gl, c * CPI);
                        if (++c == nci) { c = 0; pass++; }
                    }
                    if (nint > 0) __syncthreads();
                }
            }
        }
    }
}

template <int E, bool WAVE>
hipError_t launch_fused_mode(const uint8_t* reads, const uint8_t* refs, int64_t n_pairs, int32_t m, int T, int GB,
                             int U, int fast, size_t shmem, uint16_t* out, uint32_t* err, hipStream_t s)
{
    const int64_t G = cdiv(n_pairs, 32);
    const void* fn = reinterpret_cast<const void*>(&k_fused<E, WAVE>);
    if (shmem > 65536) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    // persistent blocks: as many as are resident at once (LDS and registers), at most one per tile
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, shmem);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const int64_t grid = std::min<int64_t>(cdiv(G, T), (int64_t)std::max(1, per_cu) * cus);
    hipLaunchKernelGGL((k_fused<E, WAVE>), dim3((unsigned)grid), dim3(256), shmem, s, reads, refs, n_pairs, m, T,
                       GB, U, fast, out, err);
    return hipGetLastError();
}

template <int E>
hipError_t launch_fused_E(const uint8_t* reads, const uint8_t* refs, int64_t n_pairs, int32_t m, int T, int GB,
                          int U, int fast, size_t shmem, uint16_t* out, uint32_t* err, hipStream_t s)
{
    return U > 0 ? launch_fused_mode<E, true>(reads, refs, n_pairs, m, T, GB, U, fast, shmem, out, err, s)
                 : launch_fused_mode<E, false>(reads, refs, n_pairs, m, T, GB, U, fast, shmem, out, err, s);
}

template <int... Es>
struct FusedTable {
    static hipError_t run(int E, const uint8_t* reads, const uint8_t* refs, int64_t n, int32_t m, int T, int GB,
                          int U, int fast, size_t shmem, uint16_t* out, uint32_t* err, hipStream_t s)
    {
        hipError_t r = hipErrorInvalidValue;
        ((E == Es ? (r = launch_fused_E<Es>(reads, refs, n, m, T, GB, U, fast, shmem, out, err, s), 0) : 0), ...);
        return r;
    }
};

}  // namespace sliced
}  // namespace ss
