// The device-resident serving loop (layouts and protocol in ss_loop.h).
//
// Block 0, wavefront 0 schedules: lane s polls the publication word of slot s
// in host memory; a new generation is activated by copying its descriptor into
// the device slot table, resetting the slot's counters and publishing its claim
// counters.  Every other block is a worker: its first wavefront picks, among
// the active slots with a unit left to claim, the one admitted first (slots
// with encoding units left before slots with only items left), and
// claims a unit with a fetch-and-add on the slot's counter (ss_loop.h: a
// compare-and-swap would fail for all but one of the blocks that aim at the
// same slot); the whole block then runs it.  An encoding unit turns 1,024
// words of each of the four planes into bits (the same per-word encoder as the
// stream layout's kernel); an item is swept exactly as the batched persistent
// kernel sweeps it.  A request's items can be claimed only once the block that
// finishes its last encoding unit has opened its item counter.
//
// Ordering: the scheduler's writes of a slot happen before its counters are
// published (release); a worker acquires after its claim.  Encoding units
// release before counting themselves done, and the block that counts the last
// one opens the item counter with a release; items acquire after their claim.  Items release their result words to system scope
// before counting themselves done; the block that counts the last one writes
// the completion word with a system-scope release.
//
// Exit: every wait here ends.  The scheduler returns once no request has been
// active or new for idle_ticks (or once host->stop is set and nothing is
// active), or when requests are active but no unit has finished for
// stall_ticks (then it also sets host->stalled), and raises the launch's quit
// epoch.  A worker returns when it finds no unit to claim and sees that epoch,
// or, should the scheduler have gone, when no slot is active and the
// scheduler's heartbeat (and the worker's own start) are older than four idle
// periods and an eighth of the stall limit.  A claimed unit is always run to
// its end before its block looks again.
#include <hip/hip_runtime.h>

#include "ss_items.h"
#include "ss_loop.h"
#include "ss_pack_ops.h"

namespace ss {
namespace loop {
namespace {

__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_system(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void scheduler(Host* __restrict__ H, Dev* __restrict__ D, uint32_t epoch,
                                          uint64_t idle_ticks, uint64_t stall_ticks)
{
    const int s = (int)threadIdx.x;          // one lane per slot
    uint64_t seen = D->seen[s];
    uint64_t t_busy = wall_clock64(), t_prog = t_busy;
    uint32_t last_prog = ld_agent32(&D->progress);
    for (;;) {
        const uint64_t pub = ld_system(&H->pub[s]);
        const bool fresh = pub != seen;
        if (fresh) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");      // the descriptor was written before pub
            Slot* S = &D->slot[s];
            S->d = H->desc[s];
            S->pack_done = 0;
            S->item_done = 0;
            S->err = 0;
            S->gen = pub;
            S->adm = atomicAdd((unsigned long long*)&D->adm_next, 1ull);
            H->t_act[s] = wall_clock64();
            // items closed until the planes are complete; then the encoding units go public
            __hip_atomic_store(&S->item_ctr, make_ctr(pub, 0u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&S->pack_ctr, make_ctr(pub, (uint32_t)S->d.n_pack), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            atomicOr((unsigned long long*)&D->active, 1ull << s);
            seen = pub;
            D->seen[s] = seen;
        }
        const bool any_fresh = __ballot(fresh) != 0;
        const uint64_t act = ld_agent(&D->active);
        const uint32_t prog = ld_agent32(&D->progress);
        const uint64_t now = wall_clock64();
        if (s == 0) __hip_atomic_store(&D->beat, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (any_fresh || act == 0 || prog != last_prog) {
            t_prog = now;
            last_prog = prog;
        }
        if (any_fresh || act != 0) {
            t_busy = now;
            if (now - t_prog > stall_ticks) {
                // requests are active but nothing has finished for stall_ticks: end the launch and
                // say so (the host fails the requests in flight)
                if (s == 0) __hip_atomic_store(&H->stalled, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&D->quit, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        } else if (ld_system(&H->stop) != 0 || now - t_busy > idle_ticks) {
            __hip_atomic_store(&D->quit, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

enum Op { OP_NONE = 0, OP_PACK = 1, OP_ITEM = 2, OP_EXIT = 3, OP_RETRY = 4 };   // RETRY: a claim past the count

template <int RSMAX>
__device__ __forceinline__ void worker(Host* __restrict__ H, Dev* __restrict__ D, uint32_t epoch, uint64_t idle_ticks,
                                       uint64_t stall_ticks)
{
    __shared__ int s_op, s_slot, s_unit;
    __shared__ PItem s_item;
    __shared__ long long s_lo[4], s_hi[4];
    __shared__ uint32_t s_stage[4 * item_sweep::kStageWords];
    const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const uint64_t t_start = wall_clock64();
    for (;;) {
        if (wv == 0) {
            // lane s looks at slot s
            const uint64_t act = ld_agent(&D->active);
            bool cand = false;
            int kind = OP_NONE;
            uint64_t key = ~0ull;
            if ((act >> lane) & 1ull) {
                Slot* S = &D->slot[lane];
                const uint64_t pc = ld_agent(&S->pack_ctr);
                const uint64_t ic = ld_agent(&S->item_ctr);
                if (ctr_next(pc) < ctr_count(pc)) {
                    cand = true;
                    kind = OP_PACK;
                } else if (ctr_next(ic) < ctr_count(ic)) {
                    cand = true;
                    kind = OP_ITEM;
                }
                // encoding units first (they are short and open a request's items), then admission order
                key = ((kind == OP_ITEM ? 1ull : 0ull) << 62) | S->adm;
            }
            uint64_t best = cand ? key : ~0ull;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const uint64_t other = __shfl_xor(best, o);
                best = other < best ? other : best;
            }
            int op = OP_NONE, slot = -1, unit = 0;
            if (best != ~0ull) {
                const uint64_t win = __ballot(cand && key == best);
                const int L = __ffsll((unsigned long long)win) - 1;
                if (lane == L) {
                    uint64_t* c = kind == OP_PACK ? &D->slot[lane].pack_ctr : &D->slot[lane].item_ctr;
                    const uint64_t got = atomicAdd((unsigned long long*)c, 1ull);
                    op = ctr_next(got) < ctr_count(got) ? kind : OP_RETRY;
                    slot = lane;
                    unit = (int)ctr_next(got);
                }
                op = __shfl(op, L);
                slot = __shfl(slot, L);
                unit = __shfl(unit, L);
            } else if (__hip_atomic_load(&D->quit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
                op = OP_EXIT;
            } else if (act == 0) {
                // no scheduler left to activate anything (its heartbeat, and this worker's start, are
                // old).  Looked at only while no slot is active: the heartbeat's line is rewritten on
                // every scheduler pass, and reading it on every poll while requests are in flight
                // doubled their device time.
                const uint64_t beat = ld_agent(&D->beat);
                const uint64_t last = beat > t_start ? beat : t_start;
                const uint64_t orphan = 4 * idle_ticks > stall_ticks / 8 ? 4 * idle_ticks : stall_ticks / 8;
                if (wall_clock64() - last > orphan) op = OP_EXIT;
            }
            if (lane == 0) {
                s_op = op;
                s_slot = slot;
                s_unit = unit;
            }
        }
        __syncthreads();
        const int op = __builtin_amdgcn_readfirstlane(s_op);
        const int slot = __builtin_amdgcn_readfirstlane(s_slot);
        const int unit = __builtin_amdgcn_readfirstlane(s_unit);
        __syncthreads();
        if (op == OP_EXIT) return;
        if (op == OP_NONE) {
            __builtin_amdgcn_s_sleep(8);
            continue;
        }
        if (op == OP_RETRY) continue;
        Slot* S = &D->slot[slot];
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");     // the slot's descriptor (and planes for items)
        if (op == OP_PACK) {
            const uint8_t* reads = S->d.reads;
            const uint8_t* refs = S->d.refs;
            const int64_t total = S->d.total, SW = S->d.SW;
            const int aligned = S->d.aligned;
            uint32_t* packed = S->d.packed;
            uint32_t bad = 0;
#pragma unroll
            for (int k = 0; k < kPackWords / 256; k++) {
                const int64_t w = (int64_t)unit * kPackWords + k * 256 + threadIdx.x;
                if (w < SW) bad |= stream_pack::pack_word<true>(reads, refs, total, SW, aligned, packed, w);
            }
            if (bad) atomicOr(&S->err, 1u);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0) {
                const uint32_t done =
                    __hip_atomic_fetch_add(&S->pack_done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
                if (done == (uint32_t)S->d.n_pack) {
                    // the planes are complete: open the items
                    H->t_packed[slot] = wall_clock64();
                    __hip_atomic_store(&S->item_ctr, make_ctr(S->gen, (uint32_t)S->d.n_items), __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
                atomicAdd(&D->progress, 1u);
            }
        } else {
            if (threadIdx.x == 0) s_item = S->d.items[unit];
            __syncthreads();
            const int64_t first = s_item.first;
            const int count = __builtin_amdgcn_readfirstlane(s_item.count);
            const int LP = __builtin_amdgcn_readfirstlane(s_item.lp);
            const int rs = __builtin_amdgcn_readfirstlane(s_item.rs);
            const int emax = __builtin_amdgcn_readfirstlane(s_item.emax);
            const wave::GlobalPlanes planes = wave::GlobalPlanes::four(S->d.packed, S->d.SW);
            item_sweep::sweep_item<RSMAX>(first, count, LP, rs, emax, S->d.perm, planes, S->d.offsets,
                                          S->d.lengths, S->d.E, S->d.results, s_lo, s_hi, s_stage);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");      // result words reach host memory first
            __syncthreads();
            if (threadIdx.x == 0) {
                const uint32_t done =
                    __hip_atomic_fetch_add(&S->item_done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM) + 1u;
                if (done == (uint32_t)S->d.n_items) {
                    // the request's last item: report it
                    const uint64_t gen = S->gen;
                    H->err[slot] = ld_agent32(&S->err);
                    H->t_done[slot] = wall_clock64();
                    atomicAnd((unsigned long long*)&D->active, ~(1ull << slot));
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                    __hip_atomic_store(&H->fin[slot], gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                atomicAdd(&D->progress, 1u);
            }
        }
        __syncthreads();
    }
}

template <int RSMAX>
__global__ __launch_bounds__(256) void k_loop(Host* __restrict__ H, Dev* __restrict__ D, uint32_t epoch,
                                              uint64_t idle_ticks, uint64_t stall_ticks)
{
    if (blockIdx.x == 0) {
        // the scheduler is one wavefront; the block's other wavefronts have nothing to do
        if (threadIdx.x < 64) scheduler(H, D, epoch, idle_ticks, stall_ticks);
        return;
    }
    worker<RSMAX>(H, D, epoch, idle_ticks, stall_ticks);
}

}  // namespace

hipError_t launch_loop(int rsmax, int grid, size_t lds_pad, Host* host, Dev* dev, uint32_t epoch,
                       uint64_t idle_ticks, uint64_t stall_ticks, hipStream_t s)
{
    if (grid < 2) grid = 2;
    const void* fn = rsmax == 1   ? (const void*)k_loop<1>
                     : rsmax == 2 ? (const void*)k_loop<2>
                     : rsmax == 4 ? (const void*)k_loop<4>
                                  : (const void*)k_loop<8>;
    if (lds_pad > 0) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_pad);
        if (e != hipSuccess) return e;
    }
    switch (rsmax) {
    case 1: hipLaunchKernelGGL(k_loop<1>, dim3(grid), dim3(256), lds_pad, s, host, dev, epoch, idle_ticks,
                                   stall_ticks); break;
    case 2: hipLaunchKernelGGL(k_loop<2>, dim3(grid), dim3(256), lds_pad, s, host, dev, epoch, idle_ticks,
                                   stall_ticks); break;
    case 4: hipLaunchKernelGGL(k_loop<4>, dim3(grid), dim3(256), lds_pad, s, host, dev, epoch, idle_ticks,
                                   stall_ticks); break;
    default: hipLaunchKernelGGL(k_loop<8>, dim3(grid), dim3(256), lds_pad, s, host, dev, epoch, idle_ticks,
                                   stall_ticks); break;
    }
    return hipGetLastError();
}

size_t loop_static_lds(int rsmax)
{
    hipFuncAttributes a;
    const void* fn = rsmax == 1   ? (const void*)k_loop<1>
                     : rsmax == 2 ? (const void*)k_loop<2>
                     : rsmax == 4 ? (const void*)k_loop<4>
                                  : (const void*)k_loop<8>;
    if (hipFuncGetAttributes(&a, fn) != hipSuccess) return 0;
    return a.sharedSizeBytes;
}

}  // namespace loop
}  // namespace ss
