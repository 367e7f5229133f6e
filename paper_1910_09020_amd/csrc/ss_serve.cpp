// Serving loop: continuous batching of filter requests on one device.
//
// A request is a batch of pairs (ASCII, lengths, per-pair thresholds) with host
// output arrays.  The server owns a fixed number of slots, each with its own
// HIP stream.  Admission is by HBM budget: the device footprints of the
// requests in flight never total more than the budget given at creation; a
// request that does not fit waits in a FIFO queue until slots and memory free
// up.  Device memory comes from the stream-ordered pool (hipMallocAsync on the
// slot's stream, hipFreeAsync after the last copy), kept resident between
// requests, so dispatching never synchronises the device.  Inputs are staged
// in pooled pinned blocks at submission.  An admitted request is enqueued on
// its slot's stream: copies in, bit-stream encoding, a per-request plan of the
// batched launch (ss_batch.hip), the persistent filter kernel, copies out.
// Requests in different slots run concurrently on the device, and requests
// that arrive while others are running are admitted as soon as a slot and
// memory are free.  A completion thread polls the slots' events, writes the
// results to the caller's arrays and timestamps the completion.
//
// Device-resident mode (ss_server_create_loop): the same queue and admission,
// but an admitted request is handed to the persistent loop kernel of
// ss_loop.hip instead of being enqueued on a stream: the dispatcher writes its
// descriptor into a slot of a control block in coherent host memory and
// publishes it, the kernel encodes the request's ASCII straight from the
// staging block and sweeps its plan, writes the result words into the staging
// block and marks the slot finished, and the completion thread polls those
// marks.  No HIP call is made per request; the kernel is launched again when
// it has ended after an idle period and a request is waiting.  Its device
// memory is one arena of the budget's size, reserved at creation, from which
// each request takes the room of its bit planes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ss.h"
#include "ss_common.h"
#include "ss_arena.h"
#include "ss_copy.h"
#include "ss_loop.h"
#include "ss_trace.h"

using namespace ss;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int map_err(hipError_t e)
{
    if (e == hipSuccess) return SS_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SS_ENOMEM;
    return SS_EDEVICE;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of one request's buffers inside a slot arena.
struct Layout {
    size_t reads, refs, packed, offsets, lengths, E, items, perm, head, results, err, total;
    size_t in_bytes;     // staged host -> device (reads .. perm)
    int64_t SW;
    Layout(int64_t n, int64_t T, int64_t n_items)
    {
        SW = cdiv(T, 32) + 2;
        size_t o = 0;
        reads = o; o += al((size_t)T + 16);
        refs = o; o += al((size_t)T + 16);
        offsets = o; o += al((size_t)n * 8);
        lengths = o; o += al((size_t)n * 4);
        E = o; o += al((size_t)n * 4);
        items = o; o += al((size_t)n_items * sizeof(PItem));
        perm = o; o += al((size_t)n * 8);
        in_bytes = o;
        packed = o; o += al((size_t)SW * 16);
        head = o; o += 256;
        results = o; o += al((size_t)n * 2);
        err = o; o += 256;
        total = o;
    }
};

enum State { QUEUED = 0, RUNNING = 1, DONE = 2, CANCELLED = 3 };

struct Request {
    uint64_t id = 0;
    int64_t n = 0, total = 0;
    int64_t n_items = 0;
    int rsmax = 2;                 // slice width the plan was made for
    // staging in the device layout (inputs, then results and the error word):
    // a pooled pinned block when available, else pageable memory copied into
    // the slot's pinned buffer at launch
    void* pin = nullptr;
    size_t pin_cls = 0;
    std::vector<uint8_t> page;
    // a staged submission (ss_server_submit_staged): the bases stay in the caller's block of the
    // server's staging (reads at its start, refs at owned_refs), which returns to the pool when the
    // request is done; the staging above then holds only the per-pair arrays
    uint8_t* owned = nullptr;
    size_t owned_cls = 0, owned_refs = 0;
    uint8_t* stage = nullptr;      // where results come back (set at launch)
    uint8_t* accept_out = nullptr;
    int32_t* edits_out = nullptr;
    size_t footprint = 0;
    size_t arena_off = 0;          // device-resident mode: offset of the request's planes in the arena
    uint64_t gen = 0;              // device-resident mode: the generation it was published under
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    // stages: host time to enqueue the request's work, and the device spans between the slot's
    // timing events (copy in, encode + filter, copy out), in nanoseconds
    int64_t ns_enqueue = 0, ns_h2d = 0, ns_compute = 0, ns_d2h = 0;
    int status = SS_OK;
    State state = QUEUED;
    int slot = -1;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // timing: before the copy in, after it,
                                                               // after the kernel, after the copy out
    void* arena = nullptr;           // the running request's device memory (stream-ordered)
    size_t arena_cap = 0;
    void* pinned = nullptr;
    size_t pinned_cap = 0;
    Request* cur = nullptr;
    bool launched = false;     // cur's work (and the completion event) is enqueued
};

}  // namespace

// Pinned host blocks in power-of-two size classes, reused across requests.
struct PinnedPool {
    std::mutex mu;
    std::unordered_map<size_t, std::vector<void*>> free_blocks;
    size_t total = 0;
    size_t cap = (size_t)4 << 30;
    unsigned flags = hipHostMallocDefault;     // coherent in device-resident mode (the kernel reads it)
    // One region pinned (and written) when the server is created, handed out first fit in 4 KiB
    // steps: a block pinned when a request first needed its size class cost that request 1.3 ms
    // (2 MB), 2.2 ms (13 MB) or 11 ms (82 MB) in its submission, against 0.05-1.4 ms warm.  Blocks of
    // power-of-two classes, pinned on demand and kept, take what the region cannot hold.
    uint8_t* region = nullptr;
    size_t region_bytes = 0;
    Arena region_free;
    void reserve(size_t bytes)
    {
        void* p = nullptr;
        if (bytes == 0 || hipHostMalloc(&p, bytes, flags) != hipSuccess) return;   // then blocks only
        // written once here: the first write of a page of this memory is slow (a submission into
        // never-written staging measured 0.9 ms more for 2 MB and 7 ms more for 82 MB)
        std::memset(p, 0, bytes);
        std::lock_guard<std::mutex> lk(mu);
        region = (uint8_t*)p;
        region_bytes = bytes;
        region_free.reset(bytes);
    }
    void* get(size_t need, size_t* cls)
    {
        if (need == 0 || need > cap) return nullptr;     // (also keeps the class doubling below from overflowing)
        {
            std::lock_guard<std::mutex> lk(mu);
            const size_t r = std::max<size_t>(4096, (need + 4095) & ~(size_t)4095);
            size_t off = 0;
            if (region && region_free.alloc(r, &off)) {
                *cls = r;
                return region + off;
            }
        }
        size_t c = (size_t)1 << 20;
        while (c < need) c <<= 1;
        *cls = c;
        {
            std::lock_guard<std::mutex> lk(mu);
            auto& v = free_blocks[c];
            if (!v.empty()) {
                void* p = v.back();
                v.pop_back();
                return p;
            }
            if (total + c > cap) return nullptr;
            total += c;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, c, flags) != hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            total -= c;
            return nullptr;
        }
        return p;
    }
    void put(void* p, size_t cls)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu);
        uint8_t* q = (uint8_t*)p;
        if (region && q >= region && q < region + region_bytes) {
            region_free.release((size_t)(q - region), cls);
            return;
        }
        free_blocks[cls].push_back(p);
    }
    void release_all()
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& kv : free_blocks)
            for (void* p : kv.second) (void)hipHostFree(p);
        free_blocks.clear();
        total = 0;
        if (region) (void)hipHostFree(region);
        region = nullptr;
        region_bytes = 0;
        region_free.reset(0);
    }
};

// Bytes of the staging region pinned at creation: a request's staging is about four times its room
// in the device budget (ASCII of both sides and per-pair arrays against 2-bit planes).
static size_t staging_region_bytes(size_t hbm_budget_bytes)
{
    const size_t lo = (size_t)16 << 20, hi = (size_t)512 << 20;
    const size_t four = hbm_budget_bytes > hi / 4 ? hi : 4 * hbm_budget_bytes;   // 4 x budget, at most hi
    return std::max(lo, four);
}

struct ss_server {
    ss_ctx* ctx = nullptr;
    PinnedPool pool;
    CopyCrew copier{3};              // submissions stage large requests' bases with three helpers
    std::mutex blocks_mu;            // blocks of the staging handed to callers (ss_server_stage_alloc):
    std::unordered_map<void*, std::pair<size_t, size_t>> blocks;    // block -> (pool class, bytes)
    int device = 0;
    size_t budget = 0;
    size_t used = 0;                 // sum of the footprints of requests in flight
    int rsmax = 1;                   // slices per lane for new requests
    int grid_cap[9] = {0};
    std::vector<Slot> slots;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> reqs;
    uint64_t next_id = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread dispatcher, completer;
    bool stop = false;
    bool hold = false;
    bool broken = false;             // device-resident mode: the loop kernel could not run; submissions fail
    int running = 0;
    // statistics
    int64_t admitted = 0, deferred = 0, completed = 0, peak_used = 0, peak_running = 0;
    // device-resident mode
    bool loop = false;
    int loop_rs = 1;                 // slice width the loop kernel is built for
    int loop_grid = 0;
    size_t loop_lds_pad = 0;
    loop::Host* H = nullptr;         // control block (coherent host memory)
    loop::Host* H_dev = nullptr;     // the same as the kernel addresses it
    loop::Dev* D = nullptr;          // device-side slot table
    uint8_t* arena = nullptr;
    Arena arena_alloc;               // guarded by mu
    uint64_t gen[loop::kSlots] = {};
    std::mutex loop_mu;              // guards the kernel's launch state
    hipStream_t loop_stream = nullptr;
    hipEvent_t loop_ev = nullptr;
    bool loop_launched = false;
    uint32_t epoch = 0;
    uint64_t idle_ticks = 0;
    uint64_t stall_ticks = 0;        // no unit finished for this long with requests active: the loop gave up
    uint64_t khz = 100000;           // device clock rate
    double tick_ns = 10.0;
    int64_t loop_launches = 0;
};

namespace {

size_t footprint_of(int64_t n, int64_t T)
{
    // items <= n (one pair per item at worst)
    return Layout(n, T, n).total;
}

// Bytes of a request's staging: the device layout's inputs, results, error word.
size_t stage_bytes(const Layout& L, int64_t n) { return L.in_bytes + al((size_t)n * 2) + 256; }
// Layout of a request's host staging: the device layout, or for a staged submission the same
// per-pair arrays without the bases (which stay in the caller's block)
Layout stage_layout(const Request* r) { return Layout(r->n, r->owned ? 0 : r->total, r->n_items); }

// Device-resident mode: a request's device memory is its four bit planes.
size_t loop_footprint(int64_t T) { return al((size_t)(cdiv(T, 32) + 2) * 16); }

// Device-resident mode: make sure a loop kernel is running (launch one when the
// last has ended).  Returns SS_EDEVICE when the last launch failed.
int ensure_loop(ss_server* S)
{
    std::lock_guard<std::mutex> lk(S->loop_mu);
    if (S->loop_launched) {
        const hipError_t q = hipEventQuery(S->loop_ev);
        if (q == hipErrorNotReady) return SS_OK;
        S->loop_launched = false;
        if (q != hipSuccess) return map_err(q);
    }
    if (__atomic_load_n(&S->H->stalled, __ATOMIC_ACQUIRE) != 0) return SS_EDEVICE;
    S->epoch++;
    roctxMarkA("serve: launch the loop kernel");
    hipError_t e = loop::launch_loop(S->loop_rs, S->loop_grid, S->loop_lds_pad, S->H_dev, S->D, S->epoch,
                                     S->idle_ticks, S->stall_ticks, S->loop_stream);
    if (e == hipSuccess) e = hipEventRecord(S->loop_ev, S->loop_stream);
    if (e != hipSuccess) return map_err(e);
    S->loop_launched = true;
    S->loop_launches++;
    return SS_OK;
}

// Device-resident mode: publish the request in its slot.  Called without the lock.
int launch_request_loop(ss_server* S, Slot& sl, int si, Request* r)
{
    TraceRange tr("serve: publish request to the loop");
    const Layout L = stage_layout(r);
    uint8_t* h = (uint8_t*)r->pin;
    if (!h) {
        const size_t need = stage_bytes(L, r->n);
        if (sl.pinned_cap < need) {
            if (sl.pinned) (void)hipHostFree(sl.pinned);
            sl.pinned = nullptr;
            sl.pinned_cap = 0;
            const size_t want = std::max(need, (size_t)1 << 20);
            hipError_t e = hipHostMalloc(&sl.pinned, want, hipHostMallocCoherent | hipHostMallocMapped);
            if (e != hipSuccess) return map_err(e);
            sl.pinned_cap = want;
        }
        h = (uint8_t*)sl.pinned;
        std::memcpy(h, r->page.data(), L.in_bytes);
    }
    r->stage = h;
    const int64_t t0 = now_ns();
    uint8_t* hd = nullptr;
    hipError_t e = hipHostGetDevicePointer((void**)&hd, h, 0);
    if (e != hipSuccess) return map_err(e);
    loop::Desc& d = S->H->desc[si];
    if (r->owned) {
        // staged: the kernel reads the bases from the caller's block
        uint8_t* od = nullptr;
        e = hipHostGetDevicePointer((void**)&od, r->owned, 0);
        if (e != hipSuccess) return map_err(e);
        d.reads = od;
        d.refs = od + r->owned_refs;
    } else {
        d.reads = hd + L.reads;
        d.refs = hd + L.refs;
    }
    d.offsets = (const int64_t*)(hd + L.offsets);
    d.lengths = (const int32_t*)(hd + L.lengths);
    d.E = (const int32_t*)(hd + L.E);
    d.items = (const PItem*)(hd + L.items);
    d.perm = (const int64_t*)(hd + L.perm);
    d.results = (uint16_t*)(hd + L.in_bytes);
    d.packed = (uint32_t*)(S->arena + r->arena_off);
    d.total = r->total;
    d.SW = cdiv(r->total, 32) + 2;
    d.n_items = (int32_t)r->n_items;
    d.n_pack = (int32_t)cdiv(d.SW, loop::kPackWords);
    d.aligned = ((((uintptr_t)d.reads) | ((uintptr_t)d.refs)) & 15u) == 0;
    d.pad = 0;
    r->gen = ++S->gen[si];
    // the descriptor is complete before the publication word changes
    __atomic_store_n(&S->H->pub[si], r->gen, __ATOMIC_RELEASE);
    const int rc = ensure_loop(S);
    r->ns_enqueue = now_ns() - t0;
    return rc;
}

// Enqueue the whole request on its slot's stream.  Called without the lock.
int launch_request(ss_server* S, Slot& sl, Request* r)
{
    TraceRange tr("serve: enqueue request on its slot stream");
    const Layout L(r->n, r->total, r->n_items);      // on the device
    const Layout Ls = stage_layout(r);                // in the host staging
    uint8_t* h = (uint8_t*)r->pin;
    if (!h) {
        // pageable staging: copy into the slot's own pinned buffer first
        const size_t need = stage_bytes(Ls, r->n);
        if (sl.pinned_cap < need) {
            if (sl.pinned) (void)hipHostFree(sl.pinned);
            sl.pinned = nullptr;
            sl.pinned_cap = 0;
            const size_t want = std::max(need, (size_t)1 << 20);
            hipError_t e = hipHostMalloc(&sl.pinned, want, hipHostMallocDefault);
            if (e != hipSuccess) return map_err(e);
            sl.pinned_cap = want;
        }
        h = (uint8_t*)sl.pinned;
        std::memcpy(h, r->page.data(), Ls.in_bytes);
    }
    r->stage = h;
    const int64_t t0 = now_ns();
    hipStream_t s = sl.stream;
    void* arena = nullptr;
    hipError_t e = hipMallocAsync(&arena, r->footprint, s);
    if (e != hipSuccess) return map_err(e);
    sl.arena = arena;
    sl.arena_cap = r->footprint;
    uint8_t* d = (uint8_t*)arena;
    e = hipEventRecord(sl.ev[0], s);
    if (r->owned) {
        // staged: the two sides straight from the caller's block, then the per-pair arrays
        if (e == hipSuccess && r->total)
            e = hipMemcpyAsync(d + L.reads, r->owned, (size_t)r->total, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && r->total)
            e = hipMemcpyAsync(d + L.refs, r->owned + r->owned_refs, (size_t)r->total, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d + L.offsets, h + Ls.offsets, L.in_bytes - L.offsets, hipMemcpyHostToDevice, s);
    } else if (e == hipSuccess) {
        e = hipMemcpyAsync(d, h, L.in_bytes, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipMemsetAsync(d + L.err, 0, 4, s);
    if (e == hipSuccess) e = hipEventRecord(sl.ev[1], s);
    if (e == hipSuccess)
        e = launch_pack_stream(d + L.reads, d + L.refs, r->total, (uint32_t*)(d + L.packed), (uint32_t*)(d + L.err), s);
    if (e == hipSuccess) {
        const int cap = S->grid_cap[r->rsmax] > 0 ? S->grid_cap[r->rsmax] : 1;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(r->n_items, cap));
        e = launch_persist(r->rsmax, grid, (const PItem*)(d + L.items), (int)r->n_items, (int*)(d + L.head),
                           (const int64_t*)(d + L.perm), (const uint32_t*)(d + L.packed), r->total,
                           (const int64_t*)(d + L.offsets), (const int32_t*)(d + L.lengths),
                           (const int32_t*)(d + L.E), (uint16_t*)(d + L.results), s);
    }
    if (e == hipSuccess) e = hipEventRecord(sl.ev[2], s);
    const size_t hres = Ls.in_bytes, herr = Ls.in_bytes + al((size_t)r->n * 2);
    if (e == hipSuccess && r->n)
        e = hipMemcpyAsync(h + hres, d + L.results, (size_t)r->n * 2, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + herr, d + L.err, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(sl.ev[3], s);
    // the memory returns to the pool once the stream has passed this point
    const hipError_t ef = hipFreeAsync(arena, s);
    if (e == hipSuccess) e = ef;
    sl.arena = nullptr;
    sl.arena_cap = 0;
    if (e == hipSuccess) e = hipEventRecord(sl.done, s);
    r->ns_enqueue = now_ns() - t0;
    return map_err(e);
}

// Pick a free slot for the head request if its footprint fits the budget next
// to the requests in flight.  Returns the slot index or -1.  Lock held.
int admit_slot(ss_server* S, Request* r)
{
    if (S->used + r->footprint > S->budget) return -1;
    for (int i = 0; i < (int)S->slots.size(); i++) {
        if (S->slots[(size_t)i].cur) continue;
        if (S->loop && !S->arena_alloc.alloc(r->footprint, &r->arena_off)) return -1;
        S->used += r->footprint;
        S->peak_used = std::max<int64_t>(S->peak_used, (int64_t)S->used);
        return i;
    }
    return -1;
}

// Return a request's pinned staging (and a staged submission's block) to the pool.
void release_staging(ss_server* S, Request* r)
{
    if (r->pin) {
        S->pool.put(r->pin, r->pin_cls);
        r->pin = nullptr;
    }
    if (r->owned) {
        S->pool.put(r->owned, r->owned_cls);
        r->owned = nullptr;
    }
}

void finish(ss_server* S, Request* r, int status)
{
    // lock held
    if (r->state == RUNNING) {
        S->used -= r->footprint;
        if (S->loop) S->arena_alloc.release(r->arena_off, r->footprint);
    }
    r->status = status;
    r->state = DONE;
    r->t_done = now_ns();
    release_staging(S, r);
    r->page.clear();
    r->page.shrink_to_fit();
    r->stage = nullptr;
    S->completed++;
    S->cv_done.notify_all();
}

void dispatcher_main(ss_server* S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_work.wait(lk, [&] { return S->stop || (!S->hold && !S->queue.empty()); });
        if (S->stop) return;
        Request* r = S->queue.front();
        const int si = admit_slot(S, r);
        if (si < 0) {
            S->deferred++;
            // wait for a completion (or new state) and try again
            S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            continue;
        }
        S->queue.pop_front();
        Slot& sl = S->slots[(size_t)si];
        sl.cur = r;
        r->slot = si;
        r->state = RUNNING;
        r->t_admit = now_ns();
        S->admitted++;
        S->running++;
        S->peak_running = std::max<int64_t>(S->peak_running, S->running);
        lk.unlock();
        const int rc = S->loop ? launch_request_loop(S, sl, si, r) : launch_request(S, sl, r);
        lk.lock();
        if (rc != SS_OK && S->loop && r->gen != 0) {
            // published, but the kernel could not be launched: the completion thread retries the
            // launch and fails the request if the device has failed
            sl.launched = true;
        } else if (rc != SS_OK) {
            // the stream may hold part of the work: wait for it before reusing the slot
            if (!S->loop) (void)hipStreamSynchronize(sl.stream);
            sl.cur = nullptr;
            S->running--;
            finish(S, r, rc);
        } else {
            sl.launched = true;      // only now may the completion thread poll the event
        }
        S->cv_work.notify_all();     // wake the completion thread
    }
}

void completer_main(ss_server* S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<int> busy;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop && S->running == 0) return;
            for (int i = 0; i < (int)S->slots.size(); i++)
                if (S->slots[(size_t)i].cur && S->slots[(size_t)i].launched) busy.push_back(i);
            if (busy.empty()) {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
        }
        bool any = false;
        if (S->loop) {
            // a request may wait for a launch (the last kernel ended idle just before it was published)
            const int rc = ensure_loop(S);
            if (rc != SS_OK) {
                std::lock_guard<std::mutex> lk(S->mu);
                for (int i : busy) {
                    Slot& sl = S->slots[(size_t)i];
                    Request* r = sl.cur;
                    // the staging block (and a staged submission's block) stays with the request: a
                    // kernel may still read or write it
                    r->pin = nullptr;
                    r->owned = nullptr;
                    sl.cur = nullptr;
                    sl.launched = false;
                    S->running--;
                    finish(S, r, rc);
                }
                S->broken = true;
                S->cv_work.notify_all();
                continue;
            }
        }
        for (int i : busy) {
            Slot& sl = S->slots[(size_t)i];
            if (S->loop) {
                Request* r = sl.cur;
                if (__atomic_load_n(&S->H->fin[i], __ATOMIC_ACQUIRE) != r->gen) continue;
                TraceRange tr("serve: hand results to the caller");
                const uint64_t ta = S->H->t_act[i], tp = S->H->t_packed[i], td = S->H->t_done[i];
                const bool ordered = ta <= tp && tp <= td;
                r->ns_h2d = ordered ? (int64_t)(S->tick_ns * (double)(tp - ta)) : 0;
                r->ns_compute = (int64_t)(S->tick_ns * (double)(td - (ordered ? tp : ta)));
                r->ns_d2h = 0;
                const Layout L = stage_layout(r);
                const uint16_t* res = (const uint16_t*)(r->stage + L.in_bytes);
                int status = SS_OK;
                if (S->H->err[i]) {
                    status = SS_EBASE;                 // outputs untouched
                } else {
                    for (int64_t k = 0; k < r->n; k++) {
                        r->accept_out[k] = (uint8_t)(res[k] >> 15);
                        r->edits_out[k] = (int32_t)(res[k] & SS_RESULT_COUNT);
                    }
                }
                std::lock_guard<std::mutex> lk(S->mu);
                sl.cur = nullptr;
                sl.launched = false;
                S->running--;
                finish(S, r, status);
                S->cv_work.notify_all();
                any = true;
                continue;
            }
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            TraceRange tr("serve: hand results to the caller");
            Request* r = sl.cur;
            int status = map_err(q);
            if (status == SS_OK) {
                float ms[3] = {0.f, 0.f, 0.f};
                for (int k = 0; k < 3; k++)
                    if (hipEventElapsedTime(&ms[k], sl.ev[k], sl.ev[k + 1]) != hipSuccess) ms[k] = 0.f;
                r->ns_h2d = (int64_t)(1e6 * ms[0]);
                r->ns_compute = (int64_t)(1e6 * ms[1]);
                r->ns_d2h = (int64_t)(1e6 * ms[2]);
                const Layout L = stage_layout(r);
                const uint8_t* h = r->stage;
                const uint16_t* res = (const uint16_t*)(h + L.in_bytes);
                uint32_t err = 0;
                std::memcpy(&err, h + L.in_bytes + al((size_t)r->n * 2), 4);
                if (err) {
                    status = SS_EBASE;                 // outputs untouched
                } else {
                    for (int64_t k = 0; k < r->n; k++) {
                        r->accept_out[k] = (uint8_t)(res[k] >> 15);
                        r->edits_out[k] = (int32_t)(res[k] & SS_RESULT_COUNT);
                    }
                }
            }
            std::lock_guard<std::mutex> lk(S->mu);
            sl.cur = nullptr;
            sl.launched = false;
            S->running--;
            finish(S, r, status);
            S->cv_work.notify_all();
            any = true;
        }
        // requests in flight: look again at once (a sleep here costs its timer slack and, on a busy
        // host, a wake-up delay in the completion latency)
        if (!any) std::this_thread::yield();
    }
}

}  // namespace

extern "C" int64_t ss_server_footprint(int64_t n_pairs, int64_t total_bases)
{
    if (n_pairs < 0 || total_bases < 0) return -1;
    return (int64_t)footprint_of(n_pairs, total_bases);
}

extern "C" int ss_server_create(ss_ctx* ctx, size_t hbm_budget_bytes, int32_t n_slots, ss_server** out)
{
    if (!ctx || !out || n_slots < 1 || n_slots > 64 || hbm_budget_bytes < 4096) return SS_EINVAL;
    ss_server* S = new (std::nothrow) ss_server();
    if (!S) return SS_ENOMEM;
    S->ctx = ctx;
    (void)hipGetDevice(&S->device);
    S->budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, S->device) != hipSuccess) { delete S; return SS_EDEVICE; }
    for (int w : {1, 2, 4, 8}) S->grid_cap[w] = persist_blocks_per_cu(w) * prop.multiProcessorCount;
    {
        // keep freed request memory in the device's stream-ordered pool
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, S->device) == hipSuccess && pool) {
            uint64_t keep = (uint64_t)hbm_budget_bytes;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
    }
    S->slots.resize((size_t)n_slots);
    for (auto& sl : S->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        for (int k = 0; k < 4 && e == hipSuccess; k++) e = hipEventCreate(&sl.ev[k]);
        if (e != hipSuccess) {
            for (auto& o : S->slots) {
                if (o.done) (void)hipEventDestroy(o.done);
                for (hipEvent_t x : o.ev)
                    if (x) (void)hipEventDestroy(x);
                if (o.stream) (void)hipStreamDestroy(o.stream);
            }
            delete S;
            return map_err(e);
        }
    }
    S->pool.reserve(staging_region_bytes(hbm_budget_bytes));
    S->dispatcher = std::thread(dispatcher_main, S);
    S->completer = std::thread(completer_main, S);
    *out = S;
    return SS_OK;
}

namespace {

constexpr int kLoopIdleMs = 200;     // the loop kernel ends after this long with nothing to do (default)
constexpr int kLoopStallMs = 2000;   // requests active and no unit finished for this long: give up

// Devices that hold a device-resident loop server: its kernel takes every CU
// while it runs, so a second one on the same device would wait for the first
// to go idle.
std::mutex g_loop_mu;
bool g_loop_dev[64] = {};

void free_loop(ss_server* S)
{
    if (S->loop_stream) (void)hipStreamSynchronize(S->loop_stream);
    if (S->loop_ev) (void)hipEventDestroy(S->loop_ev);
    if (S->loop_stream) (void)hipStreamDestroy(S->loop_stream);
    if (S->arena) (void)hipFree(S->arena);
    if (S->D) (void)hipFree(S->D);
    if (S->H) (void)hipHostFree(S->H);
    S->loop_ev = nullptr;
    S->loop_stream = nullptr;
    S->arena = nullptr;
    S->D = nullptr;
    S->H = nullptr;
}

}  // namespace

extern "C" int ss_server_create_loop(ss_ctx* ctx, size_t hbm_budget_bytes, int32_t n_slots, int32_t slices_per_lane,
                                     ss_server** out)
{
    if (!ctx || !out || n_slots < 1 || n_slots > loop::kSlots || hbm_budget_bytes < 4096) return SS_EINVAL;
    if (slices_per_lane != 1 && slices_per_lane != 2 && slices_per_lane != 4 && slices_per_lane != 8)
        return SS_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SS_EDEVICE;
    {
        std::lock_guard<std::mutex> lk(g_loop_mu);
        if (g_loop_dev[dev]) return SS_EAGAIN;          // one device-resident loop per device
        g_loop_dev[dev] = true;
    }
    ss_server* S = new (std::nothrow) ss_server();
    if (!S) {
        std::lock_guard<std::mutex> lk(g_loop_mu);
        g_loop_dev[dev] = false;
        return SS_ENOMEM;
    }
    S->ctx = ctx;
    S->device = dev;
    S->budget = hbm_budget_bytes;
    S->loop = true;
    S->loop_rs = slices_per_lane;
    S->rsmax = slices_per_lane;
    S->pool.flags = hipHostMallocCoherent | hipHostMallocMapped;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, S->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(g_loop_mu);
        g_loop_dev[dev] = false;
        delete S;
        return SS_EDEVICE;
    }
    {
        // One block per CU, so that a request's long items each own a CU's four SIMDs: every block
        // reserves more than half of a CU's LDS, and the dispatcher cannot stack two on one CU (with
        // as many blocks per CU as fit, items shared CUs and the 99th percentile of the service time
        // measured 1.6 times longer).
        const size_t lds_cu = (size_t)prop.maxSharedMemoryPerMultiProcessor;
        const size_t st = loop::loop_static_lds(slices_per_lane);
        S->loop_lds_pad = lds_cu / 2 + 1024 > st ? lds_cu / 2 + 1024 - st : 0;
        S->loop_grid = prop.multiProcessorCount;
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, S->device) != hipSuccess || khz <= 0)
        khz = 100000;
    S->tick_ns = 1e6 / (double)khz;
    S->khz = (uint64_t)khz;
    S->idle_ticks = (uint64_t)khz * kLoopIdleMs;
    S->stall_ticks = (uint64_t)khz * kLoopStallMs;
    hipError_t e = hipHostMalloc((void**)&S->H, sizeof(loop::Host), hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess) {
        std::memset((void*)S->H, 0, sizeof(loop::Host));
        e = hipHostGetDevicePointer((void**)&S->H_dev, S->H, 0);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->loop_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->loop_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void**)&S->D, sizeof(loop::Dev));
    // zeroed on the loop's own stream, so before any launch of the loop
    if (e == hipSuccess) e = hipMemsetAsync(S->D, 0, sizeof(loop::Dev), S->loop_stream);
    if (e == hipSuccess) e = hipMalloc((void**)&S->arena, hbm_budget_bytes);
    if (e == hipSuccess) e = hipStreamSynchronize(S->loop_stream);
    if (e != hipSuccess) {
        free_loop(S);
        delete S;
        std::lock_guard<std::mutex> lk(g_loop_mu);
        g_loop_dev[dev] = false;
        return map_err(e);
    }
    S->arena_alloc.reset(hbm_budget_bytes);
    S->slots.resize((size_t)n_slots);
    S->pool.reserve(staging_region_bytes(hbm_budget_bytes));
    S->dispatcher = std::thread(dispatcher_main, S);
    S->completer = std::thread(completer_main, S);
    *out = S;
    return SS_OK;
}

namespace {

// Submission shared by ss_server_submit and ss_server_submit_staged.  block: a staged submission's
// block of the server's staging (NULL: copy reads and refs into staging), block_bytes its size and
// refs_off where its refs start.  The request takes the block only when it returns SS_OK.
int submit_impl(ss_server* S, const uint8_t* reads, const uint8_t* refs, uint8_t* block, size_t block_cls,
                size_t block_bytes, size_t refs_off, const int32_t* lengths, const int32_t* E_per_pair,
                int64_t n_pairs, uint8_t* accept_out, int32_t* edits_out, ss_ticket* ticket)
{
    if (!S || !ticket || n_pairs < 0) return SS_EINVAL;
    if (n_pairs > 0 && (!reads || !refs || !lengths || !E_per_pair || !accept_out || !edits_out)) return SS_EINVAL;
    TraceRange tr("serve: submit (plan and stage)");
    int64_t T = 0;
    for (int64_t i = 0; i < n_pairs; i++) {
        if (lengths[i] < 0 || E_per_pair[i] < 0) return SS_EINVAL;
        if (lengths[i] > SS_MAX_LEN || E_per_pair[i] > SS_MAX_E) return SS_ELEN;
        T += lengths[i];
    }
    if (T > SS_MAX_STREAM_BASES) return SS_ELEN;
    if (block && (refs_off < (size_t)T || refs_off > block_bytes || block_bytes - refs_off < (size_t)T))
        return SS_EINVAL;            // the two sides must lie in the block, apart
    if (S->loop && cdiv(cdiv(T, 32) + 2, loop::kPackWords) > loop::kMaxUnits) return SS_ELEN;
    Request* r = nullptr;
    try {
        r = new Request();
        r->n = n_pairs;
        r->total = T;
        r->footprint = S->loop ? loop_footprint(T) : footprint_of(n_pairs, T);
        if (r->footprint > S->budget) {
            delete r;
            return SS_EBUDGET;
        }
        const int rsmin = plan_min_slices(E_per_pair, n_pairs);
        if (rsmin == 0 || (S->loop && rsmin > S->loop_rs)) {
            delete r;
            return SS_ELEN;
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            r->rsmax = std::max(S->rsmax, rsmin);
        }
        std::vector<PItem> items;
        std::vector<int64_t> perm;
        int nc = 0;
        double cost = 0;
        if (!plan_items(lengths, E_per_pair, n_pairs, r->rsmax, items, perm, &nc, &cost) ||
            (S->loop && (int64_t)items.size() > loop::kMaxUnits)) {
            delete r;
            return SS_ELEN;
        }
        r->n_items = (int64_t)items.size();
        // the staging layout (as stage_layout gives it once the request holds the block)
        const Layout L(n_pairs, block ? 0 : T, r->n_items);
        const size_t need = stage_bytes(L, n_pairs);
        uint8_t* h = (uint8_t*)S->pool.get(need, &r->pin_cls);
        if (h) {
            r->pin = h;
        } else {
            r->page.resize(need);
            h = r->page.data();
        }
        if (T && !block) {
            S->copier.copy(h + L.reads, reads, (size_t)T);
            S->copier.copy(h + L.refs, refs, (size_t)T);
        }
        int64_t* off = (int64_t*)(h + L.offsets);
        int64_t o = 0;
        for (int64_t i = 0; i < n_pairs; i++) { off[i] = o; o += lengths[i]; }
        std::memcpy(h + L.lengths, lengths, (size_t)n_pairs * 4);
        std::memcpy(h + L.E, E_per_pair, (size_t)n_pairs * 4);
        if (!items.empty()) std::memcpy(h + L.items, items.data(), items.size() * sizeof(PItem));
        std::memcpy(h + L.perm, perm.data(), (size_t)n_pairs * 8);
    } catch (const std::bad_alloc&) {
        if (r && r->pin) S->pool.put(r->pin, r->pin_cls);
        delete r;
        return SS_ENOMEM;
    }
    r->accept_out = accept_out;
    r->edits_out = edits_out;
    r->t_submit = now_ns();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop || S->broken) {
        if (r->pin) S->pool.put(r->pin, r->pin_cls);
        delete r;
        return S->broken ? SS_EDEVICE : SS_EINVAL;
    }
    if (block) {
        r->owned = block;            // from here the request returns it to the pool
        r->owned_cls = block_cls;
        r->owned_refs = refs_off;
    }
    r->id = S->next_id++;
    S->reqs[r->id] = r;
    *ticket = r->id;
    if (n_pairs == 0) {
        finish(S, r, SS_OK);
        return SS_OK;
    }
    S->queue.push_back(r);
    S->cv_work.notify_all();
    return SS_OK;
}

}  // namespace

extern "C" int ss_server_submit(ss_server* S, const uint8_t* reads, const uint8_t* refs, const int32_t* lengths,
                                const int32_t* E_per_pair, int64_t n_pairs, uint8_t* accept_out, int32_t* edits_out,
                                ss_ticket* ticket)
{
    return submit_impl(S, reads, refs, nullptr, 0, 0, 0, lengths, E_per_pair, n_pairs, accept_out, edits_out, ticket);
}

extern "C" void* ss_server_stage_alloc(ss_server* S, size_t bytes)
{
    if (!S || bytes == 0) return nullptr;
    size_t cls = 0;
    void* p = S->pool.get(bytes, &cls);
    if (!p) return nullptr;
    std::lock_guard<std::mutex> lk(S->blocks_mu);
    S->blocks[p] = std::make_pair(cls, bytes);
    return p;
}

extern "C" int ss_server_stage_free(ss_server* S, void* block)
{
    if (!S || !block) return SS_EINVAL;
    size_t cls = 0;
    {
        std::lock_guard<std::mutex> lk(S->blocks_mu);
        auto it = S->blocks.find(block);
        if (it == S->blocks.end()) return SS_EINVAL;
        cls = it->second.first;
        S->blocks.erase(it);
    }
    S->pool.put(block, cls);
    return SS_OK;
}

extern "C" int ss_server_submit_staged(ss_server* S, void* block, size_t refs_offset, const int32_t* lengths,
                                       const int32_t* E_per_pair, int64_t n_pairs, uint8_t* accept_out,
                                       int32_t* edits_out, ss_ticket* ticket)
{
    if (!S || !block) return SS_EINVAL;
    std::pair<size_t, size_t> info;
    {
        // out of the registry while the submission runs (back in if it fails): once submitted, the
        // request may finish and the pool hand the same address out again
        std::lock_guard<std::mutex> lk(S->blocks_mu);
        auto it = S->blocks.find(block);
        if (it == S->blocks.end()) return SS_EINVAL;
        info = it->second;
        S->blocks.erase(it);
    }
    uint8_t* b = (uint8_t*)block;
    const int rc = submit_impl(S, b, b + std::min(refs_offset, info.second), b, info.first, info.second, refs_offset,
                               lengths, E_per_pair, n_pairs, accept_out, edits_out, ticket);
    if (rc != SS_OK) {
        std::lock_guard<std::mutex> lk(S->blocks_mu);
        S->blocks[block] = info;
    }
    return rc;
}

extern "C" int ss_server_poll(ss_server* S, ss_ticket t, int* done)
{
    if (!S || !done) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return SS_EINVAL;
    *done = it->second->state == DONE || it->second->state == CANCELLED;
    return SS_OK;
}

extern "C" int ss_server_wait(ss_server* S, ss_ticket t, int64_t timeout_us)
{
    if (!S) return SS_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return SS_EINVAL;
    Request* r = it->second;
    auto pred = [&] { return r->state == DONE || r->state == CANCELLED; };
    if (timeout_us < 0) S->cv_done.wait(lk, pred);
    else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred)) return SS_ETIMEOUT;
    return r->state == CANCELLED ? SS_EAGAIN : r->status;
}

extern "C" int ss_server_times(ss_server* S, ss_ticket t, int64_t* submit_ns, int64_t* admit_ns, int64_t* done_ns)
{
    if (!S) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return SS_EINVAL;
    if (submit_ns) *submit_ns = it->second->t_submit;
    if (admit_ns) *admit_ns = it->second->t_admit;
    if (done_ns) *done_ns = it->second->t_done;
    return SS_OK;
}

extern "C" int ss_server_stages(ss_server* S, ss_ticket t, int64_t* enqueue_ns, int64_t* h2d_ns, int64_t* compute_ns,
                                int64_t* d2h_ns)
{
    if (!S) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return SS_EINVAL;
    const Request* r = it->second;
    if (enqueue_ns) *enqueue_ns = r->ns_enqueue;
    if (h2d_ns) *h2d_ns = r->ns_h2d;
    if (compute_ns) *compute_ns = r->ns_compute;
    if (d2h_ns) *d2h_ns = r->ns_d2h;
    return SS_OK;
}

extern "C" int ss_server_cancel(ss_server* S, ss_ticket t)
{
    if (!S) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return SS_EINVAL;
    Request* r = it->second;
    if (r->state != QUEUED) return SS_EAGAIN;
    S->queue.erase(std::remove(S->queue.begin(), S->queue.end(), r), S->queue.end());
    r->state = CANCELLED;
    r->t_done = now_ns();
    release_staging(S, r);
    r->page.clear();
    S->cv_done.notify_all();
    return SS_OK;
}

extern "C" int ss_server_release(ss_server* S, ss_ticket t)
{
    if (!S) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return SS_EINVAL;
    if (it->second->state == QUEUED || it->second->state == RUNNING) return SS_EAGAIN;
    delete it->second;
    S->reqs.erase(it);
    return SS_OK;
}

extern "C" int ss_server_set_hold(ss_server* S, int hold)
{
    if (!S) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    S->hold = hold != 0;
    S->cv_work.notify_all();
    return SS_OK;
}

extern "C" int ss_server_set_slices(ss_server* S, int32_t slices_per_lane)
{
    if (!S) return SS_EINVAL;
    if (slices_per_lane != 1 && slices_per_lane != 2 && slices_per_lane != 4 && slices_per_lane != 8) return SS_EINVAL;
    if (S->loop) return SS_EINVAL;       // the loop kernel's slice width is fixed at creation
    std::lock_guard<std::mutex> lk(S->mu);
    S->rsmax = slices_per_lane;
    return SS_OK;
}

extern "C" int ss_server_set_loop_idle(ss_server* S, int64_t idle_us)
{
    if (!S || !S->loop || idle_us < 1 || idle_us > 60ll * 1000 * 1000) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->loop_mu);
    S->idle_ticks = std::max<uint64_t>(1, S->khz * (uint64_t)idle_us / 1000);   // takes effect at the next launch
    return SS_OK;
}

extern "C" int ss_server_stats(ss_server* S, int64_t* admitted, int64_t* deferred, int64_t* completed,
                               int64_t* peak_bytes, int64_t* peak_in_flight)
{
    if (!S) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (admitted) *admitted = S->admitted;
    if (deferred) *deferred = S->deferred;
    if (completed) *completed = S->completed;
    if (peak_bytes) *peak_bytes = S->peak_used;
    if (peak_in_flight) *peak_in_flight = S->peak_running;
    return SS_OK;
}

extern "C" int ss_server_destroy(ss_server* S)
{
    if (!S) return SS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        // queued requests are cancelled; running ones finish
        for (Request* r : S->queue) {
            r->state = CANCELLED;
            r->t_done = now_ns();
            release_staging(S, r);
        }
        S->queue.clear();
        S->hold = false;
        S->stop = true;
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    S->dispatcher.join();
    S->completer.join();
    if (S->loop) {
        // nothing is in flight any more: the loop kernel ends at its next look at the stop word
        __atomic_store_n(&S->H->stop, 1ull, __ATOMIC_RELEASE);
        free_loop(S);
        std::lock_guard<std::mutex> lk(g_loop_mu);
        g_loop_dev[S->device] = false;
    }
    for (auto& sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        if (sl.done) (void)hipEventDestroy(sl.done);
        for (hipEvent_t x : sl.ev)
            if (x) (void)hipEventDestroy(x);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto& kv : S->reqs) delete kv.second;
    {
        // blocks a caller took and never submitted or freed
        std::lock_guard<std::mutex> lk(S->blocks_mu);
        for (auto& kv : S->blocks) S->pool.put(kv.first, kv.second.first);
        S->blocks.clear();
    }
    S->pool.release_all();
    delete S;
    return SS_OK;
}
