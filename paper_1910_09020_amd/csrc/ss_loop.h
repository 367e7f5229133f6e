// Device-resident serving loop: the layouts shared by the host runtime
// (ss_serve.cpp) and the loop kernel (ss_loop.hip).
//
// The host publishes a request by writing its descriptor into one of kSlots
// slots of a control block in coherent host memory and then the slot's
// publication word (a generation number, one higher for each request of the
// slot).  One persistent kernel serves every slot: its first wavefront polls
// the publication words and activates new requests in a device-side slot
// table; the other blocks take work units from the active slots, oldest
// admission first: first the encoding of the request's ASCII (read straight
// from host memory) into four bit planes in device memory, then the items of
// the request's plan, whose result words go straight to host memory.  The
// block that finishes a request's last item writes the request's generation
// into the slot's completion word, which the host polls.
#pragma once
#include <stdint.h>

#include "ss_common.h"

namespace ss {
namespace loop {

constexpr int kSlots = 64;           // requests in flight at most
constexpr int kPackWords = 1024;     // plane words one block encodes per unit (4 per thread)
// Pack units and items of one request: the claim counter's 24-bit next field
// may run past the count by as many claims as there are worker blocks.
constexpr int64_t kMaxUnits = (1 << 24) - (1 << 16);

// A request as published.  Pointers to host memory are device-visible
// (coherent pinned host memory); packed is device memory.
struct Desc {
    const uint8_t* reads;        // ASCII of both sides, pair i at offsets[i]
    const uint8_t* refs;
    const int64_t* offsets;
    const int32_t* lengths;
    const int32_t* E;
    const PItem* items;          // the request's plan
    const int64_t* perm;
    uint16_t* results;           // one result word per pair (host memory)
    uint32_t* packed;            // four planes of SW words (device memory)
    int64_t total;               // bases of each side
    int64_t SW;                  // words per plane
    int32_t n_items;
    int32_t n_pack;              // encoding units: cdiv(SW, kPackWords)
    int32_t aligned;             // reads and refs are 16-byte aligned
    int32_t pad;
};

// Control block in coherent host memory.
struct Host {
    uint64_t pub[kSlots];        // host: generation of the request last published in the slot (0: none)
    uint64_t fin[kSlots];        // device: generation of the request last finished in the slot
    uint64_t t_act[kSlots];      // device clock when the request was activated,
    uint64_t t_packed[kSlots];   // when its encoding was complete,
    uint64_t t_done[kSlots];     // and when its last item was done
    uint32_t err[kSlots];        // device: the finished request's error word (bit 0: a byte that is not a base)
    uint64_t stop;               // host: nonzero ends the loop as soon as nothing is in flight
    uint64_t stalled;            // device: nonzero when a launch ended because no unit finished for
                                 // ten idle periods while requests were active (never expected)
    Desc desc[kSlots];           // host: written before the publication word
};

// A claim counter: generation (16 bits) | number of units (24 bits) | next
// unit (24 bits).  A worker claims with a fetch-and-add of one, and only after
// seeing next < count; the value returned is its claim, valid when its next is
// below its count.  Because the count travels in the same word, a claim is
// judged against the request it belongs to, even when the slot was reused
// since the worker looked (a late claim on the new request is then a valid
// unit of the new request); an invalid claim changes nothing that matters.
// A request's item counter starts closed (count 0) and is opened by the block
// that finishes its last encoding unit, so every item claimed finds the planes
// complete.
__host__ __device__ inline uint64_t make_ctr(uint64_t gen, uint32_t count)
{
    return ((gen & 0xFFFFull) << 48) | ((uint64_t)(count & 0xFFFFFFu) << 24);
}
__host__ __device__ inline uint32_t ctr_count(uint64_t c) { return (uint32_t)(c >> 24) & 0xFFFFFFu; }
__host__ __device__ inline uint32_t ctr_next(uint64_t c) { return (uint32_t)c & 0xFFFFFFu; }
__host__ __device__ inline uint32_t ctr_gen(uint64_t c) { return (uint32_t)(c >> 48); }

// Device-side slot state, kept across launches of the loop (device memory,
// zeroed when the server is created).
struct Slot {
    uint64_t pack_ctr;           // claims of encoding units
    uint64_t item_ctr;           // claims of items (opened once every encoding unit is done)
    uint32_t pack_done;          // encoding units done
    uint32_t item_done;          // items done
    uint32_t err;
    uint32_t pad;
    uint64_t gen;                // generation of the request in the slot
    uint64_t adm;                // admission number: the lowest is served first
    Desc d;
};

struct Dev {
    Slot slot[kSlots];
    uint64_t seen[kSlots];       // generation last activated, per slot
    uint64_t active;             // bit s: slot s holds a request not finished yet
    uint64_t adm_next;
    uint32_t quit;               // epoch of the launch whose scheduler ended the loop
    uint32_t progress;           // units finished (any slot), watched by the scheduler
    alignas(128) uint64_t beat;  // device clock at the scheduler's last look (its heartbeat; a cache
                                 // line of its own, away from the words the workers poll)
    uint64_t pad_beat[15];
};

// The loop kernel on stream s: grid blocks of 256 threads (block 0 schedules).
// It returns once nothing has been in flight for idle_ticks of the device's
// constant-rate clock, sooner after host->stop is set, and also when requests
// are active but no unit has finished for stall_ticks (host->stalled).
// lds_pad: dynamic LDS reserved (and left unused) per block, which caps the
// blocks a CU can hold.
hipError_t launch_loop(int rsmax, int grid, size_t lds_pad, Host* host, Dev* dev, uint32_t epoch,
                       uint64_t idle_ticks, uint64_t stall_ticks, hipStream_t s);
// Static LDS bytes of one block of the loop kernel.
size_t loop_static_lds(int rsmax);

}  // namespace loop
}  // namespace ss
