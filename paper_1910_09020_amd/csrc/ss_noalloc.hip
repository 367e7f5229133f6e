// The one-call encode + filter without any allocation (ss_filter_ascii_noalloc):
// the variant of ss_filter_ascii_async for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// it).  Its scratch, the lane-sliced encoding of one chunk of pairs for the
// two-kernel schedule, is a file-scope device array: each GPU the library runs
// on holds its own copy for the life of the process, and every call on that GPU
// uses it, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "ss.h"
#include "ss_common.h"
#include "ss_ctx.h"

using namespace ss;

static __device__ __align__(256) uint32_t scratch[SS_NOALLOC_SCRATCH_BYTES / 4];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // the array's device address on each device

int map_err(hipError_t e)
{
    if (e == hipSuccess) return SS_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SS_ENOMEM;
    return SS_EDEVICE;
}

}  // namespace

// Called by ss_create with dev current: the array's address on this device
// (the host-side name of the array is not a device address).
int ss_noalloc_init_device(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[dev]) return SS_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return SS_EDEVICE;
    g_scratch[dev] = ptr;
    return SS_OK;
}

extern "C" int ss_filter_ascii_noalloc(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs, int64_t n_pairs,
                                       int32_t m, int32_t E, uint16_t* out, uint32_t* err, void* stream)
{
    if (!ctx || n_pairs < 0 || m < 0 || E < 0) return SS_EINVAL;
    if (E > SS_MAX_E_SLICED || m > SS_MAX_LEN_FUSED) return SS_ELEN;
    if (n_pairs == 0) return SS_OK;
    if (!out || (m > 0 && (!reads || !refs))) return SS_EINVAL;
    if (((uintptr_t)out & 15u) != 0) return SS_EINVAL;
    int T = 0, GB = 0, U = 0;
    const bool contiguous = (((uintptr_t)reads | (uintptr_t)refs) & 15u) == 0;
    if (fused_shape(m, 0, contiguous, &T, &GB, &U, fused_tile_cap(n_pairs)) == 0) return SS_EINVAL;
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) ptr = g_scratch[ctx->device];
    }
    if (!ptr) return SS_EDEVICE;
    const hipStream_t s = (hipStream_t)stream;
    // the same schedule as ss_filter_ascii_async with the automatic tile: the fused kernel (no scratch)
    // in its wave mode, or for unaligned inputs; else the two kernels over chunks that fit the scratch
    // (pairs of length 0 take the two kernels: the sweep reads nothing and writes each result)
    if (E <= kMaxEFused && m > 0 && (U > 0 || !contiguous))
        return map_err(launch_fused(reads, refs, n_pairs, m, E, 0, out, err, s));
    const int64_t group_bytes = std::max<int64_t>(1, ss_sliced_bytes(32, m));   // one group's encoding (0 at m = 0)
    static_assert(SS_NOALLOC_SCRATCH_BYTES >= 4LL * ((SS_MAX_LEN_FUSED + 3) / 4) * 64 * 16,
                  "the scratch holds a whole layout block of the longest pairs");
    // chunks of whole 64-group layout blocks, so that each chunk's encoding is laid out on its own
    const int64_t chunk = std::max<int64_t>(64, (SS_NOALLOC_SCRATCH_BYTES / group_bytes) / 64 * 64) * 32;
    for (int64_t s0 = 0; s0 < n_pairs; s0 += chunk) {
        const int64_t k = std::min(chunk, n_pairs - s0);
        if (ss_sliced_bytes(k, m) > SS_NOALLOC_SCRATCH_BYTES) return SS_ELEN;   // cannot happen (see above)
        hipError_t e = launch_pack_sliced(reads + s0 * m, refs + s0 * m, nullptr, nullptr, k, m, (uint32_t*)ptr, err,
                                          s);
        if (e == hipSuccess) e = launch_sliced((const uint32_t*)ptr, k, m, E, out + s0, s);
        if (e != hipSuccess) return map_err(e);
    }
    return SS_OK;
}
