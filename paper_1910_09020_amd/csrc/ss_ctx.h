// The library context (ss_ctx of ss.h): device buffers reused across calls and
// the context's own stream.  Shared by the host-runtime sources.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <mutex>

// Device buffers that grow on demand and are reused across calls.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (p) { (void)hipFree(p); p = nullptr; cap = 0; }
        size_t want = std::max(bytes, (size_t)256);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Pinned host buffers that grow on demand (hipHostMalloc: copies from them run
// on the copy engine at full speed and can overlap kernels).
struct HostBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (p) { (void)hipHostFree(p); p = nullptr; cap = 0; }
        size_t want = std::max(bytes, (size_t)4096);
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct ss_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuf reads, refs, offsets, lengths, epp, packed, results, err;
    DevBuf chunk;            // lane-sliced encoding of ss_filter_ascii_async's two-kernel schedule
    DevBuf qside, rside;     // the two sides packed apart (ss_filter_batch_ex from ASCII)
    DevBuf uoff, ulen;       // offsets / lengths of pairs of one length back to back
    DevBuf roff, rlen;       // reference offsets / lengths (the host one-call for unequal lengths)
    // the host entry point's pipeline for pinned input: two device staging buffers, a copy stream,
    // events (a staging buffer's copy done; its filter done); pinned room for the result words
    HostBuf hres;
    DevBuf dstage[2];
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_h2d[2] = {nullptr, nullptr}, ev_used[2] = {nullptr, nullptr};
    std::mutex host_mu;      // the one-call host entry points use this context's buffers one call at a time
};

// The process-wide context of the current HIP device (created on first use),
// used by the one-call host entry points.
int ss_default_ctx(ss_ctx** out);

// Called by ss_create with hip_device current: looks up the device address of
// the no-allocation entry point's scratch array on that device (ss_noalloc.hip).
int ss_noalloc_init_device(int dev);
