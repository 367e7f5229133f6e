// C ABI of libss.so: argument validation, device-memory management and the
// one-call host entry points.  Every step of the filter runs in the HIP kernels
// of ss_sliced.hip / ss_stream.hip; this file only moves data and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "ss.h"
#include "ss_common.h"
#include "ss_ctx.h"
#include "ss_trace.h"

using namespace ss;

namespace {

int map_err(hipError_t e)
{
    if (e == hipSuccess) return SS_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SS_ENOMEM;
    return SS_EDEVICE;
}

#define SS_TRY(expr)                                   \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return map_err(_e);      \
    } while (0)

}  // namespace

extern "C" const char* ss_status_str(int status)
{
    switch (status) {
    case SS_OK: return "SS_OK";
    case SS_EINVAL: return "SS_EINVAL: invalid argument";
    case SS_EBASE: return "SS_EBASE: byte outside ACGTacgt";
    case SS_ELEN: return "SS_ELEN: length or threshold beyond the supported range";
    case SS_ENOMEM: return "SS_ENOMEM: allocation failed";
    case SS_EBUDGET: return "SS_EBUDGET: request exceeds the HBM budget";
    case SS_EDEVICE: return "SS_EDEVICE: HIP device error";
    case SS_EAGAIN: return "SS_EAGAIN: not ready";
    case SS_ETIMEOUT: return "SS_ETIMEOUT: deadline passed";
    default: return "unknown status";
    }
}

extern "C" int ss_create(ss_ctx** out, int hip_device)
{
    if (!out) return SS_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return SS_EDEVICE;
    if (hip_device < 0 || hip_device >= count) return SS_EINVAL;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return SS_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SS_EDEVICE;   // code objects are gfx950 only
    ss_ctx* c = new (std::nothrow) ss_ctx();
    if (!c) return SS_ENOMEM;
    c->device = hip_device;
    int prev = 0;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(hip_device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    // with the device current: the address of the no-allocation entry point's scratch on it
    const int rc = e == hipSuccess ? ss_noalloc_init_device(hip_device) : SS_OK;
    (void)hipSetDevice(prev);
    if (e != hipSuccess || rc != SS_OK) {
        if (c->stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return e != hipSuccess ? map_err(e) : rc;
    }
    *out = c;
    return SS_OK;
}

extern "C" int ss_destroy(ss_ctx* ctx)
{
    if (!ctx) return SS_EINVAL;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->copy_stream) (void)hipStreamSynchronize(ctx->copy_stream);
    for (DevBuf* b : {&ctx->reads, &ctx->refs, &ctx->offsets, &ctx->lengths, &ctx->epp, &ctx->packed,
                      &ctx->results, &ctx->err, &ctx->chunk, &ctx->qside, &ctx->rside, &ctx->uoff, &ctx->ulen,
                      &ctx->roff, &ctx->rlen, &ctx->dstage[0], &ctx->dstage[1]})
        b->release();
    ctx->hres.release();
    for (hipEvent_t ev : {ctx->ev_h2d[0], ctx->ev_h2d[1], ctx->ev_used[0], ctx->ev_used[1]})
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    (void)hipSetDevice(prev);
    delete ctx;
    return SS_OK;
}

// ---------------------------------------------------------------- sizes
extern "C" int64_t ss_sliced_bytes(int64_t n_pairs, int32_t m)
{
    if (n_pairs < 0 || m < 0) return -1;
    const int64_t G = cdiv(n_pairs, 32);
    return 4LL * cdiv(m, kChunk) * G * kChunk * 4LL;
}

extern "C" int64_t ss_stream_words(int64_t total_bases)
{
    if (total_bases < 0) return -1;
    return cdiv(total_bases, 32) + 2;
}

// ---------------------------------------------------------------- asynchronous device entry points
extern "C" int ss_pack_sliced_async(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs,
                                    const int64_t* offsets, const int64_t* index, int64_t n_pairs, int32_t m,
                                    uint32_t* packed, uint32_t* err, void* stream)
{
    if (!ctx || n_pairs < 0 || m < 0) return SS_EINVAL;
    if (m > SS_MAX_LEN) return SS_ELEN;
    if (n_pairs == 0 || m == 0) return SS_OK;
    if (!reads || !refs || !packed) return SS_EINVAL;
    if (((uintptr_t)packed & 15u) != 0) return SS_EINVAL;
    return map_err(launch_pack_sliced(reads, refs, offsets, index, n_pairs, m, packed, err, (hipStream_t)stream));
}

extern "C" int ss_filter_sliced_async(ss_ctx* ctx, const uint32_t* packed, int64_t n_pairs, int32_t m,
                                      int32_t E, uint16_t* out, void* stream)
{
    if (!ctx || n_pairs < 0 || m < 0 || E < 0) return SS_EINVAL;
    if (E > SS_MAX_E_SLICED || m > SS_MAX_LEN) return SS_ELEN;
    if (n_pairs == 0) return SS_OK;
    if (!out || (m > 0 && !packed)) return SS_EINVAL;
    if ((((uintptr_t)packed | (uintptr_t)out) & 15u) != 0) return SS_EINVAL;
    return map_err(launch_sliced(packed, n_pairs, m, E, out, (hipStream_t)stream));
}

extern "C" int ss_filter_sliced_range_async(ss_ctx* ctx, const uint32_t* packed, int64_t n_pairs, int32_t m,
                                            int32_t E_lo, int32_t E_hi, uint16_t* out, int64_t out_stride,
                                            void* stream)
{
    if (!ctx || n_pairs < 0 || m < 0 || E_lo < 0 || E_hi < E_lo || out_stride < n_pairs) return SS_EINVAL;
    if (E_hi > SS_MAX_E_SLICED || m > SS_MAX_LEN) return SS_ELEN;
    if (n_pairs == 0) return SS_OK;
    if (!out || (m > 0 && !packed)) return SS_EINVAL;
    if ((((uintptr_t)packed | (uintptr_t)out) & 15u) != 0 || (out_stride & 7) != 0) return SS_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    for (int E = E_lo; E <= E_hi;) {
        uint16_t* o = out + (int64_t)(E - E_lo) * out_stride;
        const int span = sliced_multi_span(E);
        if (span > 0 && E + span - 1 <= E_hi) {
            SS_TRY(launch_sliced_multi_group(E, packed, n_pairs, m, o, out_stride, s));
            E += span;
        } else {
            SS_TRY(launch_sliced(packed, n_pairs, m, E, o, s));
            E++;
        }
    }
    return SS_OK;
}

// Thresholds up to kMaxEFused (up to 10% of a 100 bp read) run the fused
// kernel; above it (and for aligned pairs longer than the fused kernel's wave
// mode takes) encode and sweep run as two kernels over chunks of packed data.
// Chunk size, measured on 10 M x 250 bp and 30 M x 100 bp: up to E = 8 the
// sweep is light and a 192 MB chunk, which stays in the device's 256 MB cache
// between the two kernels, is 4-8% faster than 400 MB; from E = 9 the sweep's
// VALU work grows and each extra launch's partly filled last wave costs more
// than the cache saves (E = 10: 1.70 -> 1.73 ms, E = 25: 2.06 -> 2.29 ms).
constexpr int64_t kChunkPackedBytes = 400ll << 20;
constexpr int64_t kChunkPackedBytesLowE = 192ll << 20;

extern "C" int ss_filter_ascii_async(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs, int64_t n_pairs,
                                     int32_t m, int32_t E, int32_t tile_groups, uint16_t* out, uint32_t* err,
                                     void* stream)
{
    if (!ctx || n_pairs < 0 || m < 0 || E < 0 || tile_groups < 0 || tile_groups > 256) return SS_EINVAL;
    if (E > SS_MAX_E_SLICED || m > SS_MAX_LEN_FUSED) return SS_ELEN;
    if (n_pairs == 0) return SS_OK;
    if (!out || (m > 0 && (!reads || !refs))) return SS_EINVAL;
    if (((uintptr_t)out & 15u) != 0) return SS_EINVAL;
    int T = 0, GB = 0, U = 0;
    const bool contiguous = (((uintptr_t)reads | (uintptr_t)refs) & 15u) == 0;
    if (fused_shape(m, tile_groups, contiguous, &T, &GB, &U, fused_tile_cap(n_pairs)) == 0) return SS_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    // The fused kernel in wave mode (aligned pairs of up to a few hundred bases) beats the two kernels;
    // in block mode it does not for aligned inputs (250 bp: 2.2-2.4 ms against 1.7 ms), so with the
    // automatic tile those go to the chunked schedule.  A tile the caller gives asks for the fused kernel.
    // (pairs of length 0 take the chunked schedule: the sweep reads nothing and writes each result)
    if (E <= kMaxEFused && m > 0 && (tile_groups > 0 || U > 0 || !contiguous))
        return map_err(launch_fused(reads, refs, n_pairs, m, E, tile_groups, out, err, s));
    // chunks of whole groups; slot offsets keep the encoder's and the sweep's alignment
    const int64_t per_pair = std::max<int64_t>(1, ss_sliced_bytes(32, m) / 32);
    const int64_t chunk_bytes = E <= 8 ? kChunkPackedBytesLowE : kChunkPackedBytes;
    const int64_t chunk = std::min<int64_t>(n_pairs, std::max<int64_t>(32, (chunk_bytes / per_pair) / 32 * 32));
    SS_TRY(ctx->chunk.ensure((size_t)ss_sliced_bytes(chunk, m)));
    for (int64_t s0 = 0; s0 < n_pairs; s0 += chunk) {
        const int64_t k = std::min(chunk, n_pairs - s0);
        SS_TRY(launch_pack_sliced(reads + s0 * m, refs + s0 * m, nullptr, nullptr, k, m, (uint32_t*)ctx->chunk.p,
                                  err, s));
        SS_TRY(launch_sliced((const uint32_t*)ctx->chunk.p, k, m, E, out + s0, s));
    }
    return SS_OK;
}

extern "C" int ss_verify_async(ss_ctx* ctx, const uint32_t* packed, int64_t total_bases, const int64_t* offsets,
                               const int32_t* lengths, const int64_t* index, int64_t n, int32_t max_len,
                               int32_t* ed_out, void* stream)
{
    if (!ctx || n < 0 || total_bases < 0 || max_len < 0) return SS_EINVAL;
    if (max_len > SS_MAX_LEN_VERIFY) return SS_ELEN;
    if (n == 0) return SS_OK;
    if (!packed || !offsets || !lengths || !ed_out) return SS_EINVAL;
    return map_err(launch_verify(packed, ss_stream_words(total_bases), offsets, lengths, index, n, max_len, ed_out,
                                 (hipStream_t)stream));
}

extern "C" int ss_verify_banded_async(ss_ctx* ctx, const uint32_t* packed, int64_t total_bases,
                                      const int64_t* offsets, const int32_t* lengths, const int32_t* E_per_pair,
                                      int32_t E, const int64_t* index, int64_t n, int32_t* ed_out, void* stream)
{
    if (!ctx || n < 0 || total_bases < 0 || E < 0) return SS_EINVAL;
    if (E > SS_MAX_E_VERIFY_BANDED) return SS_ELEN;
    if (n == 0) return SS_OK;
    if (!packed || !offsets || !lengths || !ed_out) return SS_EINVAL;
    return map_err(launch_verify_banded(packed, ss_stream_words(total_bases), offsets, lengths, E_per_pair, E, index,
                                        n, ed_out, (hipStream_t)stream));
}

extern "C" int ss_select_accepted_async(ss_ctx* ctx, const uint16_t* results, int64_t n, int64_t* index_out,
                                        int64_t* count_out, void* stream)
{
    if (!ctx || n < 0 || !count_out) return SS_EINVAL;
    if (n > 0 && (!results || !index_out)) return SS_EINVAL;
    return map_err(launch_select(results, n, index_out, reinterpret_cast<unsigned long long*>(count_out),
                                 (hipStream_t)stream));
}

extern "C" int ss_filter_submaze_async(ss_ctx* ctx, const uint32_t* packed, int64_t n_pairs, int32_t m, int32_t E,
                                       int32_t sub_width, uint16_t* out, void* stream)
{
    if (!ctx || n_pairs < 0 || m < 0 || E < 0 || sub_width < 1) return SS_EINVAL;
    if (E > SS_MAX_E_SLICED || m > SS_MAX_LEN) return SS_ELEN;
    if (n_pairs == 0) return SS_OK;
    if (!out || (m > 0 && !packed)) return SS_EINVAL;
    if ((((uintptr_t)packed | (uintptr_t)out) & 15u) != 0) return SS_EINVAL;
    return map_err(launch_sliced(packed, n_pairs, m, E, out, (hipStream_t)stream, sub_width));
}

extern "C" int ss_pack_stream_async(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs, int64_t total_bases,
                                    uint32_t* packed, uint32_t* err, void* stream)
{
    if (!ctx || total_bases < 0 || !packed) return SS_EINVAL;
    if (total_bases > 0 && (!reads || !refs)) return SS_EINVAL;
    return map_err(launch_pack_stream(reads, refs, total_bases, packed, err, (hipStream_t)stream));
}

extern "C" int ss_filter_plain_async(ss_ctx* ctx, const uint32_t* packed, int64_t total_bases,
                                     const int64_t* offsets, const int32_t* lengths, const int32_t* E_per_pair,
                                     int64_t n_pairs, int32_t E, uint16_t* out, void* stream)
{
    if (!ctx || n_pairs < 0 || total_bases < 0 || E < 0) return SS_EINVAL;
    if (E > SS_MAX_E_PLAIN) return SS_ELEN;
    if (n_pairs == 0) return SS_OK;
    if (!packed || !offsets || !lengths || !out) return SS_EINVAL;
    return map_err(launch_plain(packed, ss_stream_words(total_bases), offsets, lengths, E_per_pair, n_pairs, E, out,
                                (hipStream_t)stream));
}

extern "C" int ss_filter_wave_async(ss_ctx* ctx, const uint32_t* packed, int64_t total_bases,
                                    const int64_t* offsets, const int32_t* lengths, const int32_t* E_per_pair,
                                    int64_t n_pairs, int32_t E, uint16_t* out, void* stream)
{
    if (!ctx || n_pairs < 0 || total_bases < 0 || E < 0) return SS_EINVAL;
    if (E > SS_MAX_E || total_bases > SS_MAX_STREAM_BASES) return SS_ELEN;
    if (n_pairs == 0) return SS_OK;
    if (!packed || !offsets || !lengths || !out) return SS_EINVAL;
    return map_err(launch_wave(packed, ss_stream_words(total_bases), offsets, lengths, E_per_pair, n_pairs, E, out,
                               (hipStream_t)stream));
}

extern "C" int ss_unpack_results_async(ss_ctx* ctx, const uint16_t* results, int64_t n_pairs, uint8_t* accept_out,
                                       int32_t* edits_out, void* stream)
{
    if (!ctx || n_pairs < 0) return SS_EINVAL;
    if (n_pairs == 0) return SS_OK;
    if (!results) return SS_EINVAL;
    return map_err(launch_unpack(results, n_pairs, accept_out, edits_out, (hipStream_t)stream));
}

// ---------------------------------------------------------------- one-call host API
namespace {
std::mutex g_default_mu;
std::vector<ss_ctx*> g_default;   // one per device, created on first use
}  // namespace

int ss_default_ctx(ss_ctx** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SS_EDEVICE;
    std::lock_guard<std::mutex> lk(g_default_mu);
    if ((int)g_default.size() <= dev) g_default.resize(dev + 1, nullptr);
    if (!g_default[dev]) {
        int rc = ss_create(&g_default[dev], dev);
        if (rc != SS_OK) return rc;
    }
    *out = g_default[dev];
    return SS_OK;
}

namespace {

// ---------------------------------------------------------------- host entry point pipeline

// Host threads that split a loop between them for the length of one host call.
class Crew {
public:
    explicit Crew(int n) : n_(std::max(1, n))
    {
        for (int i = 1; i < n_; i++) th_.emplace_back([this, i] { loop(i); });
    }
    ~Crew()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            gen_++;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    // fn(a, b) over [0, n) cut in one piece per thread; returns when all are done
    void parallel(size_t n, const std::function<void(size_t, size_t)>& fn)
    {
        if (n_ == 1 || n < 4096) {
            fn(0, n);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &fn;
            count_ = n;
            left_ = n_ - 1;
            gen_++;
        }
        cv_.notify_all();
        piece(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return left_ == 0; });
        fn_ = nullptr;
    }

private:
    void piece(int i)
    {
        const size_t per = (count_ + (size_t)n_ - 1) / (size_t)n_;
        const size_t a = std::min(count_, per * (size_t)i), b = std::min(count_, a + per);
        if (b > a) (*fn_)(a, b);
    }
    void loop(int i)
    {
        uint64_t seen = 0;
        for (;;) {
            std::unique_lock<std::mutex> lk(mu_);
            cv_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (stop_) return;
            lk.unlock();
            piece(i);
            lk.lock();
            if (--left_ == 0) done_cv_.notify_one();
        }
    }
    int n_;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    uint64_t gen_ = 0;
    bool stop_ = false;
    const std::function<void(size_t, size_t)>* fn_ = nullptr;
    size_t count_ = 0;
    int left_ = 0;
};

int host_threads()
{
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::min(16u, std::max(1u, h));
}

constexpr int64_t kStageBytes = 256ll << 20;      // one chunk of reads and refs (both sides)

// True when p is pinned host memory (hipHostMalloc, or a pinned tensor of a framework built on it).
bool is_pinned_host(const void* p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();          // pageable memory is reported as an error; clear it
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

// Pairs of one length m, one threshold E <= SS_MAX_E_SLICED, m <= SS_MAX_LEN_FUSED, in pinned host
// memory: the one-call filter over chunks copied straight from the caller's arrays by the copy
// engine into two device staging buffers (the context's copy stream), chunk i's copy overlapping
// the filter of chunk i-1 (the context's stream); results come back once and are expanded by host
// threads.  (From pageable memory a staging copy on the host is needed, which measured slower than
// the runtime's own pageable copy, so pageable input takes the plain path.)
int filter_host_pipelined(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs, int64_t n, int32_t m, int32_t E,
                          uint8_t* accept_out, int32_t* edits_out)
{
    TraceRange tr("ss_filter_batch: pinned input in chunks");
    const hipStream_t s = ctx->stream;
    // chunks of a multiple of 2048 pairs: each chunk's bases and results start 16-byte aligned
    int64_t K = std::max<int64_t>(2048, (kStageBytes / std::max<int64_t>(1, 2 * (int64_t)m)) / 2048 * 2048);
    if (K > n) K = n;
    const int64_t nchunks = cdiv(n, K);
    const size_t side = (size_t)((K * (int64_t)m + 15) & ~(int64_t)15);    // refs start here in a stage
    const size_t stage_bytes = 2 * side + 64;
    if (!ctx->copy_stream) SS_TRY(hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking));
    for (int b = 0; b < 2; b++) {
        if (!ctx->ev_h2d[b]) SS_TRY(hipEventCreateWithFlags(&ctx->ev_h2d[b], hipEventDisableTiming));
        if (!ctx->ev_used[b]) SS_TRY(hipEventCreateWithFlags(&ctx->ev_used[b], hipEventDisableTiming));
        SS_TRY(ctx->dstage[b].ensure(stage_bytes));
    }
    const size_t err_at = ((size_t)n * 2 + 15) / 16 * 16;
    SS_TRY(ctx->hres.ensure(err_at + 16));
    SS_TRY(ctx->results.ensure((size_t)n * 2 + 16));
    SS_TRY(ctx->err.ensure(16));
    uint16_t* d_res = (uint16_t*)ctx->results.p;
    uint32_t* d_err = (uint32_t*)ctx->err.p;
    SS_TRY(hipMemsetAsync(d_err, 0, 4, s));
    // host threads for the expansion of the results
    Crew crew(n >= (1 << 20) ? host_threads() : 1);
    // once work is enqueued, an error returns only after both streams have drained: the copies read
    // the caller's arrays and write the staging buffers, which must not be in use after the return
    auto drain = [&](int rc) {
        (void)hipStreamSynchronize(ctx->copy_stream);
        (void)hipStreamSynchronize(s);
        return rc;
    };
#define SS_TRY_DRAIN(expr)                               \
    do {                                                 \
        const hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return drain(map_err(e_)); \
    } while (0)
    for (int64_t i = 0; i < nchunks; i++) {
        const int b = (int)(i & 1);
        const int64_t s0 = i * K, k = std::min(K, n - s0);
        uint8_t* ds = (uint8_t*)ctx->dstage[b].p;
        if (i >= 2) SS_TRY_DRAIN(hipStreamWaitEvent(ctx->copy_stream, ctx->ev_used[b], 0));   // chunk i-2 was filtered
        SS_TRY_DRAIN(hipMemcpyAsync(ds, reads + s0 * m, (size_t)(k * m), hipMemcpyHostToDevice, ctx->copy_stream));
        SS_TRY_DRAIN(hipMemcpyAsync(ds + side, refs + s0 * m, (size_t)(k * m), hipMemcpyHostToDevice, ctx->copy_stream));
        SS_TRY_DRAIN(hipEventRecord(ctx->ev_h2d[b], ctx->copy_stream));
        SS_TRY_DRAIN(hipStreamWaitEvent(s, ctx->ev_h2d[b], 0));
        const int rc = ss_filter_ascii_async(ctx, ds, ds + side, k, m, E, 0, d_res + s0, d_err, s);
        if (rc != SS_OK) return drain(rc);
        SS_TRY_DRAIN(hipEventRecord(ctx->ev_used[b], s));
    }
    uint8_t* hr = (uint8_t*)ctx->hres.p;
    SS_TRY_DRAIN(hipMemcpyAsync(hr, d_res, (size_t)n * 2, hipMemcpyDeviceToHost, s));
    SS_TRY_DRAIN(hipMemcpyAsync(hr + err_at, d_err, 4, hipMemcpyDeviceToHost, s));
    SS_TRY_DRAIN(hipStreamSynchronize(s));
#undef SS_TRY_DRAIN
    uint32_t h_err = 0;
    std::memcpy(&h_err, hr + err_at, 4);
    if (h_err & 2u) return SS_EDEVICE;   // a bounded wait inside the fused kernel gave up
    if (h_err) return SS_EBASE;          // outputs untouched
    const uint16_t* res = (const uint16_t*)hr;
    crew.parallel((size_t)n, [&](size_t a, size_t e) {
        for (size_t i = a; i < e; i++) {
            accept_out[i] = (uint8_t)(res[i] >> 15);
            edits_out[i] = (int32_t)(res[i] & SS_RESULT_COUNT);
        }
    });
    return SS_OK;
}

// Shared implementation: E_per_pair == nullptr means a single threshold E.
int filter_host(const uint8_t* reads, const uint8_t* refs, const int32_t* lengths, const int32_t* E_per_pair,
                int64_t n, int32_t E, uint8_t* accept_out, int32_t* edits_out)
{
    if (n < 0) return SS_EINVAL;
    if (n == 0) return SS_OK;
    if (!reads || !refs || !lengths || !accept_out || !edits_out) return SS_EINVAL;
    int32_t Emax = E;
    if (E_per_pair) {
        Emax = 0;
        for (int64_t i = 0; i < n; i++) {
            if (E_per_pair[i] < 0) return SS_EINVAL;
            Emax = std::max(Emax, E_per_pair[i]);
        }
    } else if (E < 0) {
        return SS_EINVAL;
    }
    if (Emax > SS_MAX_E) return SS_ELEN;
    std::vector<int64_t> off((size_t)n);
    int64_t total = 0;
    bool uniform = true;
    for (int64_t i = 0; i < n; i++) {
        const int32_t L = lengths[i];
        if (L < 0 || L > SS_MAX_LEN) return SS_ELEN;
        off[(size_t)i] = total;
        total += L;
        uniform = uniform && (L == lengths[0]);
    }

    ss_ctx* ctx = nullptr;
    int rc = ss_default_ctx(&ctx);
    if (rc != SS_OK) return rc;
    // the device's default context is shared by every host thread: one call at a time uses its buffers
    std::lock_guard<std::mutex> lk(ctx->host_mu);
    TraceRange tr("ss_filter_batch");
    if (uniform && !E_per_pair && E <= SS_MAX_E_SLICED && lengths[0] > 0 && lengths[0] <= SS_MAX_LEN_FUSED &&
        is_pinned_host(reads) && is_pinned_host(refs))
        return filter_host_pipelined(ctx, reads, refs, n, lengths[0], E, accept_out, edits_out);
    hipStream_t s = ctx->stream;
    // an error after work was enqueued returns once the stream has drained: its copies read the
    // caller's arrays (and the offsets built here) and write the context's buffers
    auto run = [&]() -> int {
        SS_TRY(ctx->reads.ensure((size_t)std::max<int64_t>(total, 1)));
        SS_TRY(ctx->refs.ensure((size_t)std::max<int64_t>(total, 1)));
        SS_TRY(ctx->results.ensure((size_t)n * 2 + 16));
        SS_TRY(ctx->err.ensure(16));
        uint32_t* d_err = (uint32_t*)ctx->err.p;
        uint16_t* d_res = (uint16_t*)ctx->results.p;
        if (total > 0) {
            SS_TRY(hipMemcpyAsync(ctx->reads.p, reads, (size_t)total, hipMemcpyHostToDevice, s));
            SS_TRY(hipMemcpyAsync(ctx->refs.p, refs, (size_t)total, hipMemcpyHostToDevice, s));
        }
        SS_TRY(hipMemsetAsync(d_err, 0, 4, s));

        const bool sliced = uniform && !E_per_pair && E <= SS_MAX_E_SLICED;
        if (sliced && lengths[0] <= SS_MAX_LEN_FUSED) {
            // encode and filter in one call; the alphabet check is read before any output is written
            rc = ss_filter_ascii_async(ctx, (const uint8_t*)ctx->reads.p, (const uint8_t*)ctx->refs.p, n, lengths[0],
                                       E, 0, d_res, d_err, s);
            if (rc != SS_OK) return rc;
        } else if (sliced) {
            const int32_t m = lengths[0];
            SS_TRY(ctx->packed.ensure((size_t)std::max<int64_t>(ss_sliced_bytes(n, m), 16)));
            rc = ss_pack_sliced_async(ctx, (const uint8_t*)ctx->reads.p, (const uint8_t*)ctx->refs.p, nullptr, nullptr,
                                      n, m, (uint32_t*)ctx->packed.p, d_err, s);
            if (rc != SS_OK) return rc;
        } else {
            SS_TRY(ctx->packed.ensure((size_t)ss_stream_words(total) * 16));
            SS_TRY(ctx->offsets.ensure((size_t)n * 8));
            SS_TRY(ctx->lengths.ensure((size_t)n * 4));
            SS_TRY(hipMemcpyAsync(ctx->offsets.p, off.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
            SS_TRY(hipMemcpyAsync(ctx->lengths.p, lengths, (size_t)n * 4, hipMemcpyHostToDevice, s));
            if (E_per_pair) {
                SS_TRY(ctx->epp.ensure((size_t)n * 4));
                SS_TRY(hipMemcpyAsync(ctx->epp.p, E_per_pair, (size_t)n * 4, hipMemcpyHostToDevice, s));
            }
            rc = ss_pack_stream_async(ctx, (const uint8_t*)ctx->reads.p, (const uint8_t*)ctx->refs.p, total,
                                      (uint32_t*)ctx->packed.p, d_err, s);
            if (rc != SS_OK) return rc;
        }
        uint32_t h_err = 0;
        SS_TRY(hipMemcpyAsync(&h_err, d_err, 4, hipMemcpyDeviceToHost, s));
        SS_TRY(hipStreamSynchronize(s));
        if (h_err & 2u) return SS_EDEVICE;   // a bounded wait inside the fused kernel gave up
        if (h_err) return SS_EBASE;

        if (sliced && lengths[0] <= SS_MAX_LEN_FUSED) {
            rc = SS_OK;     // filtered above
        } else if (sliced) {
            rc = ss_filter_sliced_async(ctx, (const uint32_t*)ctx->packed.p, n, lengths[0], E, d_res, s);
        } else {
            rc = ss_filter_wave_async(ctx, (const uint32_t*)ctx->packed.p, total, (const int64_t*)ctx->offsets.p,
                                      (const int32_t*)ctx->lengths.p, E_per_pair ? (const int32_t*)ctx->epp.p : nullptr,
                                      n, Emax, d_res, s);
        }
        if (rc != SS_OK) return rc;
        SS_TRY(ctx->hres.ensure((size_t)n * 2 + 16));
        const uint16_t* res = (const uint16_t*)ctx->hres.p;
        SS_TRY(hipMemcpyAsync(ctx->hres.p, d_res, (size_t)n * 2, hipMemcpyDeviceToHost, s));
        SS_TRY(hipStreamSynchronize(s));
        Crew crew(n >= (1 << 20) ? host_threads() : 1);
        crew.parallel((size_t)n, [&](size_t a, size_t e) {
            for (size_t i = a; i < e; i++) {
                accept_out[i] = (uint8_t)(res[i] >> 15);
                edits_out[i] = (int32_t)(res[i] & SS_RESULT_COUNT);
            }
        });
        return SS_OK;
    };
    rc = run();
    if (rc != SS_OK) (void)hipStreamSynchronize(s);
    return rc;
}

}  // namespace

extern "C" int ss_filter_batch(const uint8_t* reads, const uint8_t* refs, const int32_t* lengths, int64_t n_pairs,
                               int32_t E, uint8_t* accept_out, int32_t* edits_out)
{
    try {
        return filter_host(reads, refs, lengths, nullptr, n_pairs, E, accept_out, edits_out);
    } catch (const std::bad_alloc&) {
        return SS_ENOMEM;
    } catch (...) {
        return SS_EDEVICE;
    }
}

extern "C" int ss_filter_batch_var(const uint8_t* reads, const uint8_t* refs, const int32_t* lengths,
                                   const int32_t* E_per_pair, int64_t n_pairs, uint8_t* accept_out,
                                   int32_t* edits_out)
{
    if (n_pairs > 0 && !E_per_pair) return SS_EINVAL;
    try {
        return filter_host(reads, refs, lengths, E_per_pair, n_pairs, 0, accept_out, edits_out);
    } catch (const std::bad_alloc&) {
        return SS_ENOMEM;
    } catch (...) {
        return SS_EDEVICE;
    }
}
