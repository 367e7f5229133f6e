// The batch-descriptor boundary: ss_pack (one side to 2-bit planes),
// ss_filter_batch_ex (one call, any input form, the kernel chosen by the
// pairs' shape or by the caller) and ss_filter_batch_pairs (the host one-call
// form for pairs of unequal length).  Arguments are validated here; every step
// of the filter runs in the kernels of the other sources.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <new>
#include <vector>

#include "ss.h"
#include "ss_common.h"
#include "ss_ctx.h"

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

// offsets and lengths of n pairs of m bases stored back to back
__global__ __launch_bounds__(256) void k_fill_uniform(int64_t* __restrict__ off, int32_t* __restrict__ len, int64_t n,
                                                      int32_t m)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    off[i] = i * (int64_t)m;
    len[i] = m;
}

struct Sides {
    const uint32_t* q;
    const uint32_t* r;
    int64_t SWq, SWr;
};

}  // namespace

extern "C" int64_t ss_pack_words(int64_t bases)
{
    if (bases < 0) return -1;
    return 2 * (cdiv(bases, 32) + 2);
}

extern "C" int ss_pack(ss_ctx* ctx, const uint8_t* ascii, int64_t bases, uint32_t* packed, uint32_t* err,
                       void* stream)
{
    if (!ctx || bases < 0 || !packed) return SS_EINVAL;
    if (bases > SS_MAX_STREAM_BASES) return SS_ELEN;
    if (bases > 0 && !ascii) return SS_EINVAL;
    return map_err(launch_pack_side(ascii, bases, packed, err, (hipStream_t)stream));
}

extern "C" int ss_filter_batch_ex(ss_ctx* ctx, const ss_batch_desc* d, void* stream)
{
    if (!ctx || !d) return SS_EINVAL;
    const uint32_t input = d->flags & SS_INPUT_MASK, kernel = d->flags & SS_KERNEL_MASK;
    if ((d->flags & ~(SS_INPUT_MASK | SS_KERNEL_MASK)) != 0 || d->reserved != 0) return SS_EINVAL;
    if (input > SS_INPUT_PACKED_SLICED || kernel > SS_KERNEL_PERSISTENT) return SS_EINVAL;
    if (d->n_pairs < 0 || d->E < 0 || d->read_bases < 0 || d->ref_bases < 0 || d->length < -1) return SS_EINVAL;
    if (d->E > SS_MAX_E || d->length > SS_MAX_LEN) return SS_ELEN;
    if (d->n_pairs == 0) return SS_OK;
    const bool uniform = d->length >= 0;
    const bool uneq = d->ref_lengths != nullptr || d->ref_offsets != nullptr;
    const bool per_pair = d->E_per_pair != nullptr;
    if (!d->out || !d->reads) return SS_EINVAL;
    if (input != SS_INPUT_PACKED_SLICED && !d->refs) return SS_EINVAL;
    if (!uniform && (!d->lengths || !d->offsets)) return SS_EINVAL;
    if ((d->ref_lengths == nullptr) != (d->ref_offsets == nullptr)) return SS_EINVAL;
    if (input == SS_INPUT_ASCII && !d->err) return SS_EINVAL;
    if (((uintptr_t)d->out & 15u) != 0) return SS_EINVAL;
    const hipStream_t s = (hipStream_t)stream;

    // the kernel: the caller's, or by the pairs' shape (one length and one threshold: the lane-sliced
    // sweep, fused with the encoding for ASCII stored back to back; a plan: its persistent launch;
    // anything else: the wavefront kernel)
    uint32_t k = kernel;
    if (k == SS_KERNEL_AUTO) {
        if (input == SS_INPUT_PACKED_SLICED)
            k = SS_KERNEL_SLICED;
        else if (d->plan)
            k = SS_KERNEL_PERSISTENT;
        else if (input == SS_INPUT_ASCII && uniform && !uneq && !per_pair && d->E <= SS_MAX_E_SLICED)
            k = (!d->offsets && d->length <= SS_MAX_LEN_FUSED) ? SS_KERNEL_FUSED : SS_KERNEL_SLICED;
        else
            k = SS_KERNEL_WAVE;
    }
    const bool one_shape = uniform && !uneq && !per_pair;

    if (k == SS_KERNEL_FUSED) {
        if (input != SS_INPUT_ASCII || !one_shape || d->offsets) return SS_EINVAL;
        if (d->E > SS_MAX_E_SLICED || d->length > SS_MAX_LEN_FUSED) return SS_ELEN;
        return ss_filter_ascii_async(ctx, (const uint8_t*)d->reads, (const uint8_t*)d->refs, d->n_pairs, d->length,
                                     d->E, 0, d->out, d->err, stream);
    }
    if (k == SS_KERNEL_SLICED) {
        if (!one_shape) return SS_EINVAL;
        if (d->E > SS_MAX_E_SLICED) return SS_ELEN;
        if (input == SS_INPUT_PACKED_SLICED)
            return ss_filter_sliced_async(ctx, (const uint32_t*)d->reads, d->n_pairs, d->length, d->E, d->out, stream);
        if (input != SS_INPUT_ASCII) return SS_EINVAL;   // bit streams are not in the lane-sliced layout
        const int64_t bytes = ss_sliced_bytes(d->n_pairs, d->length);
        SS_TRY(ctx->chunk.ensure((size_t)std::max<int64_t>(bytes, 16)));
        int rc = ss_pack_sliced_async(ctx, (const uint8_t*)d->reads, (const uint8_t*)d->refs, d->offsets, nullptr,
                                      d->n_pairs, d->length, (uint32_t*)ctx->chunk.p, d->err, stream);
        if (rc != SS_OK) return rc;
        return ss_filter_sliced_async(ctx, (const uint32_t*)ctx->chunk.p, d->n_pairs, d->length, d->E, d->out, stream);
    }
    if (input == SS_INPUT_PACKED_SLICED) return SS_EINVAL;

    // the remaining kernels read the two sides as bit streams; every check comes before any work
    if (d->read_bases > SS_MAX_STREAM_BASES || d->ref_bases > SS_MAX_STREAM_BASES) return SS_ELEN;
    if (uniform && !d->offsets && d->length > 0) {
        // pairs back to back at i * length must lie inside the bases the caller declared
        // (n_pairs * length <= bases, compared by division: the product may not fit)
        if (d->n_pairs > d->read_bases / d->length || (!uneq && d->n_pairs > d->ref_bases / d->length))
            return SS_EINVAL;
    }
    if (k == SS_KERNEL_PLAIN) {
        if (uneq) return SS_EINVAL;                  // one length per pair
        if (d->E > SS_MAX_E_PLAIN) return SS_ELEN;
    }
    if (k == SS_KERNEL_PERSISTENT) {
        if (!d->plan || uneq || !per_pair) return SS_EINVAL;
        if (plan_pairs(d->plan) != d->n_pairs || plan_device(d->plan) != ctx->device) return SS_EINVAL;
    }
    Sides sd;
    sd.SWq = cdiv(d->read_bases, 32) + 2;
    sd.SWr = cdiv(d->ref_bases, 32) + 2;
    if (input == SS_INPUT_ASCII) {
        SS_TRY(ctx->qside.ensure((size_t)(2 * sd.SWq) * 4));
        SS_TRY(ctx->rside.ensure((size_t)(2 * sd.SWr) * 4));
        SS_TRY(launch_pack_side((const uint8_t*)d->reads, d->read_bases, (uint32_t*)ctx->qside.p, d->err, s));
        SS_TRY(launch_pack_side((const uint8_t*)d->refs, d->ref_bases, (uint32_t*)ctx->rside.p, d->err, s));
        sd.q = (const uint32_t*)ctx->qside.p;
        sd.r = (const uint32_t*)ctx->rside.p;
    } else {
        sd.q = (const uint32_t*)d->reads;
        sd.r = (const uint32_t*)d->refs;
    }
    const int64_t* off = d->offsets;
    const int32_t* len = d->lengths;
    if (!off || !len) {
        // pairs of one length back to back: the kernels read offsets and lengths per pair
        SS_TRY(ctx->uoff.ensure((size_t)d->n_pairs * 8));
        SS_TRY(ctx->ulen.ensure((size_t)d->n_pairs * 4));
        hipLaunchKernelGGL(k_fill_uniform, dim3((unsigned)cdiv(d->n_pairs, 256)), dim3(256), 0, s,
                           (int64_t*)ctx->uoff.p, (int32_t*)ctx->ulen.p, d->n_pairs, d->length);
        SS_TRY(hipGetLastError());
        off = off ? off : (const int64_t*)ctx->uoff.p;
        len = len ? len : (const int32_t*)ctx->ulen.p;
    }

    if (k == SS_KERNEL_PLAIN) {
        return map_err(launch_plain_sides(sd.q, sd.SWq, sd.r, sd.SWr, off, len, d->E_per_pair, d->n_pairs, d->E,
                                          d->out, s));
    }
    if (k == SS_KERNEL_WAVE) {
        const int64_t* roff = d->ref_offsets ? d->ref_offsets : off;
        const int32_t* rlen = d->ref_lengths ? d->ref_lengths : len;
        return map_err(launch_wave_sides(sd.q, sd.SWq, sd.r, sd.SWr, off, len, roff, rlen, d->E_per_pair, d->n_pairs,
                                         d->E, d->out, s));
    }
    // SS_KERNEL_PERSISTENT
    return map_err(plan_enqueue_planes(d->plan, sd.q, sd.SWq, sd.r, sd.SWr, off, len, d->E_per_pair, d->out, s));
}

// ---------------------------------------------------------------- host one-call for unequal lengths
extern "C" int ss_filter_batch_pairs(const uint8_t* reads, const int32_t* read_lengths, const uint8_t* refs,
                                     const int32_t* ref_lengths, int64_t n_pairs, const int32_t* E_per_pair, int32_t E,
                                     uint8_t* accept_out, int32_t* edits_out)
{
    try {
        if (n_pairs < 0) return SS_EINVAL;
        if (n_pairs == 0) return SS_OK;
        if (!reads || !refs || !read_lengths || !ref_lengths || !accept_out || !edits_out) return SS_EINVAL;
        int32_t Emax = E;
        if (E_per_pair) {
            Emax = 0;
            for (int64_t i = 0; i < n_pairs; i++) {
                if (E_per_pair[i] < 0) return SS_EINVAL;
                Emax = std::max(Emax, E_per_pair[i]);
            }
        } else if (E < 0) {
            return SS_EINVAL;
        }
        if (Emax > SS_MAX_E) return SS_ELEN;
        const size_t n = (size_t)n_pairs;
        std::vector<int64_t> qoff(n), roff(n);
        int64_t qt = 0, rt = 0;
        for (size_t i = 0; i < n; i++) {
            if (read_lengths[i] < 0 || ref_lengths[i] < 0) return SS_EINVAL;
            if (read_lengths[i] > SS_MAX_LEN || ref_lengths[i] > SS_MAX_LEN) return SS_ELEN;
            qoff[i] = qt;
            roff[i] = rt;
            qt += read_lengths[i];
            rt += ref_lengths[i];
        }
        if (qt > SS_MAX_STREAM_BASES || rt > SS_MAX_STREAM_BASES) return SS_ELEN;

        ss_ctx* ctx = nullptr;
        int rc = ss_default_ctx(&ctx);
        if (rc != SS_OK) return rc;
        std::lock_guard<std::mutex> lk(ctx->host_mu);
        const hipStream_t s = ctx->stream;
        SS_TRY(ctx->reads.ensure((size_t)std::max<int64_t>(qt, 1)));
        SS_TRY(ctx->refs.ensure((size_t)std::max<int64_t>(rt, 1)));
        SS_TRY(ctx->offsets.ensure(n * 8));
        SS_TRY(ctx->lengths.ensure(n * 4));
        SS_TRY(ctx->roff.ensure(n * 8));
        SS_TRY(ctx->rlen.ensure(n * 4));
        SS_TRY(ctx->results.ensure(n * 2 + 16));
        SS_TRY(ctx->err.ensure(16));
        if (E_per_pair) SS_TRY(ctx->epp.ensure(n * 4));
        if (qt) SS_TRY(hipMemcpyAsync(ctx->reads.p, reads, (size_t)qt, hipMemcpyHostToDevice, s));
        if (rt) SS_TRY(hipMemcpyAsync(ctx->refs.p, refs, (size_t)rt, hipMemcpyHostToDevice, s));
        SS_TRY(hipMemcpyAsync(ctx->offsets.p, qoff.data(), n * 8, hipMemcpyHostToDevice, s));
        SS_TRY(hipMemcpyAsync(ctx->lengths.p, read_lengths, n * 4, hipMemcpyHostToDevice, s));
        SS_TRY(hipMemcpyAsync(ctx->roff.p, roff.data(), n * 8, hipMemcpyHostToDevice, s));
        SS_TRY(hipMemcpyAsync(ctx->rlen.p, ref_lengths, n * 4, hipMemcpyHostToDevice, s));
        if (E_per_pair) SS_TRY(hipMemcpyAsync(ctx->epp.p, E_per_pair, n * 4, hipMemcpyHostToDevice, s));
        SS_TRY(hipMemsetAsync(ctx->err.p, 0, 4, s));
        ss_batch_desc d{};
        d.reads = ctx->reads.p;
        d.refs = ctx->refs.p;
        d.offsets = (const int64_t*)ctx->offsets.p;
        d.lengths = (const int32_t*)ctx->lengths.p;
        d.ref_offsets = (const int64_t*)ctx->roff.p;
        d.ref_lengths = (const int32_t*)ctx->rlen.p;
        d.E_per_pair = E_per_pair ? (const int32_t*)ctx->epp.p : nullptr;
        d.n_pairs = n_pairs;
        d.read_bases = qt;
        d.ref_bases = rt;
        d.length = -1;
        d.E = Emax;
        d.flags = SS_INPUT_ASCII | SS_KERNEL_WAVE;
        d.out = (uint16_t*)ctx->results.p;
        d.err = (uint32_t*)ctx->err.p;
        rc = ss_filter_batch_ex(ctx, &d, s);
        if (rc != SS_OK) return rc;
        std::vector<uint16_t> res(n);
        uint32_t h_err = 0;
        SS_TRY(hipMemcpyAsync(&h_err, ctx->err.p, 4, hipMemcpyDeviceToHost, s));
        SS_TRY(hipMemcpyAsync(res.data(), ctx->results.p, n * 2, hipMemcpyDeviceToHost, s));
        SS_TRY(hipStreamSynchronize(s));
        if (h_err) return SS_EBASE;     // outputs untouched
        for (size_t i = 0; i < n; i++) {
            accept_out[i] = (uint8_t)(res[i] >> 15);
            edits_out[i] = (int32_t)(res[i] & SS_RESULT_COUNT);
        }
        return SS_OK;
    } catch (const std::bad_alloc&) {
        return SS_ENOMEM;
    } catch (...) {
        return SS_EDEVICE;
    }
}
