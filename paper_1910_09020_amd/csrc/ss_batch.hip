// Batched launch for pairs of uneven lengths and per-pair thresholds: the
// kernels, plans on the device, graph capture and the autotuner (the host
// planner that cuts a batch into work items is ss_plan.cpp).
//
// Launch: one persistent kernel; each 256-thread block runs the wavefront
// sweep of ss_wave.h on the item of its own index, then on items popped from
// a device counter, until the queue is empty.  Every block exits once the
// counter passes the number of items, so the grid always drains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "ss.h"
#include "ss_common.h"
#include "ss_items.h"
#include "ss_trace.h"
#include "ss_wave.h"

namespace ss {

namespace {

__global__ void k_zero_counter(int* c) { if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0; }

template <int RSMAX>
__global__ __launch_bounds__(256) void k_persist(const PItem* __restrict__ items, int n_items, int* __restrict__ head,
                                                 const int64_t* __restrict__ perm, wave::GlobalPlanes planes,
                                                 const int64_t* __restrict__ offsets,
                                                 const int32_t* __restrict__ lengths,
                                                 const int32_t* __restrict__ Epp, uint16_t* __restrict__ out)
{
    __shared__ int s_item;
    __shared__ long long s_lo[4], s_hi[4];
    __shared__ uint32_t s_stage[4 * item_sweep::kStageWords];
    // The first item of a block is its own index (the grid starts on the
    // largest items without a round of atomics); later items are popped from
    // the counter, offset by the grid.  How those first items fall on the CUs
    // is the dispatcher's: it fills a CU's resident slots before the next
    // CU's, which is why the autotuner also tries two blocks per CU.
    int it = blockIdx.x;
    for (;;) {
        if (it >= n_items) break;
        // the item is the same for the whole block: keep its fields in scalar registers
        const int64_t first = items[it].first;
        const int count = __builtin_amdgcn_readfirstlane(items[it].count);
        const int LP = __builtin_amdgcn_readfirstlane(items[it].lp);
        const int rs = __builtin_amdgcn_readfirstlane(items[it].rs);
        const int emax = __builtin_amdgcn_readfirstlane(items[it].emax);
        item_sweep::sweep_item<RSMAX>(first, count, LP, rs, emax, perm, planes, offsets, lengths, Epp, out, s_lo, s_hi,
                                 s_stage);
        if (threadIdx.x == 0) s_item = (int)gridDim.x + atomicAdd(head, 1);
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
    }
}

}  // namespace

int persist_blocks_per_cu(int rsmax)
{
    int per_cu = 1;
    switch (rsmax) {
    case 1: (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<1>, 256, 0); break;
    case 2: (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<2>, 256, 0); break;
    case 4: (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<4>, 256, 0); break;
    default: (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<8>, 256, 0); break;
    }
    return per_cu < 1 ? 1 : per_cu;
}

hipError_t launch_persist_planes(int rsmax, int grid, const PItem* d_items, int n_items, int* d_head,
                                 const int64_t* d_perm, const uint32_t* qpk, int64_t SWq, const uint32_t* rpk,
                                 int64_t SWr, const int64_t* offsets, const int32_t* lengths, const int32_t* Epp,
                                 uint16_t* out, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    const wave::GlobalPlanes planes{qpk, rpk, SWq, SWr};
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, d_head);
#define SS_PERSIST(RS)                                                                                     \
    hipLaunchKernelGGL(k_persist<RS>, dim3(grid), dim3(256), 0, s, d_items, n_items, d_head, d_perm, planes, \
                       offsets, lengths, Epp, out)
    switch (rsmax) {
    case 1: SS_PERSIST(1); break;
    case 2: SS_PERSIST(2); break;
    case 4: SS_PERSIST(4); break;
    default: SS_PERSIST(8); break;
    }
#undef SS_PERSIST
    return hipGetLastError();
}

hipError_t launch_persist(int rsmax, int grid, const PItem* d_items, int n_items, int* d_head, const int64_t* d_perm,
                          const uint32_t* packed, int64_t total_bases, const int64_t* offsets, const int32_t* lengths,
                          const int32_t* Epp, uint16_t* out, hipStream_t s)
{
    const int64_t SW = cdiv(total_bases, 32) + 2;
    return launch_persist_planes(rsmax, grid, d_items, n_items, d_head, d_perm, packed, SW, packed + 2 * SW, SW,
                                 offsets, lengths, Epp, out, s);
}

}  // namespace ss

using namespace ss;

// Tunables chosen per plan.
struct PlanCfg {
    int rsmax = 8;          // slices per lane at most (1, 2, 4 or 8)
    int blocks_per_cu = 0;  // resident blocks per CU of the persistent grid (0: as many as fit)
};

struct ss_plan {
    int device = 0;
    int64_t n = 0;
    PlanCfg cfg;
    std::vector<PItem> items;
    std::vector<int64_t> perm;
    PItem* d_items = nullptr;
    int64_t* d_perm = nullptr;
    int* d_head = nullptr;
    int grid = 0;
    double est_cost = 0;
    int n_classes = 0;
    // captured launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int map_err(hipError_t e)
{
    if (e == hipSuccess) return SS_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SS_ENOMEM;
    return SS_EDEVICE;
}

int build_plan(ss_plan* P, const int32_t* lengths, const int32_t* E, int64_t n)
{
    return plan_items(lengths, E, n, P->cfg.rsmax, P->items, P->perm, &P->n_classes, &P->est_cost) ? SS_OK
                                                                                                     : SS_ELEN;
}

int upload_plan(ss_plan* P)
{
    hipError_t e;
    const size_t ib = std::max<size_t>(P->items.size(), 1) * sizeof(PItem);
    const size_t pb = std::max<size_t>(P->perm.size(), 1) * sizeof(int64_t);
    if ((e = hipMalloc(&P->d_items, ib)) != hipSuccess) return map_err(e);
    if ((e = hipMalloc(&P->d_perm, pb)) != hipSuccess) return map_err(e);
    if ((e = hipMalloc(&P->d_head, 256)) != hipSuccess) return map_err(e);
    if (!P->items.empty() &&
        (e = hipMemcpy(P->d_items, P->items.data(), P->items.size() * sizeof(PItem), hipMemcpyHostToDevice)) != hipSuccess)
        return map_err(e);
    if (!P->perm.empty() &&
        (e = hipMemcpy(P->d_perm, P->perm.data(), P->perm.size() * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess)
        return map_err(e);
    // persistent grid: resident blocks per CU x CUs, no more blocks than items
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return map_err(e);
    int per_cu = persist_blocks_per_cu(P->cfg.rsmax);
    if (P->cfg.blocks_per_cu > 0) per_cu = std::min(per_cu, P->cfg.blocks_per_cu);
    P->grid = (int)std::min<int64_t>((int64_t)per_cu * prop.multiProcessorCount, std::max<size_t>(P->items.size(), 1));
    return SS_OK;
}

void free_plan(ss_plan* P)
{
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->d_items) (void)hipFree(P->d_items);
    if (P->d_perm) (void)hipFree(P->d_perm);
    if (P->d_head) (void)hipFree(P->d_head);
    P->exec = nullptr; P->graph = nullptr; P->d_items = nullptr; P->d_perm = nullptr; P->d_head = nullptr;
}

hipError_t enqueue(const ss_plan* P, const uint32_t* packed, int64_t total_bases, const int64_t* offsets,
                   const int32_t* lengths, const int32_t* Epp, uint16_t* out, hipStream_t s)
{
    return launch_persist(P->cfg.rsmax, P->grid, P->d_items, (int)P->items.size(), P->d_head, P->d_perm, packed,
                          total_bases, offsets, lengths, Epp, out, s);
}

int make_plan(const PlanCfg& cfg, const int32_t* lengths, const int32_t* E, int64_t n, ss_plan** out)
{
    ss_plan* P = new (std::nothrow) ss_plan();
    if (!P) return SS_ENOMEM;
    (void)hipGetDevice(&P->device);
    P->n = n;
    P->cfg = cfg;
    int rc = build_plan(P, lengths, E, n);
    if (rc == SS_OK) rc = upload_plan(P);
    if (rc != SS_OK) {
        free_plan(P);
        delete P;
        return rc;
    }
    *out = P;
    return SS_OK;
}

}  // namespace

extern "C" int ss_plan_create(ss_ctx* ctx, const int32_t* lengths, const int32_t* E_per_pair, int64_t n_pairs,
                              int32_t slices_per_lane, ss_plan** out)
{
    if (!ctx || !out) return SS_EINVAL;
    if (slices_per_lane != 1 && slices_per_lane != 2 && slices_per_lane != 4 && slices_per_lane != 8) return SS_EINVAL;
    int rc = validate_plan_inputs(lengths, E_per_pair, n_pairs);
    if (rc != SS_OK) return rc;
    const int rsmin = plan_min_slices(E_per_pair, n_pairs);
    if (rsmin == 0) return SS_ELEN;
    PlanCfg cfg;
    cfg.rsmax = std::max<int>(slices_per_lane, rsmin);
    try {
        return make_plan(cfg, lengths, E_per_pair, n_pairs, out);
    } catch (const std::bad_alloc&) {
        return SS_ENOMEM;
    }
}

extern "C" int ss_plan_destroy(ss_plan* plan)
{
    if (!plan) return SS_EINVAL;
    free_plan(plan);
    delete plan;
    return SS_OK;
}

extern "C" int ss_plan_info(const ss_plan* plan, int64_t* n_items, int32_t* n_classes, int32_t* grid,
                            int32_t* slices_per_lane)
{
    if (!plan) return SS_EINVAL;
    if (n_items) *n_items = (int64_t)plan->items.size();
    if (n_classes) *n_classes = plan->n_classes;
    if (grid) *grid = plan->grid;
    if (slices_per_lane) *slices_per_lane = plan->cfg.rsmax;
    return SS_OK;
}

namespace ss {
// A plan's launch over the two sides packed apart (used by ss_filter_batch_ex).
hipError_t plan_enqueue_planes(const ss_plan* P, const uint32_t* qpk, int64_t SWq, const uint32_t* rpk, int64_t SWr,
                               const int64_t* offsets, const int32_t* lengths, const int32_t* Epp, uint16_t* out,
                               hipStream_t s)
{
    return launch_persist_planes(P->cfg.rsmax, P->grid, P->d_items, (int)P->items.size(), P->d_head, P->d_perm, qpk,
                                 SWq, rpk, SWr, offsets, lengths, Epp, out, s);
}

int64_t plan_pairs(const ss_plan* P) { return P->n; }
int plan_device(const ss_plan* P) { return P->device; }
int32_t plan_max_e(const ss_plan* P)
{
    int32_t e = 0;
    for (const PItem& it : P->items) e = std::max(e, it.emax);
    return e;
}
}  // namespace ss

extern "C" int ss_filter_planned_async(ss_ctx* ctx, const ss_plan* plan, const uint32_t* packed, int64_t total_bases,
                                       const int64_t* offsets, const int32_t* lengths, const int32_t* E_per_pair,
                                       uint16_t* out, void* stream)
{
    if (!ctx || !plan || total_bases < 0) return SS_EINVAL;
    if (total_bases > SS_MAX_STREAM_BASES) return SS_ELEN;
    if (plan->n == 0) return SS_OK;
    if (!packed || !offsets || !lengths || !E_per_pair || !out) return SS_EINVAL;
    return map_err(enqueue(plan, packed, total_bases, offsets, lengths, E_per_pair, out, (hipStream_t)stream));
}

// Capture the planned launch (counter reset + persistent kernel) into a HIP
// graph bound to these device buffers; ss_plan_launch replays it.
extern "C" int ss_plan_capture(ss_ctx* ctx, ss_plan* plan, const uint32_t* packed, int64_t total_bases,
                               const int64_t* offsets, const int32_t* lengths, const int32_t* E_per_pair,
                               uint16_t* out)
{
    if (!ctx || !plan || total_bases < 0) return SS_EINVAL;
    if (total_bases > SS_MAX_STREAM_BASES) return SS_ELEN;
    if (plan->n > 0 && (!packed || !offsets || !lengths || !E_per_pair || !out)) return SS_EINVAL;
    if (plan->exec) { (void)hipGraphExecDestroy(plan->exec); plan->exec = nullptr; }
    if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return map_err(e);
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = enqueue(plan, packed, total_bases, offsets, lengths, E_per_pair, out, s);
        e = hipStreamEndCapture(s, &plan->graph);
        if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(s);
    return map_err(e);
}

extern "C" int ss_plan_launch(ss_plan* plan, void* stream)
{
    if (!plan) return SS_EINVAL;
    if (plan->n == 0) return SS_OK;
    if (!plan->exec) return SS_EINVAL;
    return map_err(hipGraphLaunch(plan->exec, (hipStream_t)stream));
}

// ---------------------------------------------------------------- autotuner
// Candidate configurations are timed on the batch itself (two launches each,
// the faster counts): every slice width, each with the grid at as many
// resident blocks per CU as fit and at two.  The work-group dispatcher fills
// a CU's slots before the next CU's, so with three or more slots the first
// (largest) items can land three to a CU and run a third as fast; two slots
// avoid that for batches led by a few long pairs, while batches of short
// pairs gain from the extra wavefronts.  The winner is stored in a JSON cache
// keyed by device architecture and a coarse signature of the batch (pair
// count, length and threshold ranges) as slices + 100 x blocks per CU, so
// later plans for similar batches skip the timing.
namespace {

std::string signature(const char* arch, const int32_t* lengths, const int32_t* E, int64_t n)
{
    int32_t mlo = INT32_MAX, mhi = 0, elo = INT32_MAX, ehi = 0;
    for (int64_t i = 0; i < n; i++) {
        mlo = std::min(mlo, lengths[i]); mhi = std::max(mhi, lengths[i]);
        elo = std::min(elo, E[i]); ehi = std::max(ehi, E[i]);
    }
    auto lg = [](int64_t v) { int b = 0; while (v > 1) { v >>= 1; b++; } return b; };
    std::ostringstream os;
    os << arch << "|n2^" << lg(n) << "|m2^" << lg(mlo) << "-2^" << lg(mhi) << "|E2^" << lg(elo + 1) << "-2^" << lg(ehi + 1);
    return os.str();
}

// Minimal "key": value reader/writer for a flat JSON object of integers.
std::map<std::string, int> read_cache(const std::string& path)
{
    std::map<std::string, int> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        const size_t c = s.find(':', j);
        if (c == std::string::npos) break;
        m[key] = std::atoi(s.c_str() + c + 1);
        i = s.find_first_of(",}", c);
        if (i == std::string::npos) break;
    }
    return m;
}

void write_cache(const std::string& path, const std::map<std::string, int>& m)
{
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        f << "{\n";
        size_t k = 0;
        for (auto& kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
        f << "}\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

std::mutex g_cache_mu;

}  // namespace

extern "C" int ss_plan_create_tuned(ss_ctx* ctx, const int32_t* lengths, const int32_t* E_per_pair, int64_t n_pairs,
                                    const uint32_t* packed, int64_t total_bases, const int64_t* offsets_dev,
                                    const int32_t* lengths_dev, const int32_t* E_dev, uint16_t* out_dev,
                                    const char* cache_path, ss_plan** out, int32_t* chosen_slices)
{
    TraceRange tr("plan: autotune");
    if (!ctx || !out) return SS_EINVAL;
    int rc = validate_plan_inputs(lengths, E_per_pair, n_pairs);
    if (rc != SS_OK) return rc;
    if (n_pairs > 0 && (!packed || !offsets_dev || !lengths_dev || !E_dev || !out_dev)) return SS_EINVAL;
    if (total_bases < 0) return SS_EINVAL;
    if (total_bases > SS_MAX_STREAM_BASES) return SS_ELEN;
    const int rsmin = plan_min_slices(E_per_pair, n_pairs);
    if (rsmin == 0) return SS_ELEN;
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return SS_EDEVICE;
    const std::string key = signature(prop.gcnArchName, lengths, E_per_pair, n_pairs);
    try {
        if (cache_path && *cache_path) {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto m = read_cache(cache_path);
            auto it = m.find(key);
            const int sl = it != m.end() ? it->second % 100 : 0, bpc = it != m.end() ? it->second / 100 : 0;
            if (it != m.end() && (sl == 1 || sl == 2 || sl == 4 || sl == 8) && bpc >= 0 && bpc <= 64) {
                PlanCfg cfg;
                cfg.rsmax = std::max<int>(sl, rsmin);
                cfg.blocks_per_cu = bpc;
                if (chosen_slices) *chosen_slices = cfg.rsmax;
                return make_plan(cfg, lengths, E_per_pair, n_pairs, out);
            }
        }
        const int cands[4] = {1, 2, 4, 8};
        float best_ms = 1e30f;
        int best = 8, best_bpc = 0;
        hipStream_t s = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return map_err(e);
        hipEvent_t a = nullptr, b = nullptr;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        for (int c : cands) {
            if (c < rsmin) continue;        // too narrow for the largest threshold
            PlanCfg cfg;
            cfg.rsmax = c;
            ss_plan* P = nullptr;
            rc = make_plan(cfg, lengths, E_per_pair, n_pairs, &P);
            if (rc != SS_OK) break;
            // the same plan at both grids (the grid is a launch parameter only)
            const int full_grid = P->grid;
            const int two_grid = (int)std::min<int64_t>(2 * (int64_t)prop.multiProcessorCount, full_grid);
            for (int g = 0; g < 2 && rc == SS_OK; g++) {
                if (g == 1 && two_grid == full_grid) break;
                P->grid = g == 0 ? full_grid : two_grid;
                float ms = 1e30f;
                for (int rep = 0; rep < 2 && rc == SS_OK; rep++) {
                    (void)hipEventRecord(a, s);
                    e = enqueue(P, packed, total_bases, offsets_dev, lengths_dev, E_dev, out_dev, s);
                    (void)hipEventRecord(b, s);
                    if (e == hipSuccess) e = hipEventSynchronize(b);
                    float t = 0;
                    if (e == hipSuccess) (void)hipEventElapsedTime(&t, a, b);
                    else rc = map_err(e);
                    ms = std::min(ms, t);
                }
                if (rc == SS_OK && ms < best_ms) { best_ms = ms; best = c; best_bpc = g == 0 ? 0 : 2; }
            }
            free_plan(P);
            delete P;
            if (rc != SS_OK) break;
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        (void)hipStreamDestroy(s);
        if (rc != SS_OK) return rc;
        if (cache_path && *cache_path) {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto m = read_cache(cache_path);
            m[key] = best + 100 * best_bpc;
            write_cache(cache_path, m);
        }
        PlanCfg cfg;
        cfg.rsmax = best;
        cfg.blocks_per_cu = best_bpc;
        if (chosen_slices) *chosen_slices = best;
        return make_plan(cfg, lengths, E_per_pair, n_pairs, out);
    } catch (const std::bad_alloc&) {
        return SS_ENOMEM;
    }
}
