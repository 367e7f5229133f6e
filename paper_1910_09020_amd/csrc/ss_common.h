// Internal declarations shared by the kernel and host-runtime sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

typedef struct ss_plan ss_plan;

namespace ss {

constexpr int kChunk = 4;              // positions per chunk in the lane-sliced layout
constexpr int kMaxESliced = 32;
constexpr int kMaxEPlain = 31;
constexpr int kMaxEFused = 10;                 // fused encode + sweep kernel (larger E: chunked two kernels)
constexpr int64_t kMaxFusedLds = 160 * 1024;   // LDS per workgroup on gfx950

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }


// ---- launchers (all asynchronous on the given stream; return hipError_t) ----
hipError_t launch_pack_sliced(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets,
                              const int64_t* index, int64_t n_pairs, int32_t m, uint32_t* packed,
                              uint32_t* err, hipStream_t s);
// sub_width > 0: Snake-on-Chip sub-mazes of that many columns (Section 2.5)
hipError_t launch_sliced(const uint32_t* packed, int64_t n_pairs, int32_t m, int32_t E, uint16_t* out,
                         hipStream_t s, int sub_width = 0);
// Several thresholds in one pass: sliced_multi_span(E) thresholds from E (0 when no pass starts
// at E); launch_sliced_multi_group writes threshold E+k's results at out + k * out_stride.
int sliced_multi_span(int E_first);
hipError_t launch_sliced_multi_group(int E_first, const uint32_t* packed, int64_t n_pairs, int32_t m, uint16_t* out,
                                     int64_t out_stride, hipStream_t s);
// Fused encode + sweep of pairs stored back to back (pair i at byte i*m).
// tile_groups: groups of 32 pairs per block (0: automatic).
hipError_t launch_fused(const uint8_t* reads, const uint8_t* refs, int64_t n_pairs, int32_t m, int32_t E,
                        int tile_groups, uint16_t* out, uint32_t* err, hipStream_t s);
// max_t caps the automatic tile (tile_groups = 0); fused_tile_cap gives the cap
// that leaves no CU without a tile for a batch of n_pairs.
size_t fused_shape(int32_t m, int tile_groups, bool contiguous, int* T, int* GB, int* U, int max_t = 256);
int fused_tile_cap(int64_t n_pairs);
hipError_t launch_pack_stream(const uint8_t* reads, const uint8_t* refs, int64_t total_bases,
                              uint32_t* packed, uint32_t* err, hipStream_t s);
// One side (reads or refs) into two planes of cdiv(total_bases, 32) + 2 words.
hipError_t launch_pack_side(const uint8_t* ascii, int64_t total_bases, uint32_t* packed, uint32_t* err, hipStream_t s);
// The wavefront sweep over two sides packed apart (launch_pack_side): query i is
// qlen[i] bases from bit qoff[i] of qpk, reference i rlen[i] bases from bit
// roff[i] of rpk; any lengths (unequal lengths walk the columns that hold a
// real comparison).
hipError_t launch_wave_sides(const uint32_t* qpk, int64_t q_words, const uint32_t* rpk, int64_t r_words,
                             const int64_t* qoff, const int32_t* qlen, const int64_t* roff, const int32_t* rlen,
                             const int32_t* Epp, int64_t n, int32_t E, uint16_t* out, hipStream_t s);
// The one-pair-per-lane walk over the two sides packed apart (pairs of equal
// length at common offsets).
hipError_t launch_plain_sides(const uint32_t* qpk, int64_t q_words, const uint32_t* rpk, int64_t r_words,
                              const int64_t* offsets, const int32_t* lengths, const int32_t* Epp, int64_t n,
                              int32_t E, uint16_t* out, hipStream_t s);
hipError_t launch_plain(const uint32_t* packed, int64_t stream_words, const int64_t* offsets,
                        const int32_t* lengths, const int32_t* Epp, int64_t n, int32_t E, uint16_t* out,
                        hipStream_t s);
hipError_t launch_wave(const uint32_t* packed, int64_t stream_words, const int64_t* offsets,
                       const int32_t* lengths, const int32_t* Epp, int64_t n, int32_t E, uint16_t* out,
                       hipStream_t s);
// Verification: exact edit distance of the listed pairs (bit-stream layout, m <= 256), and the
// compaction of accepted pairs' indices.
// Banded edit distance (E_per_pair may be null: E for every pair; else E >= every entry).
hipError_t launch_verify_banded(const uint32_t* packed, int64_t stream_words, const int64_t* offsets,
                                const int32_t* lengths, const int32_t* E_per_pair, int32_t E, const int64_t* index,
                                int64_t n, int32_t* ed_out, hipStream_t s);
hipError_t launch_verify(const uint32_t* packed, int64_t stream_words, const int64_t* offsets, const int32_t* lengths,
                         const int64_t* index, int64_t n, int32_t max_len, int32_t* ed_out, hipStream_t s);
hipError_t launch_select(const uint16_t* results, int64_t n, int64_t* index_out, unsigned long long* count,
                         hipStream_t s);
hipError_t launch_unpack(const uint16_t* res, int64_t n, uint8_t* accept, int32_t* edits, hipStream_t s);

// Lanes per pair and row slices per lane chosen by the wavefront kernel for a
// given maximum threshold (rows 2E+1 are split in 32-row slices).
void wave_shape(int32_t E, int* lanes_per_pair, int* slices_per_lane);

// ---- batched launch (work items of the persistent kernel) ----
struct PItem {
    int64_t first;    // first slot in the permutation
    int32_t count;    // pairs in this item
    int16_t lp;       // lanes per pair
    int16_t rs;       // slices per lane
    int32_t emax;     // row layout threshold (max E over the item's pairs)
    int32_t pad;
};
static_assert(sizeof(PItem) == 24, "PItem layout");

// Host planner: shape classes, sort, items ordered largest estimated cost first.
// false (and no items) when some pair's rows do not fit 64 lanes x rsmax slices.
bool plan_items(const int32_t* lengths, const int32_t* E, int64_t n, int rsmax, std::vector<PItem>& items,
                std::vector<int64_t>& perm, int* n_classes, double* est_cost);
// Smallest slice width (1, 2, 4 or 8) whose 64 lanes hold the 2E+1 rows of
// every pair, or 0 when some E needs more than 8 (E > 8191).
int plan_min_slices(const int32_t* E, int64_t n);
// SS_EINVAL / SS_ELEN for negative or oversized lengths and thresholds, else SS_OK.
int validate_plan_inputs(const int32_t* lengths, const int32_t* E, int64_t n);
// Resident blocks per CU of the persistent kernel for this slice width.
int persist_blocks_per_cu(int rsmax);
// Counter reset + persistent kernel on stream s.
// The same over the two sides packed apart (launch_pack_side).
hipError_t launch_persist_planes(int rsmax, int grid, const PItem* d_items, int n_items, int* d_head,
                                 const int64_t* d_perm, const uint32_t* qpk, int64_t SWq, const uint32_t* rpk,
                                 int64_t SWr, const int64_t* offsets, const int32_t* lengths, const int32_t* Epp,
                                 uint16_t* out, hipStream_t s);
hipError_t launch_persist(int rsmax, int grid, const PItem* d_items, int n_items, int* d_head, const int64_t* d_perm,
                          const uint32_t* packed, int64_t total_bases, const int64_t* offsets, const int32_t* lengths,
                          const int32_t* Epp, uint16_t* out, hipStream_t s);

// A plan's persistent launch over the two sides packed apart, and what a plan
// was made for (ss_batch.hip).
hipError_t plan_enqueue_planes(const ss_plan* P, const uint32_t* qpk, int64_t SWq, const uint32_t* rpk, int64_t SWr,
                               const int64_t* offsets, const int32_t* lengths, const int32_t* Epp, uint16_t* out,
                               hipStream_t s);
int64_t plan_pairs(const ss_plan* P);
int plan_device(const ss_plan* P);
int32_t plan_max_e(const ss_plan* P);

}  // namespace ss
