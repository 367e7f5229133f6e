// Internal declarations shared by the kernel and host-runtime sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {

constexpr int kChunk = 4;              // positions per chunk in the lane-sliced layout
constexpr int kMaxESliced = 32;
constexpr int kMaxEPlain = 31;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---- launchers (all asynchronous on the given stream; return hipError_t) ----
hipError_t launch_pack_sliced(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets,
                              const int64_t* index, int64_t n_pairs, int32_t m, uint32_t* packed,
                              uint32_t* err, hipStream_t s);
hipError_t launch_sliced(const uint32_t* packed, int64_t n_pairs, int32_t m, int32_t E, uint16_t* out,
                         hipStream_t s);
hipError_t launch_pack_stream(const uint8_t* reads, const uint8_t* refs, int64_t total_bases,
                              uint32_t* packed, uint32_t* err, hipStream_t s);
hipError_t launch_plain(const uint32_t* packed, int64_t stream_words, const int64_t* offsets,
                        const int32_t* lengths, const int32_t* Epp, int64_t n, int32_t E, uint16_t* out,
                        hipStream_t s);
hipError_t launch_wave(const uint32_t* packed, int64_t stream_words, const int64_t* offsets,
                       const int32_t* lengths, const int32_t* Epp, int64_t n, int32_t E, uint16_t* out,
                       hipStream_t s);
hipError_t launch_unpack(const uint16_t* res, int64_t n, uint8_t* accept, int32_t* edits, hipStream_t s);

// Lanes per pair and row slices per lane chosen by the wavefront kernel for a
// given maximum threshold (rows 2E+1 are split in 32-row slices).
void wave_shape(int32_t E, int* lanes_per_pair, int* slices_per_lane);

}  // namespace ss
