// Column-sweep kernels for thresholds E = 11..20 and fused encode-and-sweep kernels for E = 6..10.
#include "ss_sliced_kernel.h"
#include "ss_fused.h"

namespace ss {

hipError_t launch_sliced_mid(int E, const uint32_t* packed, int64_t n, int32_t m, int sub_width, uint16_t* out,
                           hipStream_t s)
{
    return sliced::SlicedTable<11, 12, 13, 14, 15, 16, 17, 18, 19, 20>::run(E, packed, n, m, sub_width, out, s);
}

hipError_t launch_fused_mid(int E, const uint8_t* reads, const uint8_t* refs, int64_t n, int32_t m, int T, int GB,
                           int U, int fast, size_t shmem, uint16_t* out, uint32_t* err, hipStream_t s)
{
    return sliced::FusedTable<6, 7, 8, 9, 10>::run(E, reads, refs, n, m, T, GB, U, fast, shmem, out, err, s);
}

}  // namespace ss
