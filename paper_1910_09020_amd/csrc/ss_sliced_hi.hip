// Column-sweep kernels for thresholds E = 21..32.
#include "ss_sliced_kernel.h"

namespace ss {

hipError_t launch_sliced_hi(int E, const uint32_t* packed, int64_t n, int32_t m, int sub_width, uint16_t* out,
                           hipStream_t s)
{
    return sliced::SlicedTable<21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32>::run(E, packed, n, m, sub_width, out, s);
}

}  // namespace ss
