// Column-sweep kernels for thresholds E = 11..20.
#include "ss_sliced_kernel.h"

namespace ss {

hipError_t launch_sliced_mid(int E, const uint32_t* packed, int64_t n, int32_t m, int sub_width, uint16_t* out,
                           hipStream_t s)
{
    return sliced::SlicedTable<11, 12, 13, 14, 15, 16, 17, 18, 19, 20>::run(E, packed, n, m, sub_width, out, s);
}

}  // namespace ss
