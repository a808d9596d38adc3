// kc_stream_f32_euler4.hip -- the four-level FP32 forward-Euler fused kernels
// (whole-strip and split, both sensitivity laws, both prefetch depths), in a
// translation unit of their own so that the build can give them the
// latency-first machine scheduler (see kc_step_kernels.h).
#include "kc_step_kernels.h"

namespace kc {

const void *stream_kernel_f32_euler4(int chi_law, int pf, int waves)
{
    return stream_kernel_table<float, false, false, 0, 4>(chi_law, 4, pf, waves);
}

} // namespace kc
