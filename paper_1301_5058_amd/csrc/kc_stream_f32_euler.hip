// kc_stream_f32_euler.hip -- instantiates the fused step kernels (whole-strip and
// split) for FP32 fields, forward Euler (one translation unit per precision,
// integrator and noise mode, so they compile in parallel).
#include "kc_step_kernels.h"

namespace kc {

template <>
const void *stream_kernel_for<float, false, false>(int chi_law, int levels, int pf, int waves)
{
    if (levels == 4)
        return stream_kernel_f32_euler4(chi_law, pf, waves);
    return stream_kernel_table<float, false, false, 4, 0>(chi_law, levels, pf, waves);
}

} // namespace kc
