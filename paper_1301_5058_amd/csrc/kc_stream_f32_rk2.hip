// kc_stream_f32_rk2.hip -- instantiates the fused step kernels (whole-strip and
// split) for FP32 fields, the two-stage Runge-Kutta method (one translation unit per precision,
// integrator and noise mode, so they compile in parallel).
#include "kc_step_kernels.h"

namespace kc {

template <>
const void *stream_kernel_for<float, true, false>(int chi_law, int levels, int pf, int waves)
{
    return stream_kernel_table<float, true, false>(chi_law, levels, pf, waves);
}

} // namespace kc
