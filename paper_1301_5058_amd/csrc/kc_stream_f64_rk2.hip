// kc_stream_f64_rk2.hip -- instantiates the fused step kernels (whole-strip and
// split) for FP64 fields, the two-stage Runge-Kutta method (one translation unit per precision,
// integrator and noise mode, so they compile in parallel).
#include "kc_step_kernels.h"

namespace kc {

template <>
const void *stream_kernel_for<double, true, false>(int chi_law, int levels, int pf, int waves)
{
    return stream_kernel_table<double, true, false>(chi_law, levels, pf, waves);
}

} // namespace kc
