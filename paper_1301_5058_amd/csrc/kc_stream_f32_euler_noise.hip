// kc_stream_f32_euler_noise.hip -- instantiates the fused step kernels (whole-strip and
// split) for FP32 fields, forward Euler and per-step agar noise (one translation unit per precision,
// integrator and noise mode, so they compile in parallel).
#include "kc_step_kernels.h"

namespace kc {

template <>
const void *stream_kernel_for<float, false, true>(int chi_law, int levels, int pf, int waves)
{
    return stream_kernel_table<float, false, true>(chi_law, levels, pf, waves);
}

} // namespace kc
