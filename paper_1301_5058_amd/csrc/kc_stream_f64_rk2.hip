// kc_stream_f64_rk2.hip -- instantiates the fused step kernel for FP64 fields, the two-stage Runge-Kutta method
// (one translation unit per precision, integrator and noise mode, so they
// compile in parallel).
#include "kc_step_kernels.h"

namespace kc {

namespace {

template <int T, int LAW> const void *pick_pf(int pf)
{
    return pf == 4 ? reinterpret_cast<const void *>(&step_stream<double, T, LAW, 4, true, false>)
                   : reinterpret_cast<const void *>(&step_stream<double, T, LAW, 2, true, false>);
}

template <int LAW> const void *pick_levels(int levels, int pf)
{
    switch (levels) {
    case 2: return pick_pf<2, LAW>(pf);
    case 4: return pick_pf<4, LAW>(pf);
    case 6: return pick_pf<6, LAW>(pf);
    default: return nullptr;
    }
}

} // namespace

template <>
const void *stream_kernel_for<double, true, false>(int chi_law, int levels, int pf)
{
    return chi_law == 0 ? pick_levels<0>(levels, pf) : pick_levels<1>(levels, pf);
}

} // namespace kc
