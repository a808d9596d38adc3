// kc_stream_f32_euler.hip -- instantiates the fused step kernel for FP32 fields, forward Euler
// (one translation unit per precision, integrator and noise mode, so they
// compile in parallel).
#include "kc_step_kernels.h"

namespace kc {

namespace {

template <int T, int LAW> const void *pick_pf(int pf)
{
    return pf == 4 ? reinterpret_cast<const void *>(&step_stream<float, T, LAW, 4, false, false>)
                   : reinterpret_cast<const void *>(&step_stream<float, T, LAW, 2, false, false>);
}

template <int LAW> const void *pick_levels(int levels, int pf)
{
    switch (levels) {
    case 1: return pick_pf<1, LAW>(pf);
    case 2: return pick_pf<2, LAW>(pf);
    case 3: return pick_pf<3, LAW>(pf);
    case 4: return pick_pf<4, LAW>(pf);
    case 6: return pick_pf<6, LAW>(pf);
    case 8: return pick_pf<8, LAW>(pf);
    default: return nullptr;
    }
}

} // namespace

template <>
const void *stream_kernel_for<float, false, false>(int chi_law, int levels, int pf)
{
    return chi_law == 0 ? pick_levels<0>(levels, pf) : pick_levels<1>(levels, pf);
}

} // namespace kc
