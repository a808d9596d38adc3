// kc_step_kernels.h -- the fused step kernel and its launch arguments, shared
// by the translation units that instantiate it (kc_stream_*.hip) and the host
// launchers (kc_step.hip).
#pragma once

#include "kc_internal.h"
#include "kc_stream.h"

namespace kc {

template <typename R> struct StepArgs {
    const R *b_in, *n_in, *sg;
    R *b_out, *n_out;
    const R *b_avg, *n_avg; // step_ref with AVG: the level averaged with
    Noise<R> z;             // per-step agar noise (NOISE kernels)
    int nx, ny, pitch;
    int rows;           // output rows per strip
    int nsx, nstrips;   // strips along x, total strips
    int nblocks_padded; // grid size (multiple of 8)
    Coef<R> c;
    // diagnostics of the stored level, or null: strip k writes {sum b, sum n,
    // max d^2 (-1: none), count of b >= b_thr} to parts[4k .. 4k + 3]
    double *parts;
    double b_thr, cx, cy;
};

// ---------------------------------------------------------------------------
// Fused kernel
// ---------------------------------------------------------------------------
template <typename R, int T, int LAW, int PF, bool RK, bool NOISE>
__global__ __launch_bounds__(256) void step_stream(StepArgs<R> a)
{
    const int lb = xcd_block(a.nblocks_padded);
    // wave-uniform by construction; readfirstlane lets the compiler keep the strip
    // geometry and every row test in scalar registers
    const int strip = __builtin_amdgcn_readfirstlane(lb * 4 + (int)(threadIdx.x >> 6));
    if (strip >= a.nstrips)
        return; // whole wavefront leaves together
    StripArgs<R> sa;
    sa.b_in = a.b_in;
    sa.n_in = a.n_in;
    sa.sg = a.sg;
    sa.b_out = a.b_out;
    sa.n_out = a.n_out;
    sa.nx = a.nx;
    sa.ny = a.ny;
    sa.pitch = a.pitch;
    sa.rows = a.rows;
    sa.c = a.c;
    sa.z = a.z;
    sa.b_thr = a.b_thr;
    sa.cx = a.cx;
    sa.cy = a.cy;
    const int sx = strip % a.nsx, sy = strip / a.nsx;
    constexpr int VEC = StreamShape<R>::VEC;
    if (strip_inside<R, T>(sa, sx))
        stream_strip<R, T, LAW, PF, false, RK, NOISE>(sa, sx, sy);
    else if (!NOISE || a.nx % VEC == 0)
        stream_strip<R, T, LAW, PF, true, RK, NOISE>(sa, sx, sy);
    else // noise on a grid whose width is not a multiple of VEC: per-cell draws at the edges
        stream_strip<R, T, LAW, PF, true, RK, NOISE, true>(sa, sx, sy);
    if (a.parts) {
        // fold the cells this strip stored into its partials (no separate pass
        // over the fields; a wave-uniform test on a kernel argument)
        DiagAcc acc{0.0, 0.0, -1.0, 0.0};
        strip_diag<R, T>(sa, sx, sy, acc);
        const double sb = wave_sum64(acc.sb), sn = wave_sum64(acc.sn);
        const double m2 = wave_max64(acc.m2), ct = wave_sum64(acc.cnt);
        if ((threadIdx.x & 63) == 0) {
            double *q = a.parts + 4 * (size_t)strip;
            q[0] = sb;
            q[1] = sn;
            q[2] = m2;
            q[3] = ct;
        }
    }
}

// The compiled fused kernel of precision R, integrator RK and noise mode NOISE
// for (law, levels, prefetch), or null when there is none.  Each (R, RK,
// NOISE) triple is defined in a translation unit of its own
// (kc_stream_<precision>_<integrator>[_noise].hip).
template <typename R, bool RK, bool NOISE>
const void *stream_kernel_for(int chi_law, int levels, int pf);

} // namespace kc
