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
    int nsx, nstrips;   // strip columns, total strips
    int nblocks_padded; // grid size (multiple of 8)
    // folded last column: strips [0, nmain) cover the first nsx_main columns
    // row by row, strips [nmain, nstrips) the last column, fold_bands strip rows
    // each (nsx_main = nsx and nmain = nstrips when nothing is folded)
    int nsx_main, nmain, nsy, fold_bands, fold_lanes;
    uint32_t field_bytes; // pitch * ny * sizeof(R) (< 2^31 when folding)
    Coef<R> c;
    // diagnostics of the stored level, or null: strip k writes {sum b, sum n,
    // max d^2 (-1: none), count of b >= b_thr} to parts[4k .. 4k + 3]
    double *parts;
    double b_thr, cx, cy;
};

// Kernels that carry the folded-strip path (stream_strip with FOLD): FP32 with
// at most four levels.  With the path compiled into the deeper per-step-noise
// kernels as well (FP64 with six levels, FP32 with eight), those returned
// fields that differ from the reference kernel's, also on strips that fold
// nothing; the cause was not found, so they are built without it.
template <typename R, int T> struct Foldable {
    static constexpr bool value = sizeof(R) == 4 && T <= 4;
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
    sa.nsy = a.nsy;
    sa.fold_bands = a.fold_bands;
    sa.fold_lanes = a.fold_lanes;
    sa.field_bytes = a.field_bytes;
    constexpr bool FOLDS = Foldable<R, T>::value;
    const bool folded = FOLDS && strip >= a.nmain;
    const int sx = FOLDS ? (folded ? a.nsx - 1 : strip % a.nsx_main) : strip % a.nsx;
    const int sy = FOLDS ? (folded ? strip - a.nmain : strip / a.nsx_main) : strip / a.nsx;
    constexpr int VEC = StreamShape<R>::VEC;
    if (folded) {
        if constexpr (FOLDS)
            stream_strip<R, T, LAW, PF, true, RK, NOISE, false, WHOLE, true>(sa, sx, sy);
    } else if (strip_inside<R, T>(sa, sx))
        stream_strip<R, T, LAW, PF, false, RK, NOISE>(sa, sx, sy);
    else if (!NOISE || a.nx % VEC == 0)
        stream_strip<R, T, LAW, PF, true, RK, NOISE>(sa, sx, sy);
    else // noise on a grid whose width is not a multiple of VEC: per-cell draws at the edges
        stream_strip<R, T, LAW, PF, true, RK, NOISE, true>(sa, sx, sy);
    if (a.parts) {
        // fold the cells this strip stored into its partials (no separate pass
        // over the fields; a wave-uniform test on a kernel argument)
        DiagAcc acc{0.0, 0.0, -1.0, 0.0};
        if (folded) {
            if constexpr (FOLDS)
                strip_diag<R, T, true>(sa, sx, sy, acc);
        } else {
            strip_diag<R, T>(sa, sx, sy, acc);
        }
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

// Split fused kernel: one strip per workgroup of two wavefronts, the first
// running levels [0, T/2) from memory, the second levels [T/2, T) from the LDS
// ring the first fills (stream_strip roles SPLIT_FIRST / SPLIT_SECOND).  Each
// wavefront holds half the level state, so twice as many fit on a SIMD for
// the same strips and halo; fields are the same bits as step_stream's.
// Register budget of a split kernel: the FP32 four-level kernels are held to
// three wavefronts per SIMD (at most 168 VGPRs).  With the static agar field
// they fit without spilling; with per-step noise the generator's state spills
// a few dozen registers, and the third wavefront still wins (2048^2 RK2: 3 %;
// prefetch 4 at 4096^2: 30 %).  The others keep the compiler's choice.
template <typename R, int T, bool NOISE> struct SplitWaves {
    static constexpr bool three = sizeof(R) == 4 && T == 4;
    static constexpr int lo = three ? 3 : 1;
    static constexpr int hi = three ? 3 : 8;
};

template <typename R, int T, int LAW, int PF, bool RK, bool NOISE>
__global__ __launch_bounds__(128)
__attribute__((amdgpu_waves_per_eu(SplitWaves<R, T, NOISE>::lo, SplitWaves<R, T, NOISE>::hi)))
void step_split(StepArgs<R> a)
{
    __shared__ SplitRing<R, PF> ring;
    const int strip = __builtin_amdgcn_readfirstlane(xcd_block(a.nblocks_padded));
    if (strip >= a.nstrips)
        return; // both wavefronts of the workgroup leave together
    const bool second = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) != 0;
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
    sa.nsy = a.nsy;
    sa.fold_bands = a.fold_bands;
    sa.fold_lanes = a.fold_lanes;
    sa.field_bytes = a.field_bytes;
    constexpr bool FOLDS = Foldable<R, T>::value;
    const bool folded = FOLDS && strip >= a.nmain;
    const int sx = FOLDS ? (folded ? a.nsx - 1 : strip % a.nsx_main) : strip % a.nsx;
    const int sy = FOLDS ? (folded ? strip - a.nmain : strip / a.nsx_main) : strip / a.nsx;
    constexpr int VEC = StreamShape<R>::VEC;
    if (folded) {
        if constexpr (FOLDS) {
            if (second)
                stream_strip<R, T, LAW, PF, true, RK, NOISE, false, SPLIT_SECOND, true>(
                    sa, sx, sy, &ring);
            else
                stream_strip<R, T, LAW, PF, true, RK, NOISE, false, SPLIT_FIRST, true>(
                    sa, sx, sy, &ring);
        }
    } else if (strip_inside<R, T>(sa, sx)) {
        if (second)
            stream_strip<R, T, LAW, PF, false, RK, NOISE, false, SPLIT_SECOND>(sa, sx, sy, &ring);
        else
            stream_strip<R, T, LAW, PF, false, RK, NOISE, false, SPLIT_FIRST>(sa, sx, sy, &ring);
    } else if (!NOISE || a.nx % VEC == 0) {
        if (second)
            stream_strip<R, T, LAW, PF, true, RK, NOISE, false, SPLIT_SECOND>(sa, sx, sy, &ring);
        else
            stream_strip<R, T, LAW, PF, true, RK, NOISE, false, SPLIT_FIRST>(sa, sx, sy, &ring);
    } else {
        if (second)
            stream_strip<R, T, LAW, PF, true, RK, NOISE, true, SPLIT_SECOND>(sa, sx, sy, &ring);
        else
            stream_strip<R, T, LAW, PF, true, RK, NOISE, true, SPLIT_FIRST>(sa, sx, sy, &ring);
    }
    if (second && a.parts) {
        DiagAcc acc{0.0, 0.0, -1.0, 0.0};
        if (folded) {
            if constexpr (FOLDS)
                strip_diag<R, T, true>(sa, sx, sy, acc);
        } else {
            strip_diag<R, T>(sa, sx, sy, acc);
        }
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
// for (law, levels, prefetch, waves per strip), or null when there is none.
// Each (R, RK, NOISE) triple is defined in a translation unit of its own
// (kc_stream_<precision>_<integrator>[_noise].hip).
template <typename R, bool RK, bool NOISE>
const void *stream_kernel_for(int chi_law, int levels, int pf, int waves);

// Kernel table of one (R, RK, NOISE) triple: whole-strip kernels for levels
// {1, 2, 3, 4, 6, 8} (forward Euler) or {2, 4, 6} (Runge-Kutta), split kernels
// for the even level counts whose halves are whole time steps ({2, 4, 6, 8} and
// {4}), prefetch depth 2 or 4.
template <typename R, int T, int LAW, bool RK, bool NOISE>
const void *pick_kernel(int pf, int waves)
{
    constexpr bool can_split = T % 2 == 0 && (!RK || (T / 2) % 2 == 0);
    if (waves == 2) {
        if constexpr (can_split)
            return pf == 4 ? reinterpret_cast<const void *>(&step_split<R, T, LAW, 4, RK, NOISE>)
                           : reinterpret_cast<const void *>(&step_split<R, T, LAW, 2, RK, NOISE>);
        return nullptr;
    }
    return pf == 4 ? reinterpret_cast<const void *>(&step_stream<R, T, LAW, 4, RK, NOISE>)
                   : reinterpret_cast<const void *>(&step_stream<R, T, LAW, 2, RK, NOISE>);
}

// pick_kernel for the level counts a translation unit instantiates: all of them
// (ONLY = 0) or only ONLY, and never EXCLUDE (a kernel is compiled in exactly
// one translation unit).
template <typename R, int T, int LAW, bool RK, bool NOISE, int EXCLUDE, int ONLY>
const void *pick_kernel_in_unit(int pf, int waves)
{
    if constexpr ((ONLY == 0 || ONLY == T) && EXCLUDE != T)
        return pick_kernel<R, T, LAW, RK, NOISE>(pf, waves);
    else
        return nullptr;
}

template <typename R, int LAW, bool RK, bool NOISE, int EXCLUDE, int ONLY>
const void *pick_levels(int levels, int pf, int waves)
{
    if constexpr (RK) {
        switch (levels) {
        case 2: return pick_kernel_in_unit<R, 2, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        case 4: return pick_kernel_in_unit<R, 4, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        case 6: return pick_kernel_in_unit<R, 6, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        default: return nullptr;
        }
    } else {
        switch (levels) {
        case 1: return pick_kernel_in_unit<R, 1, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        case 2: return pick_kernel_in_unit<R, 2, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        case 3: return pick_kernel_in_unit<R, 3, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        case 4: return pick_kernel_in_unit<R, 4, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        case 6: return pick_kernel_in_unit<R, 6, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        case 8: return pick_kernel_in_unit<R, 8, LAW, RK, NOISE, EXCLUDE, ONLY>(pf, waves);
        default: return nullptr;
        }
    }
}

template <typename R, bool RK, bool NOISE, int EXCLUDE = 0, int ONLY = 0>
const void *stream_kernel_table(int chi_law, int levels, int pf, int waves)
{
    if ((pf != 2 && pf != 4) || (waves != 1 && waves != 2))
        return nullptr;
    return chi_law == 0 ? pick_levels<R, 0, RK, NOISE, EXCLUDE, ONLY>(levels, pf, waves)
                        : pick_levels<R, 1, RK, NOISE, EXCLUDE, ONLY>(levels, pf, waves);
}

// The four-level FP32 forward-Euler kernels (the benchmark's), defined in
// kc_stream_f32_euler4.hip, which is compiled with the latency-first
// (max-ILP) machine scheduler: at their register budgets it interleaves
// independent rows and cells more and runs them 2-3 % faster, while it slows
// the deeper and the noise kernels, which stay with the default scheduler.
const void *stream_kernel_f32_euler4(int chi_law, int pf, int waves);

} // namespace kc
