// kc_step.hip -- explicit time-step kernels of the single-instance solver.
//
// step_ref     one step per launch, one thread per cell, neighbours read from
//              global memory.  The plain form of the stencil; every other
//              kernel must reproduce its bits.
// step_stream  T steps per launch: each wavefront advances one strip with
//              stream_strip (kc_stream.h); strips are numbered x-fastest and
//              grouped four to a workgroup, and workgroups are remapped so each
//              XCD owns a contiguous band of strips.
#include "kc_internal.h"
#include "kc_stream.h"

namespace kc {

template <typename R> struct StepArgs {
    const R *b_in, *n_in, *sg;
    R *b_out, *n_out;
    int nx, ny, pitch;
    int rows;           // output rows per strip
    int nsx, nstrips;   // strips along x, total strips
    int nblocks_padded; // grid size (multiple of 8)
    Coef<R> c;
};

// ---------------------------------------------------------------------------
// Reference kernel
// ---------------------------------------------------------------------------
template <typename R, int LAW>
__device__ __forceinline__ void ref_cell(const StepArgs<R> &a, int x, int y, R &b, R &n, R &D, R &X)
{
    if (x < 0 || x >= a.nx || y < 0 || y >= a.ny) {
        b = n = D = X = R(0);
        return;
    }
    const size_t p = (size_t)y * a.pitch + x;
    b = a.b_in[p];
    n = a.n_in[p];
    const R sh = R(0.5) * a.sg[p];
    coef<R, LAW>(sh, n, b, a.c.chi2, D, X);
}

template <typename R, int LAW>
__global__ __launch_bounds__(256) void step_ref(StepArgs<R> a)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.nx || y >= a.ny)
        return;
    R bP, nP, DP, XP, bE, nE, DE, XE, bW, nW, DW, XW, bN, nN, DN, XN, bS, nS, DS, XS;
    ref_cell<R, LAW>(a, x, y, bP, nP, DP, XP);
    ref_cell<R, LAW>(a, x + 1, y, bE, nE, DE, XE);
    ref_cell<R, LAW>(a, x - 1, y, bW, nW, DW, XW);
    ref_cell<R, LAW>(a, x, y + 1, bN, nN, DN, XN);
    ref_cell<R, LAW>(a, x, y - 1, bS, nS, DS, XS);
    R geb, gen, gwb, gwn, gnb, gnn, gsb, gsn;
    face<R>(bP, nP, DP, XP, bE, nE, DE, XE, x + 1 < a.nx, geb, gen);
    face<R>(bW, nW, DW, XW, bP, nP, DP, XP, x - 1 >= 0, gwb, gwn);
    face<R>(bP, nP, DP, XP, bN, nN, DN, XN, y + 1 < a.ny, gnb, gnn);
    face<R>(bS, nS, DS, XS, bP, nP, DP, XP, y - 1 >= 0, gsb, gsn);
    const R Fb = net<R>(geb, gwb, gnb, gsb);
    const R Fn = net<R>(gen, gwn, gnn, gsn);
    R bo, no;
    update<R>(bP, nP, Fb, Fn, a.c, bo, no);
    const size_t p = (size_t)y * a.pitch + x;
    a.b_out[p] = bo;
    a.n_out[p] = no;
}

// ---------------------------------------------------------------------------
// Fused kernel
// ---------------------------------------------------------------------------
template <typename R, int T, int LAW, int PF>
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
    sa.b_thr = sa.cx = sa.cy = 0.0;
    const int sx = strip % a.nsx, sy = strip / a.nsx;
    if (strip_interior<R, T>(sa, sx, sy))
        stream_strip<R, T, LAW, PF, false>(sa, sx, sy);
    else
        stream_strip<R, T, LAW, PF, true>(sa, sx, sy);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static const int kDepths[] = {1, 2, 3, 4, 6, 8};

int stream_depth_at_most(int t)
{
    int best = 1;
    for (int d : kDepths)
        if (d <= t)
            best = d;
    return best;
}

StreamGeom stream_geom(int precision, int tsteps, int nx, int ny, int rows)
{
    const int vec = precision == 0 ? 4 : 2;
    const int hx = (tsteps + vec - 1) / vec * vec;
    StreamGeom g;
    g.out_cols = 64 * vec - 2 * hx;
    g.nsx = (nx + g.out_cols - 1) / g.out_cols;
    g.nsy = (ny + rows - 1) / rows;
    g.nstrips = g.nsx * g.nsy;
    const int nblocks = (g.nstrips + 3) / 4;
    g.nblocks_padded = (nblocks + 7) / 8 * 8;
    return g;
}

template <typename R>
static StepArgs<R> make_args(const Fields<R> &f, const Coef<R> &c)
{
    StepArgs<R> a;
    a.b_in = f.b_in;
    a.n_in = f.n_in;
    a.sg = f.sg;
    a.b_out = f.b_out;
    a.n_out = f.n_out;
    a.nx = f.nx;
    a.ny = f.ny;
    a.pitch = f.pitch;
    a.rows = 1;
    a.nsx = a.nstrips = a.nblocks_padded = 0;
    a.c = c;
    return a;
}

template <typename R, int T, int LAW>
static hipError_t launch_stream_pf(const StepArgs<R> &a, int pf, dim3 grid, hipStream_t s)
{
    if (pf == 4)
        hipLaunchKernelGGL((step_stream<R, T, LAW, 4>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((step_stream<R, T, LAW, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename R, int LAW>
static hipError_t launch_stream_t(const StepArgs<R> &a, int T, int pf, dim3 grid, hipStream_t s)
{
    switch (T) {
    case 1: return launch_stream_pf<R, 1, LAW>(a, pf, grid, s);
    case 2: return launch_stream_pf<R, 2, LAW>(a, pf, grid, s);
    case 3: return launch_stream_pf<R, 3, LAW>(a, pf, grid, s);
    case 4: return launch_stream_pf<R, 4, LAW>(a, pf, grid, s);
    case 6: return launch_stream_pf<R, 6, LAW>(a, pf, grid, s);
    case 8: return launch_stream_pf<R, 8, LAW>(a, pf, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, const Tuning &t,
                         hipStream_t s)
{
    StepArgs<R> a = make_args(f, c);
    const StreamGeom g = stream_geom(sizeof(R) == 4 ? 0 : 1, t.tsteps, f.nx, f.ny, t.rows);
    a.rows = t.rows;
    a.nsx = g.nsx;
    a.nstrips = g.nstrips;
    a.nblocks_padded = g.nblocks_padded;
    const dim3 grid(g.nblocks_padded);
    if (chi_law == 0)
        return launch_stream_t<R, 0>(a, t.tsteps, t.prefetch, grid, s);
    return launch_stream_t<R, 1>(a, t.tsteps, t.prefetch, grid, s);
}

template <typename R>
hipError_t launch_ref(const Fields<R> &f, const Coef<R> &c, int chi_law, hipStream_t s)
{
    const StepArgs<R> a = make_args(f, c);
    const dim3 grid((f.nx + 63) / 64, (f.ny + 3) / 4);
    if (chi_law == 0)
        hipLaunchKernelGGL((step_ref<R, 0>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((step_ref<R, 1>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t time_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, const Tuning &t,
                       hipStream_t s, int reps, double *ms)
{
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess)
        return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    e = launch_stream<R>(f, c, chi_law, t, s);
    if (e == hipSuccess)
        e = hipEventRecord(e0, s);
    for (int i = 0; i < reps && e == hipSuccess; ++i)
        e = launch_stream<R>(f, c, chi_law, t, s);
    if (e == hipSuccess)
        e = hipEventRecord(e1, s);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    float el = 0.f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&el, e0, e1);
    if (e == hipSuccess)
        *ms = (double)el / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

template <typename R, int T, int LAW, int PF> static int blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_stream<R, T, LAW, PF>, 256, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

template <typename R, int LAW> static int blocks_per_cu_t(int T, int pf)
{
    switch (T) {
    case 1: return pf == 4 ? blocks_per_cu<R, 1, LAW, 4>() : blocks_per_cu<R, 1, LAW, 2>();
    case 2: return pf == 4 ? blocks_per_cu<R, 2, LAW, 4>() : blocks_per_cu<R, 2, LAW, 2>();
    case 3: return pf == 4 ? blocks_per_cu<R, 3, LAW, 4>() : blocks_per_cu<R, 3, LAW, 2>();
    case 4: return pf == 4 ? blocks_per_cu<R, 4, LAW, 4>() : blocks_per_cu<R, 4, LAW, 2>();
    case 6: return pf == 4 ? blocks_per_cu<R, 6, LAW, 4>() : blocks_per_cu<R, 6, LAW, 2>();
    case 8: return pf == 4 ? blocks_per_cu<R, 8, LAW, 4>() : blocks_per_cu<R, 8, LAW, 2>();
    default: return 0;
    }
}

int resident_waves(int precision, int chi_law, int tsteps, int prefetch)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    int nb;
    if (precision == 0)
        nb = chi_law == 0 ? blocks_per_cu_t<float, 0>(tsteps, prefetch)
                          : blocks_per_cu_t<float, 1>(tsteps, prefetch);
    else
        nb = chi_law == 0 ? blocks_per_cu_t<double, 0>(tsteps, prefetch)
                          : blocks_per_cu_t<double, 1>(tsteps, prefetch);
    return nb * 4 * cus;
}

int round_fitted_rows(int precision, int tsteps, int nx, int ny, int waves, int rounds)
{
    if (waves <= 0 || rounds <= 0 || nx <= 0 || ny <= 0)
        return 0;
    const StreamGeom g = stream_geom(precision, tsteps, nx, ny, 1);
    const long m = (long)waves * rounds / g.nsx; // strip rows that fill `rounds` rounds
    if (m <= 0)
        return 0;
    return (int)((ny + m - 1) / m);
}

void tuning_candidates(int effort, int max_tsteps, int precision, int chi_law, int nx, int ny,
                       Tuning *out, int *n, int cap)
{
    static const int quick_t[] = {1, 2, 3, 4};
    static const int quick_r[] = {16, 32, 64, 128};
    static const int full_t[] = {1, 2, 3, 4, 6, 8};
    static const int full_r[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 256};
    const int *ts = effort ? full_t : quick_t;
    const int *rs = effort ? full_r : quick_r;
    const int nt = effort ? 6 : 4, nr = effort ? 10 : 4;
    int k = 0;
    auto add = [&](int t, int r, int p) {
        for (int i = 0; i < k && i < cap; ++i)
            if (out[i].tsteps == t && out[i].rows == r && out[i].prefetch == p)
                return;
        if (k < cap) {
            out[k].tsteps = t;
            out[k].rows = r;
            out[k].prefetch = p;
        }
        ++k;
    };
    for (int i = 0; i < nt; ++i) {
        if (ts[i] > max_tsteps)
            continue;
        for (int p = 0; p < (effort ? 2 : 1); ++p) {
            const int pf = p ? 2 : 4;
            for (int j = 0; j < nr; ++j)
                add(ts[i], rs[j], pf);
            // rows that fill a whole number of rounds of resident wavefronts
            if (nx <= 0 || ny <= 0)
                continue;
            const int w = resident_waves(precision, chi_law, ts[i], pf);
            for (int q = 1; q <= 8; ++q) {
                const int r = round_fitted_rows(precision, ts[i], nx, ny, w, q);
                if (r >= 4 && r <= 512)
                    add(ts[i], r, pf);
            }
        }
    }
    *n = k < cap ? k : cap;
}

template hipError_t time_stream<float>(const Fields<float> &, const Coef<float> &, int,
                                       const Tuning &, hipStream_t, int, double *);
template hipError_t time_stream<double>(const Fields<double> &, const Coef<double> &, int,
                                        const Tuning &, hipStream_t, int, double *);
template hipError_t launch_stream<float>(const Fields<float> &, const Coef<float> &, int,
                                         const Tuning &, hipStream_t);
template hipError_t launch_stream<double>(const Fields<double> &, const Coef<double> &, int,
                                          const Tuning &, hipStream_t);
template hipError_t launch_ref<float>(const Fields<float> &, const Coef<float> &, int, hipStream_t);
template hipError_t launch_ref<double>(const Fields<double> &, const Coef<double> &, int,
                                       hipStream_t);

} // namespace kc
