// kc_step.hip -- explicit time-step kernels of the single-instance solver.
//
// step_ref     one forward-Euler step per launch, one thread per cell,
//              neighbours read from global memory; with AVG the result is
//              averaged with a second input level (the last stage of a
//              two-stage Runge-Kutta step).  The plain form of the stencil;
//              every other kernel must reproduce its bits.
// step_stream  T levels per launch (T Euler steps, or T / 2 Runge-Kutta steps
//              with RK): each wavefront advances one strip with stream_strip
//              (kc_stream.h); strips are numbered x-fastest and grouped four to
//              a workgroup, and workgroups are remapped so each XCD owns a
//              contiguous band of strips.
#include "kc_step_kernels.h"

namespace kc {

// ---------------------------------------------------------------------------
// Reference kernel
// ---------------------------------------------------------------------------
template <typename R, int LAW, bool NOISE>
__device__ __forceinline__ void ref_cell(const StepArgs<R> &a, int x, int y, R &b, R &n, R &D, R &X)
{
    if (x < 0 || x >= a.nx || y < 0 || y >= a.ny) {
        b = n = D = X = R(0);
        return;
    }
    const size_t p = (size_t)y * a.pitch + x;
    b = a.b_in[p];
    n = a.n_in[p];
    const R sh = NOISE ? noise_half_sigma1<R>(a.z, 0, x, y) : R(0.5) * a.sg[p];
    coef<R, LAW>(sh, n, b, a.c.chi2, D, X);
}

template <typename R, int LAW, bool AVG, bool NOISE>
__global__ __launch_bounds__(256) void step_ref(StepArgs<R> a)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.nx || y >= a.ny)
        return;
    R bP, nP, DP, XP, bE, nE, DE, XE, bW, nW, DW, XW, bN, nN, DN, XN, bS, nS, DS, XS;
    ref_cell<R, LAW, NOISE>(a, x, y, bP, nP, DP, XP);
    ref_cell<R, LAW, NOISE>(a, x + 1, y, bE, nE, DE, XE);
    ref_cell<R, LAW, NOISE>(a, x - 1, y, bW, nW, DW, XW);
    ref_cell<R, LAW, NOISE>(a, x, y + 1, bN, nN, DN, XN);
    ref_cell<R, LAW, NOISE>(a, x, y - 1, bS, nS, DS, XS);
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
    if (AVG) {
        bo = rk2_average<R>(a.b_avg[p], bo);
        no = rk2_average<R>(a.n_avg[p], no);
    }
    a.b_out[p] = bo;
    a.n_out[p] = no;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static const int kDepths[] = {1, 2, 3, 4, 6, 8}; // Euler steps per launch
static const int kRkDepths[] = {1, 2, 3};         // Runge-Kutta steps (2 levels each)

int stream_depth_at_most(int t, int integrator)
{
    int best = 1;
    if (integrator == 0) {
        for (int d : kDepths)
            if (d <= t)
                best = d;
    } else {
        for (int d : kRkDepths)
            if (d <= t)
                best = d;
    }
    return best;
}

int stream_levels(int integrator, int tsteps) { return integrator == 0 ? tsteps : 2 * tsteps; }

StreamGeom stream_geom(int precision, int levels, int nx, int ny, int rows, int waves, bool fold)
{
    const int vec = precision == 0 ? 4 : 2;
    const int hx = (levels + vec - 1) / vec * vec;
    StreamGeom g;
    g.out_cols = 64 * vec - 2 * hx;
    g.nsx = (nx + g.out_cols - 1) / g.out_cols;
    g.nsy = (ny + rows - 1) / rows;
    g.nstrips = g.nsx * g.nsy;
    g.nsx_main = g.nsx;
    g.nmain = g.nstrips;
    g.fold_bands = 1;
    g.fold_lanes = 64;
    // folding the last column (the kernels that carry the path: FP32, at most
    // four levels): its output columns plus a halo on either side per band; the
    // whole field addressable through one buffer resource (32-bit offsets);
    // rows + levels <= ny keeps every row of a band's steady state below 2 ny
    // (one reflection)
    const int w_last = nx - (g.nsx - 1) * g.out_cols;
    const int lanes = (2 * hx + w_last + vec - 1) / vec;
    const int bands = 64 / lanes;
    const double field = (double)pitch_for(nx) * ny * (precision == 0 ? 4 : 8);
    if (fold && precision == 0 && levels <= 4 && nx % vec == 0 && bands >= 2 && g.nsy >= 2 &&
        field < 2147483648.0 && rows + levels <= ny) {
        g.nsx_main = g.nsx > 1 ? g.nsx - 1 : 1;
        g.nmain = (g.nsx - 1) * g.nsy;
        g.fold_bands = bands;
        g.fold_lanes = lanes;
        g.nstrips = g.nmain + (g.nsy + bands - 1) / bands;
    }
    const int nblocks = waves == 2 ? g.nstrips : (g.nstrips + 3) / 4;
    g.nblocks_padded = (nblocks + 7) / 8 * 8;
    return g;
}

int launch_waves(int integrator, int levels, int waves)
{
    if (waves != 2 || levels % 2 != 0)
        return 1;
    if (integrator != 0 && (levels / 2) % 2 != 0)
        return 1;
    return 2;
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
    a.b_avg = a.n_avg = nullptr;
    a.z = Noise<R>{R(1), R(0), 0u, 0u, 0u, 0u};
    a.nx = f.nx;
    a.ny = f.ny;
    a.pitch = f.pitch;
    a.rows = 1;
    a.nsx = a.nstrips = a.nblocks_padded = 0;
    a.nsx_main = 1;
    a.nmain = 0x7fffffff;
    a.nsy = 0;
    a.fold_bands = 1;
    a.fold_lanes = 64;
    a.field_bytes = 0;
    a.c = c;
    a.parts = nullptr;
    a.b_thr = a.cx = a.cy = 0.0;
    return a;
}

template <typename R>
static const void *stream_kernel(int chi_law, int integrator, bool noise, int levels, int pf,
                                 int waves)
{
    if ((pf != 2 && pf != 4) || (integrator != 0 && integrator != 1) ||
        (chi_law != 0 && chi_law != 1))
        return nullptr;
    if (noise)
        return integrator == 0 ? stream_kernel_for<R, false, true>(chi_law, levels, pf, waves)
                               : stream_kernel_for<R, true, true>(chi_law, levels, pf, waves);
    return integrator == 0 ? stream_kernel_for<R, false, false>(chi_law, levels, pf, waves)
                           : stream_kernel_for<R, true, false>(chi_law, levels, pf, waves);
}

template <typename R>
hipError_t launch_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, int integrator,
                         const Tuning &t, hipStream_t s, const Noise<R> *z, const DiagReq *d)
{
    const int levels = stream_levels(integrator, t.tsteps);
    const int waves = launch_waves(integrator, levels, t.waves);
    const void *fn = stream_kernel<R>(chi_law, integrator, z != nullptr, levels, t.prefetch, waves);
    if (!fn || t.rows < 1)
        return hipErrorInvalidValue;
    StepArgs<R> a = make_args(f, c);
    if (z)
        a.z = *z;
    const StreamGeom g =
        stream_geom(sizeof(R) == 4 ? 0 : 1, levels, f.nx, f.ny, t.rows, waves, true);
    a.rows = t.rows;
    a.nsx = g.nsx;
    a.nstrips = g.nstrips;
    a.nblocks_padded = g.nblocks_padded;
    a.nsx_main = g.nsx_main;
    a.nmain = g.nmain;
    a.nsy = g.nsy;
    a.fold_bands = g.fold_bands;
    a.fold_lanes = g.fold_lanes;
    a.field_bytes = (uint32_t)((size_t)f.pitch * f.ny * sizeof(R));
    if (d) {
        a.parts = d->parts;
        a.b_thr = d->b_thr;
        a.cx = d->cx;
        a.cy = d->cy;
    }
    void *args[] = {&a};
    return hipLaunchKernel(fn, dim3(g.nblocks_padded), dim3(waves == 2 ? 128 : 256), args, 0, s);
}

template <typename R, bool AVG, bool NOISE>
static void launch_ref_k(int chi_law, dim3 grid, hipStream_t s, const StepArgs<R> &a)
{
    if (chi_law == 0)
        hipLaunchKernelGGL((step_ref<R, 0, AVG, NOISE>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((step_ref<R, 1, AVG, NOISE>), grid, dim3(256), 0, s, a);
}

template <typename R>
hipError_t launch_ref(const Fields<R> &f, const Coef<R> &c, int chi_law, hipStream_t s,
                      const R *b_avg, const R *n_avg, const Noise<R> *z)
{
    StepArgs<R> a = make_args(f, c);
    a.b_avg = b_avg;
    a.n_avg = n_avg;
    if (z)
        a.z = *z;
    const dim3 grid((f.nx + 63) / 64, (f.ny + 3) / 4);
    const bool avg = b_avg != nullptr;
    if (z) {
        if (avg)
            launch_ref_k<R, true, true>(chi_law, grid, s, a);
        else
            launch_ref_k<R, false, true>(chi_law, grid, s, a);
    } else {
        if (avg)
            launch_ref_k<R, true, false>(chi_law, grid, s, a);
        else
            launch_ref_k<R, false, false>(chi_law, grid, s, a);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t time_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, int integrator,
                       const Tuning &t, hipStream_t s, int reps, double *ms, const Noise<R> *z,
                       R *tmp_b, R *tmp_n)
{
    // timed launches: f's output level <-> (tmp_b, tmp_n), or f itself again
    Fields<R> fa = f, fb = f;
    if (tmp_b && tmp_n) {
        fa.b_in = f.b_out;
        fa.n_in = f.n_out;
        fa.b_out = tmp_b;
        fa.n_out = tmp_n;
        fb.b_in = tmp_b;
        fb.n_in = tmp_n;
        fb.b_out = f.b_out;
        fb.n_out = f.n_out;
    }
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess)
        return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    e = launch_stream<R>(f, c, chi_law, integrator, t, s, z);
    if (e == hipSuccess)
        e = hipEventRecord(e0, s);
    for (int i = 0; i < reps && e == hipSuccess; ++i)
        e = launch_stream<R>(i % 2 ? fb : fa, c, chi_law, integrator, t, s, z);
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

int resident_waves(int precision, int chi_law, int integrator, int tsteps, int prefetch,
                   bool noise, int waves)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int levels = stream_levels(integrator, tsteps);
    waves = launch_waves(integrator, levels, waves);
    const void *fn =
        precision == 0 ? stream_kernel<float>(chi_law, integrator, noise, levels, prefetch, waves)
                       : stream_kernel<double>(chi_law, integrator, noise, levels, prefetch, waves);
    int nb = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, waves == 2 ? 128 : 256, 0) !=
                   hipSuccess)
        return 0;
    // resident strips: four per whole-strip workgroup, one per split workgroup
    return nb * (waves == 2 ? 1 : 4) * cus;
}

int round_fitted_rows(int precision, int levels, int nx, int ny, int strips, int rounds)
{
    if (strips <= 0 || rounds <= 0 || nx <= 0 || ny <= 0)
        return 0;
    const StreamGeom g = stream_geom(precision, levels, nx, ny, 1);
    const long m = (long)strips * rounds / g.nsx; // strip rows that fill `rounds` rounds
    if (m <= 0)
        return 0;
    return (int)((ny + m - 1) / m);
}

void tuning_candidates(int effort, int precision, int chi_law, int integrator, bool noise,
                       int nx, int ny, Tuning *out, int *n, int cap)
{
    static const int quick_t[] = {1, 2, 3, 4};
    static const int quick_r[] = {16, 32, 64, 128};
    static const int full_t[] = {1, 2, 3, 4, 6, 8};
    static const int full_r[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 256};
    const int *ts = effort ? full_t : quick_t;
    const int *rs = effort ? full_r : quick_r;
    const int nt = effort ? 6 : 4, nr = effort ? 10 : 4;
    const int max_t = integrator == 0 ? 8 : 3;
    int k = 0;
    auto add = [&](int t, int r, int p, int w) {
        for (int i = 0; i < k && i < cap; ++i)
            if (out[i].tsteps == t && out[i].rows == r && out[i].prefetch == p &&
                out[i].waves == w)
                return;
        if (k < cap) {
            out[k].tsteps = t;
            out[k].rows = r;
            out[k].prefetch = p;
            out[k].waves = w;
        }
        ++k;
    };
    for (int i = 0; i < nt; ++i) {
        if (ts[i] > max_t)
            continue;
        const int levels = stream_levels(integrator, ts[i]);
        for (int w = 1; w <= 2; ++w) {
            if (launch_waves(integrator, levels, w) != w)
                continue; // no split kernel at this depth
            for (int p = 0; p < (effort ? 2 : 1); ++p) {
                const int pf = p ? 2 : 4;
                for (int j = 0; j < nr; ++j)
                    add(ts[i], rs[j], pf, w);
                // rows that fill a whole number of rounds of resident strips
                if (nx <= 0 || ny <= 0)
                    continue;
                const int st = resident_waves(precision, chi_law, integrator, ts[i], pf, noise, w);
                for (int q = 1; q <= 8; ++q) {
                    const int r = round_fitted_rows(precision, levels, nx, ny, st, q);
                    if (r >= 4 && r <= 512)
                        add(ts[i], r, pf, w);
                }
            }
        }
    }
    *n = k < cap ? k : cap;
}

template hipError_t time_stream<float>(const Fields<float> &, const Coef<float> &, int, int,
                                       const Tuning &, hipStream_t, int, double *,
                                       const Noise<float> *, float *, float *);
template hipError_t time_stream<double>(const Fields<double> &, const Coef<double> &, int, int,
                                        const Tuning &, hipStream_t, int, double *,
                                        const Noise<double> *, double *, double *);
template hipError_t launch_stream<float>(const Fields<float> &, const Coef<float> &, int, int,
                                         const Tuning &, hipStream_t, const Noise<float> *,
                                         const DiagReq *);
template hipError_t launch_stream<double>(const Fields<double> &, const Coef<double> &, int, int,
                                          const Tuning &, hipStream_t, const Noise<double> *,
                                          const DiagReq *);
template hipError_t launch_ref<float>(const Fields<float> &, const Coef<float> &, int, hipStream_t,
                                      const float *, const float *, const Noise<float> *);
template hipError_t launch_ref<double>(const Fields<double> &, const Coef<double> &, int,
                                       hipStream_t, const double *, const double *,
                                       const Noise<double> *);

} // namespace kc
