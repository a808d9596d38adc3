// kc_api.hip -- the C ABI of include/kc.h: argument checking, device memory,
// launch planning.  Every step of the computation runs in the kernels of
// kc_step.hip and kc_diag.hip; this file only validates, allocates, copies and
// enqueues.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "kc.h"
#include "kc_internal.h"

using kc::Coef;
using kc::Fields;

struct kc_ctx {
    int nx = 0, ny = 0, pitch = 0;
    double h = 0, dt = 0;
    kc_params p{};
    size_t esz = 4;
    hipStream_t stream = nullptr;
    int device = 0;
    void *b[2] = {nullptr, nullptr};
    void *n[2] = {nullptr, nullptr};
    void *b1 = nullptr, *n1 = nullptr; // stage-1 level of the Runge-Kutta reference path
    void *sg = nullptr;
    int cur = 0;
    bool has_fields = false;
    int64_t steps = 0;
    kc::Tuning tune{2, 32, 4, 1};
    bool ref = false;
    double *dparts = nullptr; // diagnostics partials, then out5 (5 doubles)
    double *dout5 = nullptr;
    double *sparts = nullptr; // per-strip partials of a fused sampled step
    size_t sparts_cap = 0;    // in strips
    double *hout = nullptr; // pinned host staging (input check partials, out5)
    std::string err;
};

namespace {

int fail(kc_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

int hipfail(kc_ctx *c, hipError_t e, const char *what)
{
    const int code = (e == hipErrorOutOfMemory) ? KC_ENOMEM : KC_EHIP;
    return fail(c, code, "%s: %s", what, hipGetErrorString(e));
}

#define KC_HIP(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return hipfail((ctx), e_, #expr);                                                      \
    } while (0)

bool finite_nonneg(double v) { return isfinite(v) && v >= 0.0; }

int check_params(const kc_params *p)
{
    if (!p)
        return KC_EINVAL;
    if (!finite_nonneg(p->D_n) || !finite_nonneg(p->theta) || !finite_nonneg(p->kappa) ||
        !finite_nonneg(p->chi))
        return KC_EINVAL;
    if (p->chi_law != KC_CHI_RECEPTOR && p->chi_law != KC_CHI_CONSTANT)
        return KC_EINVAL;
    if (p->precision != KC_FP32 && p->precision != KC_FP64)
        return KC_EINVAL;
    if (isnan(p->b_thr) || p->step0 < 0)
        return KC_EINVAL;
    if (p->integrator != KC_EULER && p->integrator != KC_RK2)
        return KC_EINVAL;
    if (p->noise != KC_NOISE_STATIC && p->noise != KC_NOISE_PER_STEP)
        return KC_EINVAL;
    if (p->noise == KC_NOISE_PER_STEP &&
        (!(p->sigma0 > 0) || !isfinite(p->sigma0) || !(p->noise_amp >= 0) || !(p->noise_amp <= 1)))
        return KC_EINVAL;
    return KC_OK;
}

// Default wavefront-strip height: the fewest whole rounds of the wavefronts the
// device holds at once with strips of at most 128 rows.
int default_rows(int precision, int chi_law, int integrator, bool noise, const kc::Tuning &t,
                 int nx, int ny)
{
    // no half-empty last round; long strips amortise the warm-up rows at either end
    const int w =
        kc::resident_waves(precision, chi_law, integrator, t.tsteps, t.prefetch, noise, t.waves);
    const int levels = kc::stream_levels(integrator, t.tsteps);
    for (int q = 1; q <= 64 && w > 0; ++q) {
        const int r = kc::round_fitted_rows(precision, levels, nx, ny, w, q);
        if (r > 0 && r <= 128)
            return r < 8 ? 8 : r;
    }
    const kc::StreamGeom g = kc::stream_geom(precision, levels, nx, ny, 1);
    long rows = ((long)ny * g.nsx + 2999) / 3000;
    if (rows < 8)
        rows = 8;
    if (rows > 96)
        rows = 96;
    return (int)rows;
}

template <typename R> Coef<R> make_coef(const kc_ctx *c)
{
    const double lam = c->dt / (c->h * c->h);
    Coef<R> k;
    k.lam = (R)lam;
    k.lamDn = (R)(lam * c->p.D_n);
    k.gro = (R)(c->dt * c->p.theta * c->p.kappa);
    k.upt = (R)(c->dt * c->p.kappa);
    k.chi2 = (R)(2.0 * c->p.chi);
    return k;
}

// Per-step noise parameters for a launch starting at the context's current step.
template <typename R> kc::Noise<R> make_noise(const kc_ctx *c)
{
    kc::Noise<R> z;
    // sigma / 2 = h0 + h1 (k1 + k2): sigma0 (1 + a ((k1 + k2) 2^-16 - 1)) / 2
    z.h0 = (R)(0.5 * c->p.sigma0 * (1.0 - c->p.noise_amp));
    z.h1 = (R)(c->p.sigma0 * c->p.noise_amp * 0x1p-17);
    z.k0 = (uint32_t)(c->p.noise_seed & 0xffffffffu);
    z.k1 = (uint32_t)(c->p.noise_seed >> 32);
    z.s_lo = (uint32_t)((uint64_t)c->steps & 0xffffffffu);
    z.s_hi = (uint32_t)((uint64_t)c->steps >> 32);
    return z;
}

template <typename R> Fields<R> make_fields(const kc_ctx *c)
{
    Fields<R> f;
    f.b_in = (const R *)c->b[c->cur];
    f.n_in = (const R *)c->n[c->cur];
    f.sg = (const R *)c->sg;
    f.b_out = (R *)c->b[c->cur ^ 1];
    f.n_out = (R *)c->n[c->cur ^ 1];
    f.nx = c->nx;
    f.ny = c->ny;
    f.pitch = c->pitch;
    return f;
}

// Depth (time steps) of the last fused launch of a kc_step of nsteps >= 1.
int last_launch_depth(const kc_ctx *c, int64_t nsteps)
{
    int d = 1;
    while (nsteps > 0) {
        const int64_t want = nsteps < c->tune.tsteps ? nsteps : c->tune.tsteps;
        d = kc::stream_depth_at_most((int)want, c->p.integrator);
        nsteps -= d;
    }
    return d;
}

// nsteps steps; with dev_out5 non-null (fused kernel only) the last launch also
// folds the level it stores into per-strip partials and a final pass writes the
// diagnostics of that level to dev_out5.  The partials go to ext_parts when it
// is non-null (the caller has checked that the last launch's strips fit),
// otherwise to the context's own buffer, grown when needed.
template <typename R>
int step_impl(kc_ctx *c, int64_t nsteps, double *dev_out5 = nullptr, double *ext_parts = nullptr)
{
    const Coef<R> k = make_coef<R>(c);
    const int integ = c->p.integrator;
    if (c->ref && integ == KC_RK2 && !c->b1) {
        // the reference Runge-Kutta path keeps its first stage in a level of its own
        const size_t bytes = (size_t)c->pitch * c->ny * c->esz;
        hipError_t e = hipMalloc(&c->b1, bytes);
        if (e == hipSuccess)
            e = hipMalloc(&c->n1, bytes);
        if (e == hipSuccess)
            e = hipMemset(c->b1, 0, bytes);
        if (e == hipSuccess)
            e = hipMemset(c->n1, 0, bytes);
        if (e != hipSuccess)
            return hipfail(c, e, "stage-1 level allocation");
    }
    const bool noise = c->p.noise == KC_NOISE_PER_STEP;
    while (nsteps > 0) {
        const Fields<R> f = make_fields<R>(c);
        const kc::Noise<R> z = make_noise<R>(c);
        const kc::Noise<R> *zp = noise ? &z : nullptr;
        hipError_t e;
        int adv;
        if (c->ref && integ == KC_RK2) {
            // u1 = E(u) into the stage level, then u' = (u + E(u1)) / 2
            Fields<R> f1 = f;
            f1.b_out = (R *)c->b1;
            f1.n_out = (R *)c->n1;
            e = kc::launch_ref<R>(f1, k, c->p.chi_law, c->stream, nullptr, nullptr, zp);
            Fields<R> f2 = f;
            f2.b_in = (const R *)c->b1;
            f2.n_in = (const R *)c->n1;
            if (e == hipSuccess)
                e = kc::launch_ref<R>(f2, k, c->p.chi_law, c->stream, f.b_in, f.n_in, zp);
            adv = 1;
        } else if (c->ref) {
            e = kc::launch_ref<R>(f, k, c->p.chi_law, c->stream, nullptr, nullptr, zp);
            adv = 1;
        } else {
            kc::Tuning t = c->tune;
            const int64_t want = nsteps < t.tsteps ? nsteps : t.tsteps;
            t.tsteps = kc::stream_depth_at_most((int)want, integ);
            kc::DiagReq d{nullptr, c->p.b_thr, c->p.cx, c->p.cy};
            int nstrips = 0;
            if (dev_out5 && t.tsteps == nsteps) {
                // the last launch: strip partials of the level it stores
                nstrips = kc::stream_geom(c->p.precision, kc::stream_levels(integ, t.tsteps),
                                          c->nx, c->ny, t.rows, 1, true)
                              .nstrips;
                if (ext_parts) {
                    d.parts = ext_parts;
                } else if ((size_t)nstrips > c->sparts_cap) {
                    if (c->sparts) {
                        KC_HIP(c, hipStreamSynchronize(c->stream));
                        KC_HIP(c, hipFree(c->sparts));
                        c->sparts = nullptr;
                        c->sparts_cap = 0;
                    }
                    KC_HIP(c, hipMalloc((void **)&c->sparts, (size_t)nstrips * 4 * sizeof(double)));
                    c->sparts_cap = (size_t)nstrips;
                }
                if (!ext_parts)
                    d.parts = c->sparts;
            }
            e = kc::launch_stream<R>(f, k, c->p.chi_law, integ, t, c->stream, zp,
                                     d.parts ? &d : nullptr);
            adv = t.tsteps;
            if (e == hipSuccess && d.parts) {
                const double tt = (double)(c->steps + adv) * c->dt;
                e = kc::launch_diag_fold(d.parts, nstrips, c->h, tt, dev_out5, c->stream);
            }
        }
        if (e != hipSuccess)
            return hipfail(c, e, "step kernel launch");
        c->cur ^= 1;
        c->steps += adv;
        nsteps -= adv;
    }
    return KC_OK;
}

} // namespace

namespace kc {

template <typename R>
int host_check(int nx, int ny, const R *b, const R *n, const R *s, double sscale, double chi,
               int law, double *max_snb, double *max_rate)
{
    const size_t cells = (size_t)nx * (size_t)ny;
    double m = 0.0;
    for (size_t i = 0; i < cells; ++i) {
        const double bv = b[i], nv = n[i], sv = s ? s[i] : 1.0;
        if (!(isfinite(bv) && isfinite(nv) && isfinite(sv)) || bv < 0 || nv < 0 || sv < 0)
            return KC_ENONFINITE;
        const double v = sv * sscale * nv * bv;
        if (v > m)
            m = v;
    }
    double rate = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t i = (size_t)y * nx + x;
            const double nP = n[i];
            const double DP = (s ? (double)s[i] : 1.0) * sscale * nP * (double)b[i];
            double dsum = 0.0, up = 0.0;
            const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
            for (int q = 0; q < 4; ++q) {
                const int xq = x + dx[q], yq = y + dy[q];
                if (xq < 0 || xq >= nx || yq < 0 || yq >= ny)
                    continue;
                const size_t j = (size_t)yq * nx + xq;
                const double nQ = n[j];
                dsum += 0.5 * (DP + (s ? (double)s[j] : 1.0) * sscale * nQ * (double)b[j]);
                if (nQ > nP)
                    up += nQ - nP;
            }
            const double ch = law == KC_CHI_RECEPTOR ? 1.0 / ((1.0 + nP) * (1.0 + nP)) : 1.0;
            const double r = dsum + chi * DP * ch * up;
            if (r > rate)
                rate = r;
        }
    if (max_snb)
        *max_snb = m;
    if (max_rate)
        *max_rate = rate;
    return KC_OK;
}

template int host_check<float>(int, int, const float *, const float *, const float *, double,
                               double, int, double *, double *);
template int host_check<double>(int, int, const double *, const double *, const double *, double,
                                double, int, double *, double *);

int stability(double h, double dt, double D_n, double max_snb, double max_rate, char *msg,
              size_t msg_n)
{
    // diffusive bound of both fields, h^2 / (4 max(D_n, sigma n b)), and the
    // positivity bound of the donor-cell b-step, h^2 / max outflow rate
    const double dmax = D_n > max_snb ? D_n : max_snb;
    if (dmax > 0 && dt > h * h / (4.0 * dmax)) {
        snprintf(msg, msg_n, "dt = %g exceeds h^2/(4 max(D_n, sigma n b)) = %g", dt,
                 h * h / (4.0 * dmax));
        return KC_EUNSTABLE;
    }
    if (max_rate > 0 && dt > h * h / max_rate) {
        snprintf(msg, msg_n,
                 "dt = %g exceeds the positivity bound h^2 / max(sum of face diffusivities + "
                 "chemotactic outflow) = %g",
                 dt, h * h / max_rate);
        return KC_EUNSTABLE;
    }
    return KC_OK;
}

} // namespace kc

// Scratch of kc_step_sample_noalloc: the per-strip diagnostics partials (4
// doubles per strip) of its last step launch.  Each device holds its own copy
// for the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns for that device (scratch_parts below).
static __device__ __align__(256) double scratch[4 * (size_t)KC_NOALLOC_MAX_STRIPS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (looked up once per device, with
// that device current).
hipError_t scratch_parts(int device, double **out)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess)
            return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess)
            return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess)
                e = e2;
        }
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = (double *)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

bool sizes_ok(int nx, int ny)
{
    return nx >= 1 && ny >= 1 && nx <= (1 << 20) && ny <= (1 << 20) &&
           (double)kc::pitch_for(nx) * (double)ny < 4.0e9;
}

template <typename R> int autotune_impl(kc_ctx *c, int effort, double *best_out)
{
    const Coef<R> k = make_coef<R>(c);
    const Fields<R> f = make_fields<R>(c); // current level in, scratch level out
    kc::Tuning cand[512];
    int n = 0;
    const bool noise = c->p.noise == KC_NOISE_PER_STEP;
    const kc::Noise<R> z = make_noise<R>(c);
    const kc::Noise<R> *zp = noise ? &z : nullptr;
    kc::tuning_candidates(effort, c->p.precision, c->p.chi_law, c->p.integrator, noise, c->nx,
                          c->ny, cand, &n, 512);
    const double cells = (double)c->nx * c->ny;
    // a spare level, so that the timed launches alternate between two levels
    // like a run's (freed below; without it the launches repeat in place)
    const size_t level = (size_t)c->pitch * c->ny * sizeof(R);
    R *tmp = nullptr;
    if (hipMalloc((void **)&tmp, 2 * level) != hipSuccess) {
        (void)hipGetLastError();
        tmp = nullptr;
    }
    R *tmp_b = tmp, *tmp_n = tmp ? tmp + level / sizeof(R) : nullptr;
    struct Free {
        R *p;
        ~Free()
        {
            if (p)
                (void)hipFree(p);
        }
    } free_tmp{tmp};
    // pass 1: every candidate once; pass 2: the six fastest again, twice each
    // with longer runs, keeping each one's best (single timings are noisy)
    std::vector<std::pair<double, int>> order;
    order.reserve(n);
    for (int i = 0; i < n; ++i) {
        int reps = (int)(2e9 / (cells * cand[i].tsteps)); // about 2e9 cell-updates
        reps = reps < 3 ? 3 : reps > 30 ? 30 : reps;
        double ms = 0;
        hipError_t e =
            kc::time_stream<R>(f, k, c->p.chi_law, c->p.integrator, cand[i], c->stream, reps, &ms,
                               zp, tmp_b, tmp_n);
        if (e != hipSuccess)
            return hipfail(c, e, "autotune launch");
        order.push_back(std::make_pair(ms / cand[i].tsteps, i));
    }
    std::sort(order.begin(), order.end());
    const int top = n < 6 ? n : 6;
    double best = 1e300;
    kc::Tuning bt = c->tune;
    for (int pass = 0; pass < 2; ++pass)
        for (int j = 0; j < top; ++j) {
            const kc::Tuning &t = cand[order[j].second];
            int reps = (int)(6e9 / (cells * t.tsteps));
            reps = reps < 6 ? 6 : reps > 90 ? 90 : reps;
            double ms = 0;
            hipError_t e =
                kc::time_stream<R>(f, k, c->p.chi_law, c->p.integrator, t, c->stream, reps, &ms,
                                   zp, tmp_b, tmp_n);
            if (e != hipSuccess)
                return hipfail(c, e, "autotune launch");
            if (ms / t.tsteps < best) {
                best = ms / t.tsteps;
                bt = t;
            }
        }
    c->tune = bt;
    *best_out = cells / (best * 1e-3) / 1e9;
    return KC_OK;
}

} // namespace

extern "C" {

void kc_default_params(kc_params *p)
{
    if (!p)
        return;
    p->D_n = 1.0;
    p->theta = 1.0;
    p->kappa = 1.0;
    p->chi = 0.0;
    p->chi_law = KC_CHI_RECEPTOR;
    p->precision = KC_FP32;
    p->b_thr = 0.5;
    p->cx = NAN;
    p->cy = NAN;
    p->step0 = 0;
    p->integrator = KC_EULER;
    p->noise = KC_NOISE_STATIC;
    p->sigma0 = 1.0;
    p->noise_amp = 0.0;
    p->noise_seed = 0;
}

const char *kc_strerror(int s)
{
    switch (s) {
    case KC_OK: return "ok";
    case KC_EINVAL: return "invalid argument";
    case KC_ENONFINITE: return "non-finite or negative field value";
    case KC_EUNSTABLE: return "time step above the explicit stability bound";
    case KC_ESTATE: return "fields not set";
    case KC_ENOMEM: return "out of memory";
    case KC_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char *kc_last_error(const kc_ctx *c) { return c ? c->err.c_str() : "null context"; }

double kc_suggest_dt(double h, double D_n, double max_sigma_n_b)
{
    const double m = D_n > max_sigma_n_b ? D_n : max_sigma_n_b;
    if (!(h > 0) || !(m > 0))
        return 0.0;
    return 0.2 * h * h / m;
}

int kc_check_fields(int32_t nx, int32_t ny, int precision, const void *b0, const void *n0,
                    const void *sigma, double *max_sigma_n_b)
{
    if (!b0 || !n0 || !sigma || !sizes_ok(nx, ny))
        return KC_EINVAL;
    if (precision == KC_FP32)
        return kc::host_check<float>(nx, ny, (const float *)b0, (const float *)n0,
                                     (const float *)sigma, 1.0, 0.0, KC_CHI_CONSTANT,
                                     max_sigma_n_b, nullptr);
    if (precision == KC_FP64)
        return kc::host_check<double>(nx, ny, (const double *)b0, (const double *)n0,
                                      (const double *)sigma, 1.0, 0.0, KC_CHI_CONSTANT,
                                      max_sigma_n_b, nullptr);
    return KC_EINVAL;
}

int kc_check_step(int32_t nx, int32_t ny, int precision, const void *b0, const void *n0,
                  const void *sigma, double h, double dt, const kc_params *p, double *dt_max)
{
    if (dt_max)
        *dt_max = 0.0;
    if (!b0 || !n0 || !sizes_ok(nx, ny) || !(h > 0) || !isfinite(h) || !(dt > 0) ||
        !isfinite(dt) || check_params(p) != KC_OK || (precision != KC_FP32 && precision != KC_FP64))
        return KC_EINVAL;
    const bool noise = p->noise == KC_NOISE_PER_STEP;
    if (!noise && !sigma)
        return KC_EINVAL;
    const double sscale = noise ? p->sigma0 * (1.0 + p->noise_amp) : 1.0;
    if (noise)
        sigma = nullptr;
    double mx = 0.0, rate = 0.0;
    const int rc = precision == KC_FP32
                       ? kc::host_check<float>(nx, ny, (const float *)b0, (const float *)n0,
                                               (const float *)sigma, sscale, p->chi, p->chi_law,
                                               &mx, &rate)
                       : kc::host_check<double>(nx, ny, (const double *)b0, (const double *)n0,
                                                (const double *)sigma, sscale, p->chi, p->chi_law,
                                                &mx, &rate);
    if (rc != KC_OK)
        return rc;
    double lim = 4.0 * (p->D_n > mx ? p->D_n : mx);
    if (rate > lim)
        lim = rate;
    if (dt_max)
        *dt_max = lim > 0 ? h * h / lim : INFINITY;
    char msg[256];
    return kc::stability(h, dt, p->D_n, mx, rate, msg, sizeof msg);
}

int kc_create(const kc_grid *g, double h, double dt, const kc_params *p, void *hip_stream,
              kc_ctx **out)
{
    if (!out)
        return KC_EINVAL;
    *out = nullptr;
    if (!g || !sizes_ok(g->nx, g->ny) || !(h > 0) || !isfinite(h) || !(dt > 0) || !isfinite(dt))
        return KC_EINVAL;
    if (check_params(p) != KC_OK)
        return KC_EINVAL;

    kc_ctx *c = new (std::nothrow) kc_ctx;
    if (!c)
        return KC_ENOMEM;
    c->nx = g->nx;
    c->ny = g->ny;
    c->pitch = kc::pitch_for(g->nx);
    c->h = h;
    c->dt = dt;
    c->p = *p;
    if (isnan(c->p.cx))
        c->p.cx = 0.5 * (c->nx - 1);
    if (isnan(c->p.cy))
        c->p.cy = 0.5 * (c->ny - 1);
    c->esz = p->precision == KC_FP32 ? 4 : 8;
    c->stream = (hipStream_t)hip_stream;
    c->steps = p->step0;
    // deepest block without register spills on gfx950, 4 levels (the autotuner
    // can change it)
    c->tune.tsteps = p->integrator == KC_RK2 ? 2 : 4;
    c->tune.prefetch = 4;
    c->tune.rows = default_rows(p->precision, p->chi_law, p->integrator,
                                p->noise == KC_NOISE_PER_STEP, c->tune, c->nx, c->ny);

    int rc = KC_OK;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return KC_EHIP;
    }
    const size_t bytes = (size_t)c->pitch * c->ny * c->esz;
    void **bufs[5] = {&c->b[0], &c->n[0], &c->b[1], &c->n[1], &c->sg};
    for (void **bp : bufs) {
        e = hipMalloc(bp, bytes);
        if (e != hipSuccess) {
            rc = e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
            break;
        }
        e = hipMemset(*bp, 0, bytes);
        if (e != hipSuccess) {
            rc = KC_EHIP;
            break;
        }
    }
    if (rc == KC_OK) {
        const int np = kc::diag_parts(c->ny);
        const size_t cells = (size_t)c->nx * c->ny;
        const int cp = kc::check_parts(cells);
        const size_t nparts = (size_t)(4 * np > 4 * cp ? 4 * np : 4 * cp);
        e = hipMalloc((void **)&c->dparts, (nparts + 5) * sizeof(double));
        if (e != hipSuccess)
            rc = e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
        else
            c->dout5 = c->dparts + nparts;
    }
    if (rc == KC_OK) {
        e = hipHostMalloc((void **)&c->hout, (4 * kc::check_parts((size_t)c->nx * c->ny) + 5) *
                                                 sizeof(double),
                          hipHostMallocDefault);
        if (e != hipSuccess)
            rc = KC_ENOMEM;
    }
    if (rc != KC_OK) {
        kc_destroy(c);
        return rc;
    }
    *out = c;
    return KC_OK;
}

void kc_destroy(kc_ctx *c)
{
    if (!c)
        return;
    if (c->stream || c->b[0])
        (void)hipStreamSynchronize(c->stream);
    for (void *q : {c->b[0], c->n[0], c->b[1], c->n[1], c->sg, c->b1, c->n1, (void *)c->sparts})
        if (q)
            (void)hipFree(q);
    if (c->dparts)
        (void)hipFree(c->dparts);
    if (c->hout)
        (void)hipHostFree(c->hout);
    delete c;
}

int kc_set_fields(kc_ctx *c, const void *b0, const void *n0, const void *sigma, int mem)
{
    if (!c)
        return KC_EINVAL;
    c->err.clear();
    const bool noise = c->p.noise == KC_NOISE_PER_STEP;
    if (!b0 || !n0 || (!sigma && !noise))
        return fail(c, KC_EINVAL, "null field pointer");
    if (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE)
        return fail(c, KC_EINVAL, "bad memory kind %d", mem);
    const size_t cells = (size_t)c->nx * c->ny;
    // with per-step noise the check takes sigma = 1 (a null sigma) scaled by the
    // largest sigma the noise can draw, sigma0 (1 + amp)
    const double sscale = noise ? c->p.sigma0 * (1.0 + c->p.noise_amp) : 1.0;
    if (noise)
        sigma = nullptr;
    double mx = 0.0, rate = 0.0;
    int rc = KC_OK;
    if (mem == KC_MEM_HOST) {
        rc = c->p.precision == KC_FP32
                 ? kc::host_check<float>(c->nx, c->ny, (const float *)b0, (const float *)n0,
                                         (const float *)sigma, sscale, c->p.chi, c->p.chi_law, &mx,
                                         &rate)
                 : kc::host_check<double>(c->nx, c->ny, (const double *)b0, (const double *)n0,
                                          (const double *)sigma, sscale, c->p.chi, c->p.chi_law,
                                          &mx, &rate);
        if (rc != KC_OK)
            rc = fail(c, rc, "input fields rejected: %s", kc_strerror(rc));
    } else {
        const int cp = kc::check_parts(cells);
        hipError_t e = c->p.precision == KC_FP32
                           ? kc::launch_check<float>((const float *)b0, (const float *)n0,
                                                     (const float *)sigma, c->nx, c->ny, sscale,
                                                     c->p.chi, c->p.chi_law, c->dparts, c->stream)
                           : kc::launch_check<double>((const double *)b0, (const double *)n0,
                                                      (const double *)sigma, c->nx, c->ny, sscale,
                                                      c->p.chi, c->p.chi_law, c->dparts,
                                                      c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->hout, c->dparts, 4 * cp * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            rc = hipfail(c, e, "input check kernel");
        } else {
            double nbad = 0.0;
            for (int i = 0; i < cp; ++i) {
                nbad += c->hout[4 * i];
                mx = c->hout[4 * i + 1] > mx ? c->hout[4 * i + 1] : mx;
                rate = c->hout[4 * i + 2] > rate ? c->hout[4 * i + 2] : rate;
            }
            if (nbad > 0)
                rc = fail(c, KC_ENONFINITE, "input fields rejected: %.0f NaN/Inf/negative entries",
                          nbad);
        }
    }
    if (rc != KC_OK)
        return rc;
    char msg[256];
    if (kc::stability(c->h, c->dt, c->p.D_n, mx, rate, msg, sizeof msg) != KC_OK)
        return fail(c, KC_EUNSTABLE, "%s", msg);

    const hipMemcpyKind kind = mem == KC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const size_t spitch = (size_t)c->nx * c->esz, dpitch = (size_t)c->pitch * c->esz;
    c->cur = 0;
    KC_HIP(c, kc::copy_rows(c->b[0], dpitch, b0, spitch, spitch, c->ny, kind, c->stream));
    KC_HIP(c, kc::copy_rows(c->n[0], dpitch, n0, spitch, spitch, c->ny, kind, c->stream));
    if (!noise)
        KC_HIP(c, kc::copy_rows(c->sg, dpitch, sigma, spitch, spitch, c->ny, kind, c->stream));
    KC_HIP(c, hipStreamSynchronize(c->stream));
    c->has_fields = true;
    c->steps = c->p.step0;
    return KC_OK;
}

int kc_step(kc_ctx *c, int64_t nsteps)
{
    if (!c)
        return KC_EINVAL;
    c->err.clear();
    if (nsteps < 0)
        return fail(c, KC_EINVAL, "negative step count");
    if (!c->has_fields)
        return fail(c, KC_ESTATE, "kc_step before kc_set_fields");
    return c->p.precision == KC_FP32 ? step_impl<float>(c, nsteps) : step_impl<double>(c, nsteps);
}

int kc_step_sample(kc_ctx *c, int64_t nsteps, double *dev_out5)
{
    if (!c || !dev_out5)
        return KC_EINVAL;
    c->err.clear();
    if (nsteps < 1)
        return fail(c, KC_EINVAL, "kc_step_sample needs at least one step");
    if (!c->has_fields)
        return fail(c, KC_ESTATE, "kc_step_sample before kc_set_fields");
    if (c->ref) {
        // the reference kernel has no fused diagnostics: step, then the separate pass
        const int rc = kc_step(c, nsteps);
        return rc != KC_OK ? rc : kc_diagnostics_device(c, dev_out5);
    }
    return c->p.precision == KC_FP32 ? step_impl<float>(c, nsteps, dev_out5)
                                     : step_impl<double>(c, nsteps, dev_out5);
}

int kc_step_sample_noalloc(kc_ctx *c, int64_t nsteps, double *dev_out5)
{
    if (!c || !dev_out5)
        return KC_EINVAL;
    c->err.clear();
    if (nsteps < 1)
        return fail(c, KC_EINVAL, "kc_step_sample_noalloc needs at least one step");
    if (!c->has_fields)
        return fail(c, KC_ESTATE, "kc_step_sample_noalloc before kc_set_fields");
    if (c->ref)
        return fail(c, KC_EINVAL,
                    "kc_step_sample_noalloc runs the fused kernel only (reference kernel selected)");
    const int d = last_launch_depth(c, nsteps);
    const int nstrips = kc::stream_geom(c->p.precision, kc::stream_levels(c->p.integrator, d),
                                        c->nx, c->ny, c->tune.rows, 1, true)
                            .nstrips;
    if (nstrips > KC_NOALLOC_MAX_STRIPS)
        return fail(c, KC_EINVAL,
                    "the last launch has %d strips, more than the %d the scratch of "
                    "kc_step_sample_noalloc holds (use taller strips or kc_step_sample)",
                    nstrips, KC_NOALLOC_MAX_STRIPS);
    double *parts = nullptr;
    KC_HIP(c, scratch_parts(c->device, &parts));
    return c->p.precision == KC_FP32 ? step_impl<float>(c, nsteps, dev_out5, parts)
                                     : step_impl<double>(c, nsteps, dev_out5, parts);
}

int kc_diagnostics_device(kc_ctx *c, double *dev_out5)
{
    if (!c || !dev_out5)
        return KC_EINVAL;
    c->err.clear();
    if (!c->has_fields)
        return fail(c, KC_ESTATE, "diagnostics before kc_set_fields");
    const double t = (double)c->steps * c->dt;
    hipError_t e;
    if (c->p.precision == KC_FP32)
        e = kc::launch_diag<float>((const float *)c->b[c->cur], (const float *)c->n[c->cur], c->nx,
                                   c->ny, c->pitch, c->h, t, c->p.b_thr, c->p.cx, c->p.cy,
                                   c->dparts, dev_out5, c->stream);
    else
        e = kc::launch_diag<double>((const double *)c->b[c->cur], (const double *)c->n[c->cur],
                                    c->nx, c->ny, c->pitch, c->h, t, c->p.b_thr, c->p.cx, c->p.cy,
                                    c->dparts, dev_out5, c->stream);
    if (e != hipSuccess)
        return hipfail(c, e, "diagnostics launch");
    return KC_OK;
}

int kc_diagnostics(kc_ctx *c, double *mass, double *nutrient, double *radius)
{
    const int rc = kc_diagnostics_device(c, c ? c->dout5 : nullptr);
    if (rc != KC_OK)
        return rc;
    KC_HIP(c, hipMemcpyAsync(c->hout, c->dout5, 5 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    KC_HIP(c, hipStreamSynchronize(c->stream));
    if (!isfinite(c->hout[1]) || !isfinite(c->hout[2]))
        return fail(c, KC_ENONFINITE, "non-finite mass or nutrient (mass %g, nutrient %g)",
                    c->hout[1], c->hout[2]);
    if (mass)
        *mass = c->hout[1];
    if (nutrient)
        *nutrient = c->hout[2];
    if (radius)
        *radius = c->hout[3];
    return KC_OK;
}

int kc_get_fields(kc_ctx *c, void *b, void *n, int mem)
{
    if (!c)
        return KC_EINVAL;
    c->err.clear();
    if (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE)
        return fail(c, KC_EINVAL, "bad memory kind %d", mem);
    if (!c->has_fields)
        return fail(c, KC_ESTATE, "kc_get_fields before kc_set_fields");
    const hipMemcpyKind kind = mem == KC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    const size_t dpitch = (size_t)c->nx * c->esz, spitch = (size_t)c->pitch * c->esz;
    if (b)
        KC_HIP(c, kc::copy_rows(b, dpitch, c->b[c->cur], spitch, dpitch, c->ny, kind, c->stream));
    if (n)
        KC_HIP(c, kc::copy_rows(n, dpitch, c->n[c->cur], spitch, dpitch, c->ny, kind, c->stream));
    KC_HIP(c, hipStreamSynchronize(c->stream));
    return KC_OK;
}

int kc_time(const kc_ctx *c, double *t, int64_t *steps)
{
    if (!c)
        return KC_EINVAL;
    if (t)
        *t = (double)c->steps * c->dt;
    if (steps)
        *steps = c->steps;
    return KC_OK;
}

int kc_set_tuning(kc_ctx *c, int32_t tsteps, int32_t rows, int32_t prefetch)
{
    if (!c)
        return KC_EINVAL;
    c->err.clear();
    if (tsteps < 0 || tsteps > 8 || rows < 0 || (prefetch != 0 && prefetch != 2 && prefetch != 4))
        return fail(c, KC_EINVAL, "bad tuning (%d, %d, %d)", tsteps, rows, prefetch);
    if (tsteps)
        c->tune.tsteps = kc::stream_depth_at_most(tsteps, c->p.integrator);
    if (rows)
        c->tune.rows = rows;
    if (prefetch)
        c->tune.prefetch = prefetch;
    return KC_OK;
}

int kc_get_tuning(const kc_ctx *c, int32_t *tsteps, int32_t *rows, int32_t *prefetch)
{
    if (!c)
        return KC_EINVAL;
    if (tsteps)
        *tsteps = c->tune.tsteps;
    if (rows)
        *rows = c->tune.rows;
    if (prefetch)
        *prefetch = c->tune.prefetch;
    return KC_OK;
}

int kc_set_strip_waves(kc_ctx *c, int32_t waves)
{
    if (!c)
        return KC_EINVAL;
    c->err.clear();
    if (waves != 1 && waves != 2)
        return fail(c, KC_EINVAL, "wavefronts per strip must be 1 or 2 (got %d)", waves);
    c->tune.waves = waves;
    return KC_OK;
}

int kc_get_strip_waves(const kc_ctx *c, int32_t *waves)
{
    if (!c || !waves)
        return KC_EINVAL;
    *waves = c->tune.waves;
    return KC_OK;
}

int kc_autotune(kc_ctx *c, int32_t effort, int32_t use_cache, double *gcell_s)
{
    if (!c)
        return KC_EINVAL;
    c->err.clear();
    if (effort < 0 || effort > 1)
        return fail(c, KC_EINVAL, "effort must be 0 or 1");
    if (!c->has_fields)
        return fail(c, KC_ESTATE, "kc_autotune before kc_set_fields");
    char key[256];
    kc::device_key(key, sizeof key, c->nx, c->ny, c->p.precision, c->p.chi_law,
                   c->p.integrator, c->p.noise == KC_NOISE_PER_STEP);
    if (gcell_s)
        *gcell_s = 0.0;
    kc::Tuning t;
    double stored = 0.0;
    if (use_cache && kc::cache_lookup(key, c->p.integrator, &t, &stored)) {
        c->tune = t;
        if (gcell_s)
            *gcell_s = stored;
        return KC_OK;
    }
    double g = 0.0;
    const int rc = c->p.precision == KC_FP32 ? autotune_impl<float>(c, effort, &g)
                                             : autotune_impl<double>(c, effort, &g);
    if (rc != KC_OK)
        return rc;
    if (use_cache)
        kc::cache_store(key, c->tune, g);
    if (gcell_s)
        *gcell_s = g;
    return KC_OK;
}

int kc_set_reference_kernel(kc_ctx *c, int32_t on)
{
    if (!c)
        return KC_EINVAL;
    c->ref = on != 0;
    return KC_OK;
}

} // extern "C"
