// kb_batch.hip -- batched parameter sweep: many instances in one launch.
//
// batch_kernel<T, LAW, PF, PERSIST>: every wavefront repeatedly takes one work
// item = (time block tau, instance k, strip j) and advances that strip of
// instance k by T steps with stream_strip (kc_stream.h), so each instance
// goes through the same per-cell arithmetic as the single-instance solver.
//   PERSIST = true : one launch for the whole run; items come from a global
//                    counter in tau-major order.  Strip j of block tau reads (and
//                    overwrites the previous input of) only the strips of block
//                    tau-1 whose output overlaps its halo window, so it waits
//                    (bounded) until each of those has published progress
//                    flag >= tau; it then publishes tau+1 for itself (release
//                    fence, then a device-scope atomic store).
//   PERSIST = false: one launch per time block, item = wavefront index.
// On a sampling block each strip then reads back the cells it stored
// (strip_diag) and folds them into double partials; the last strip of the
// instance to arrive (arrive[k] counter) sums the partials in strip order and
// writes {t, mass, nutrient, envelope radius, area radius}.
// kb_fit: least-squares slope of each instance's R(t) over a radius window.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "kb.h"
#include "kc_internal.h"
#include "kc_stream.h"

namespace kc {

struct BInst {
    float *b[2], *n[2], *sg;
    int nx, ny, pitch, rows;
    int nsx, nstrips, strip0, pad_;
    Coef<float> c;
    double h, dt, b_thr, cx, cy;
};

struct BatchArgs {
    const BInst *inst;
    const int *strip_inst; // instance of each strip of a time block
    int S;                 // strips per time block, all instances
    int T;
    long long total_items; // blocks * S (persistent)
    int tau0;              // first time block of this launch (non-persistent)
    int parity0;           // buffer holding the current level at tau = 0
    int seb;               // sample every `seb` time blocks
    int sample_base;       // series index of the first sample of this run
    int cap;               // samples per instance in the series
    long long step_base;   // steps done before this run
    unsigned long long *next;
    unsigned *flags;  // [S] progress of every strip: blocks completed
    unsigned *fin;    // [count] samples of this run already reduced
    unsigned *arrive, *abort_flag;
    double *partials; // [S][4]
    double *series;   // [count][cap][5]
    long long spin_limit;
};

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

template <int T, int LAW, int PF, bool PERSIST>
__global__ __launch_bounds__(256) void batch_kernel(BatchArgs a)
{
    const int lane = threadIdx.x & 63;
    long long taken = 0; // items handled by this wavefront, at most all of them
    for (;;) {
        if (PERSIST && ++taken > a.total_items) {
            __hip_atomic_store(a.abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        // The loop body has no lane-divergent branches: every lane performs the
        // (identical) stores and the counters are bumped by lane 0's share only,
        // so the wavefront stays converged around the wave-wide broadcasts.
        unsigned long long item;
        if (PERSIST) {
            const unsigned long long got = __hip_atomic_fetch_add(
                a.next, lane == 0 ? 1ull : 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            item = bcast64(got);
            if (item >= (unsigned long long)a.total_items)
                return;
            if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                return;
        } else {
            item = (unsigned long long)__builtin_amdgcn_readfirstlane(blockIdx.x * 4 +
                                                                      (threadIdx.x >> 6));
            if (item >= (unsigned long long)a.S)
                return;
            item += (unsigned long long)a.tau0 * a.S;
        }
        const int tau = (int)(item / (unsigned long long)a.S);
        const int local = (int)(item - (unsigned long long)tau * a.S);
        const int k = a.strip_inst[local];
        const BInst &I = a.inst[k];
        const int j = local - I.strip0;

        if (PERSIST && tau > 0) {
            // strips of block tau-1 whose output rows/columns meet this strip's
            // input window [y0 - T, y1 + T) x [x0 - HX, x0 + OW + HX)
            constexpr int HX = Halo<T, 4>::HX, OW = Halo<T, 4>::OW;
            const int sx = j % I.nsx, sy = j / I.nsx;
            const int nsy = (I.ny + I.rows - 1) / I.rows;
            const int y0 = sy * I.rows, y1 = min(y0 + I.rows, I.ny);
            const int ylo = max(y0 - T, 0), yhi = min(y1 + T, I.ny) - 1;
            const int xlo = max(sx * OW - HX, 0), xhi = sx * OW + OW + HX - 1;
            const int sy_lo = ylo / I.rows, sy_hi = min(yhi / I.rows, nsy - 1);
            const int sx_lo = xlo / OW, sx_hi = min(xhi / OW, I.nsx - 1);
            long long polls = 0;
            for (int qy = sy_lo; qy <= sy_hi; ++qy)
                for (int qx = sx_lo; qx <= sx_hi; ++qx) {
                    const unsigned *f = &a.flags[I.strip0 + qy * I.nsx + qx];
                    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                           (unsigned)tau) {
                        // give up when the bound is exceeded or another wave has stopped
                        if (++polls > a.spin_limit ||
                            __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)) {
                            __hip_atomic_store(a.abort_flag, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            return;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }

        const int par = (a.parity0 + tau) & 1;
        StripArgs<float> sa;
        sa.b_in = I.b[par];
        sa.n_in = I.n[par];
        sa.sg = I.sg;
        sa.b_out = I.b[par ^ 1];
        sa.n_out = I.n[par ^ 1];
        sa.nx = I.nx;
        sa.ny = I.ny;
        sa.pitch = I.pitch;
        sa.rows = I.rows;
        sa.c = I.c;
        sa.b_thr = I.b_thr;
        sa.cx = I.cx;
        sa.cy = I.cy;
        const bool diag = ((tau + 1) % a.seb) == 0;
        DiagAcc acc{0.0, 0.0, -1.0, 0.0};
        {
            const int sx = j % I.nsx, sy = j / I.nsx;
            if (strip_inside<float, T>(sa, sx))
                stream_strip<float, T, LAW, PF, false>(sa, sx, sy);
            else
                stream_strip<float, T, LAW, PF, true>(sa, sx, sy);
            if (diag)
                strip_diag<float, T>(sa, sx, sy, acc);
        }

        if (diag) {
            const double sb = wave_sum64(acc.sb), sn = wave_sum64(acc.sn), m2 = wave_max64(acc.m2);
            const double ct = wave_sum64(acc.cnt);
            const int s = (tau + 1) / a.seb - 1; // sample index within this run
            if (PERSIST && s > 0) {
                // the partial slot of this strip still holds sample s-1 until it is reduced
                long long polls = 0;
                while (__hip_atomic_load(&a.fin[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       (unsigned)s) {
                    if (++polls > a.spin_limit ||
                        __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT)) {
                        __hip_atomic_store(a.abort_flag, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        return;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            a.partials[4 * (size_t)local + 0] = sb;
            a.partials[4 * (size_t)local + 1] = sn;
            a.partials[4 * (size_t)local + 2] = m2;
            a.partials[4 * (size_t)local + 3] = ct;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned prev = __builtin_amdgcn_readfirstlane(__hip_atomic_fetch_add(
                &a.arrive[k], lane == 0 ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (prev + 1 == (unsigned)(s + 1) * (unsigned)I.nstrips) {
                // last strip of this sample: fold the partials in strip order
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                double tb = 0.0, tn = 0.0, tm = -1.0, tc = 0.0;
                for (int jj = lane; jj < I.nstrips; jj += 64) {
                    const size_t q = 4 * (size_t)(I.strip0 + jj);
                    tb += __hip_atomic_load(&a.partials[q + 0], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
                    tn += __hip_atomic_load(&a.partials[q + 1], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
                    tm = fmax(tm, __hip_atomic_load(&a.partials[q + 2], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT));
                    tc += __hip_atomic_load(&a.partials[q + 3], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
                }
                tb = wave_sum64(tb);
                tn = wave_sum64(tn);
                tm = wave_max64(tm);
                tc = wave_sum64(tc);
                double *o = a.series + ((size_t)k * a.cap + a.sample_base + s) * 5;
                o[0] = (double)(a.step_base + (long long)(tau + 1) * a.T) * I.dt;
                o[1] = I.h * I.h * tb;
                o[2] = I.h * I.h * tn;
                o[3] = tm < 0.0 ? 0.0 : I.h * sqrt(tm);
                o[4] = I.h * sqrt(tc / 3.14159265358979323846);
                if (PERSIST) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    __hip_atomic_store(&a.fin[k], (unsigned)(s + 1), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        if (PERSIST) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); // this strip's stores first
            __hip_atomic_store(&a.flags[local], (unsigned)(tau + 1), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            return;
        }
    }
}

__global__ void batch_zero(unsigned *flags, int S, unsigned *arrive, unsigned *fin, int count,
                           unsigned *abort_flag, unsigned long long *next)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S)
        flags[i] = 0u;
    if (i < count) {
        arrive[i] = 0u;
        fin[i] = 0u;
    }
    if (i == 0) {
        *abort_flag = 0u;
        *next = 0ull;
    }
}

__global__ void series_zero(double *series, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        series[i] = 0.0;
}

// Least-squares slope per instance, one wavefront each, fixed order; `col`
// selects the radius (3 envelope, 4 area) of the 5-double samples; win holds
// (lo, hi, t_max) per instance: samples with lo <= R <= hi and t <= t_max.
__global__ __launch_bounds__(64) void kb_fit(const double *series, int cap, int nsamp, int col,
                                             const double *win, double *v, int *npts)
{
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const double lo = win[3 * k], hi = win[3 * k + 1], tmax = win[3 * k + 2];
    const double *S = series + (size_t)k * cap * 5;
    double c = 0.0, st = 0.0, sr = 0.0;
    for (int s = lane; s < nsamp; s += 64) {
        const double R = S[5 * s + col];
        if (R >= lo && R <= hi && S[5 * s + 0] <= tmax) {
            c += 1.0;
            st += S[5 * s + 0];
            sr += R;
        }
    }
    c = wave_sum64(c);
    st = wave_sum64(st);
    sr = wave_sum64(sr);
    const double tm = c > 0 ? st / c : 0.0, rm = c > 0 ? sr / c : 0.0;
    double sxy = 0.0, sxx = 0.0;
    for (int s = lane; s < nsamp; s += 64) {
        const double R = S[5 * s + col];
        if (R >= lo && R <= hi && S[5 * s + 0] <= tmax) {
            const double dt = S[5 * s + 0] - tm;
            sxy += dt * (R - rm);
            sxx += dt * dt;
        }
    }
    sxy = wave_sum64(sxy);
    sxx = wave_sum64(sxx);
    if (lane == 0) {
        v[k] = (c >= 3.0 && sxx > 0.0) ? sxy / sxx : (double)NAN;
        npts[k] = (int)c;
    }
}

// ---------------------------------------------------------------------------
// Single-row batches (every instance 1 x nx, nx <= 64 K, e.g. the 1-D front
// experiment): one wavefront per instance holds the whole row in registers,
// K cells per lane, and runs every step and sample of kb_run in one launch.
// The per-block path would need one launch per time block for a few strips.
// The cell arithmetic is stream_strip's, with the same face, flux and update
// calls on the same operands (the vertical faces of a one-row grid carry +0),
// so the fields are the same bits; samples go to the series like
// batch_kernel's, the radii identical, the sums in another order.
// ---------------------------------------------------------------------------
struct Row1Args {
    const BInst *inst;
    double *series;
    int cap, sample_base, parity0;
    int sample_every, nsamples;
    long long step_base;
};

template <int K, int LAW>
__global__ __launch_bounds__(64) void batch_row_kernel(Row1Args a)
{
    const BInst &I = a.inst[blockIdx.x];
    const int lane = threadIdx.x;
    const int x0 = lane * K;
    const float *bi = I.b[a.parity0], *ni = I.n[a.parity0];
    float b[K], n[K], sh[K];
    bool ve[K]; // east face of the cell is interior
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int x = x0 + k;
        const bool in = x < I.nx;
        b[k] = in ? bi[x] : 0.f;
        n[k] = in ? ni[x] : 0.f;
        sh[k] = in ? 0.5f * I.sg[x] : 0.f;
        ve[k] = x + 1 < I.nx;
    }
    for (int s = 0; s < a.nsamples; ++s) {
        for (int i = 0; i < a.sample_every; ++i) {
            float D[K], X[K], gb[K], gn[K];
#pragma unroll
            for (int k = 0; k < K; ++k)
                coef<float, LAW>(sh[k], n[k], b[k], I.c.chi2, D[k], X[k]);
#pragma unroll
            for (int k = 0; k + 1 < K; ++k)
                face<float>(b[k], n[k], D[k], X[k], b[k + 1], n[k + 1], D[k + 1], X[k + 1], ve[k],
                            gb[k], gn[k]);
            {
                const float eb = from_next(b[0]), en = from_next(n[0]);
                const float eD = from_next(D[0]), eX = from_next(X[0]);
                face<float>(b[K - 1], n[K - 1], D[K - 1], X[K - 1], eb, en, eD, eX, ve[K - 1],
                            gb[K - 1], gn[K - 1]);
            }
            // the west face of lane 0's first cell is the wall: from_prev gives 0
            const float wb = from_prev(gb[K - 1]), wn = from_prev(gn[K - 1]);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float Fb = net<float>(gb[k], k ? gb[k - 1] : wb, 0.f, 0.f);
                const float Fn = net<float>(gn[k], k ? gn[k - 1] : wn, 0.f, 0.f);
                float bo, no;
                update<float>(b[k], n[k], Fb, Fn, I.c, bo, no);
                b[k] = bo;
                n[k] = no;
            }
        }
        // sample: {t, h^2 sum b, h^2 sum n, h sqrt(max d^2), h sqrt(count / pi)}
        double sb = 0.0, sn = 0.0, m2 = -1.0, ct = 0.0;
        const double dy = 0.0 - I.cy;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (x0 + k < I.nx) {
                const double bv = (double)b[k];
                sb += bv;
                sn += (double)n[k];
                if (bv >= I.b_thr) {
                    const double dx = (double)(x0 + k) - I.cx;
                    m2 = fmax(m2, dx * dx + dy * dy);
                    ct += 1.0;
                }
            }
        }
        sb = wave_sum64(sb);
        sn = wave_sum64(sn);
        m2 = wave_max64(m2);
        ct = wave_sum64(ct);
        if (lane == 0) {
            double *o = a.series + ((size_t)blockIdx.x * a.cap + a.sample_base + s) * 5;
            o[0] = (double)(a.step_base + (long long)(s + 1) * a.sample_every) * I.dt;
            o[1] = I.h * I.h * sb;
            o[2] = I.h * I.h * sn;
            o[3] = m2 < 0.0 ? 0.0 : I.h * sqrt(m2);
            o[4] = I.h * sqrt(ct / 3.14159265358979323846);
        }
    }
    float *bo = I.b[a.parity0 ^ 1], *no = I.n[a.parity0 ^ 1];
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (x0 + k < I.nx) {
            bo[x0 + k] = b[k];
            no[x0 + k] = n[k];
        }
}

} // namespace kc

using kc::BInst;

struct kb_batch {
    int count = 0, law = 0, cap = 0;
    hipStream_t stream = nullptr;
    std::vector<kb_instance> inst;
    std::vector<BInst> hinst;
    std::vector<int> rows;
    std::vector<char> has_fields;
    char *arena = nullptr;
    BInst *dinst = nullptr;
    int *dstrip_inst = nullptr;
    unsigned *dflags = nullptr;
    double *dpartials = nullptr, *dseries = nullptr, *dwin = nullptr, *dv = nullptr;
    int *dnpts = nullptr;
    unsigned *dcnt = nullptr; // arrive[count], fin[count], abort
    unsigned long long *dnext = nullptr;
    double *dcheck = nullptr; // input-check partials
    double *hpin = nullptr;   // pinned staging
    size_t hpin_n = 0;
    int cur = 0, nsamp = 0;
    int64_t steps = 0;
    int T = 4, pf = 4, persistent = 0;
    long long spin_limit = 1ll << 23;
    int S = 0, geom_T = -1;
    bool geom_dirty = true;
    int row_cells = 0; // > 0: every instance is one row of at most this many (<= 512) cells
    std::string err;
};

namespace {

int bfail(kb_batch *b, int code, const char *fmt, ...)
{
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return code;
}

int bhip(kb_batch *b, hipError_t e, const char *what)
{
    return bfail(b, e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP, "%s: %s", what,
                 hipGetErrorString(e));
}

#define KB_HIP(bt, expr)                                                                           \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return bhip((bt), e_, #expr);                                                          \
    } while (0)

bool inst_ok(const kb_instance &I)
{
    auto nn = [](double v) { return isfinite(v) && v >= 0.0; };
    return I.nx >= 1 && I.ny >= 1 && I.nx <= (1 << 16) && I.ny <= (1 << 16) && I.h > 0 &&
           isfinite(I.h) && I.dt > 0 && isfinite(I.dt) && nn(I.D_n) && nn(I.theta) &&
           nn(I.kappa) && nn(I.chi) && !isnan(I.b_thr);
}

int default_rows_for(const kb_instance *inst, int count, int k)
{
    // one strip height for the whole batch: as tall as possible (less halo
    // work) while a time block still has about 4096 strips to spread over the
    // device, between 8 and 128 rows, at most the instance's height
    double cells = 0;
    for (int i = 0; i < count; ++i)
        cells += (double)inst[i].nx * inst[i].ny;
    int r = (int)(cells / (248.0 * 4096.0));
    r = r < 8 ? 8 : r > 128 ? 128 : r;
    return r < inst[k].ny ? r : inst[k].ny;
}

// depth used for a run: a compiled depth <= tuned T that divides sample_every
int run_depth(int T, int sample_every)
{
    static const int depths[] = {8, 6, 4, 3, 2, 1};
    for (int d : depths)
        if (d <= T && sample_every % d == 0)
            return d;
    return 1;
}

// Recompute strip geometry for depth T (strip numbering depends on T and rows).
int layout(kb_batch *b, int T)
{
    int S = 0;
    for (int k = 0; k < b->count; ++k) {
        const kc::StreamGeom g = kc::stream_geom(0, T, b->inst[k].nx, b->inst[k].ny, b->rows[k]);
        b->hinst[k].rows = b->rows[k];
        b->hinst[k].nsx = g.nsx;
        b->hinst[k].nstrips = g.nstrips;
        b->hinst[k].strip0 = S;
        S += g.nstrips;
    }
    std::vector<int> si(S);
    for (int k = 0; k < b->count; ++k)
        for (int j = 0; j < b->hinst[k].nstrips; ++j)
            si[b->hinst[k].strip0 + j] = k;
    if (b->dstrip_inst)
        (void)hipFree(b->dstrip_inst);
    if (b->dpartials)
        (void)hipFree(b->dpartials);
    if (b->dflags)
        (void)hipFree(b->dflags);
    b->dstrip_inst = nullptr;
    b->dpartials = nullptr;
    b->dflags = nullptr;
    KB_HIP(b, hipMalloc((void **)&b->dflags, (size_t)S * sizeof(unsigned)));
    KB_HIP(b, hipMalloc((void **)&b->dstrip_inst, (size_t)S * sizeof(int)));
    KB_HIP(b, hipMalloc((void **)&b->dpartials, (size_t)S * 4 * sizeof(double)));
    KB_HIP(b, hipMemcpyAsync(b->dstrip_inst, si.data(), (size_t)S * sizeof(int),
                             hipMemcpyHostToDevice, b->stream));
    KB_HIP(b, hipMemcpyAsync(b->dinst, b->hinst.data(), b->count * sizeof(BInst),
                             hipMemcpyHostToDevice, b->stream));
    KB_HIP(b, hipStreamSynchronize(b->stream));
    b->S = S;
    return KC_OK;
}

template <int T, int LAW, int PF, bool P>
hipError_t launch_batch(const kc::BatchArgs &a, dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((kc::batch_kernel<T, LAW, PF, P>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int T, int LAW, int PF, bool P> const void *kernel_ptr()
{
    return reinterpret_cast<const void *>(&kc::batch_kernel<T, LAW, PF, P>);
}

template <int LAW, int PF, bool P>
hipError_t dispatch_t(int T, const kc::BatchArgs &a, dim3 grid, hipStream_t s, const void **fn)
{
    switch (T) {
#define KB_CASE(TT)                                                                                \
    case TT:                                                                                       \
        if (fn) {                                                                                  \
            *fn = kernel_ptr<TT, LAW, PF, P>();                                                    \
            return hipSuccess;                                                                     \
        }                                                                                          \
        return launch_batch<TT, LAW, PF, P>(a, grid, s);
        KB_CASE(1)
        KB_CASE(2)
        KB_CASE(3)
        KB_CASE(4)
        KB_CASE(6)
        KB_CASE(8)
#undef KB_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t dispatch(int law, int pf, bool persist, int T, const kc::BatchArgs &a, dim3 grid,
                    hipStream_t s, const void **fn = nullptr)
{
    if (law == 0) {
        if (pf == 4)
            return persist ? dispatch_t<0, 4, true>(T, a, grid, s, fn)
                           : dispatch_t<0, 4, false>(T, a, grid, s, fn);
        return persist ? dispatch_t<0, 2, true>(T, a, grid, s, fn)
                       : dispatch_t<0, 2, false>(T, a, grid, s, fn);
    }
    if (pf == 4)
        return persist ? dispatch_t<1, 4, true>(T, a, grid, s, fn)
                       : dispatch_t<1, 4, false>(T, a, grid, s, fn);
    return persist ? dispatch_t<1, 2, true>(T, a, grid, s, fn)
                   : dispatch_t<1, 2, false>(T, a, grid, s, fn);
}

int ensure_pinned(kb_batch *b, size_t n)
{
    if (b->hpin_n >= n)
        return KC_OK;
    if (b->hpin)
        (void)hipHostFree(b->hpin);
    b->hpin = nullptr;
    b->hpin_n = 0;
    KB_HIP(b, hipHostMalloc((void **)&b->hpin, n * sizeof(double), hipHostMallocDefault));
    b->hpin_n = n;
    return KC_OK;
}

} // namespace

extern "C" {

const char *kb_last_error(const kb_batch *b) { return b ? b->err.c_str() : "null batch"; }

void kb_destroy(kb_batch *b)
{
    if (!b)
        return;
    (void)hipStreamSynchronize(b->stream);
    void *ptrs[] = {b->arena, b->dinst, b->dstrip_inst, b->dflags, b->dpartials, b->dseries, b->dwin,
                    b->dv, b->dnpts, b->dcnt, b->dnext, b->dcheck};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    if (b->hpin)
        (void)hipHostFree(b->hpin);
    delete b;
}

int kb_create(int32_t count, const kb_instance *inst, int32_t chi_law, int32_t max_samples,
              void *hip_stream, kb_batch **out)
{
    if (!out)
        return KC_EINVAL;
    *out = nullptr;
    if (count < 1 || count > (1 << 20) || !inst || max_samples < 1 || max_samples > (1 << 24) ||
        (chi_law != KC_CHI_RECEPTOR && chi_law != KC_CHI_CONSTANT))
        return KC_EINVAL;
    for (int k = 0; k < count; ++k)
        if (!inst_ok(inst[k]))
            return KC_EINVAL;
    int dev;
    if (hipGetDevice(&dev) != hipSuccess)
        return KC_EHIP;

    kb_batch *b = new (std::nothrow) kb_batch;
    if (!b)
        return KC_ENOMEM;
    b->count = count;
    b->law = chi_law;
    b->cap = max_samples;
    b->stream = (hipStream_t)hip_stream;
    b->inst.assign(inst, inst + count);
    b->hinst.resize(count);
    b->rows.resize(count);
    b->has_fields.assign(count, 0);
    // single-row batches of short rows run in one launch (batch_row_kernel)
    for (int k = 0; k < count; ++k) {
        if (inst[k].ny != 1 || inst[k].nx > 512) {
            b->row_cells = 0;
            break;
        }
        b->row_cells = std::max(b->row_cells, (int)inst[k].nx);
    }

    // arena: 5 padded fields per instance, each 256-byte aligned
    size_t total = 0;
    std::vector<size_t> off(count);
    for (int k = 0; k < count; ++k) {
        const size_t fb = (size_t)kc::pitch_for(inst[k].nx) * inst[k].ny * sizeof(float);
        off[k] = total;
        total += 5 * ((fb + 255) / 256 * 256);
    }
    int rc = KC_OK;
    hipError_t e = hipMalloc((void **)&b->arena, total);
    if (e == hipSuccess)
        e = hipMemset(b->arena, 0, total);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->dinst, count * sizeof(BInst));
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->dseries, (size_t)count * max_samples * 5 * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->dwin, (size_t)count * 3 * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->dv, (size_t)count * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->dnpts, (size_t)count * sizeof(int));
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->dcnt, (size_t)(2 * count + 1) * sizeof(unsigned));
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->dnext, sizeof(unsigned long long));
    if (e != hipSuccess)
        rc = e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
    if (rc == KC_OK) {
        for (int k = 0; k < count; ++k) {
            const kb_instance &I = inst[k];
            BInst &H = b->hinst[k];
            const size_t fb = (size_t)kc::pitch_for(I.nx) * I.ny * sizeof(float);
            const size_t st = (fb + 255) / 256 * 256;
            char *base = b->arena + off[k];
            H.b[0] = (float *)(base + 0 * st);
            H.n[0] = (float *)(base + 1 * st);
            H.b[1] = (float *)(base + 2 * st);
            H.n[1] = (float *)(base + 3 * st);
            H.sg = (float *)(base + 4 * st);
            H.nx = I.nx;
            H.ny = I.ny;
            H.pitch = kc::pitch_for(I.nx);
            const double lam = I.dt / (I.h * I.h);
            H.c.lam = (float)lam;
            H.c.lamDn = (float)(lam * I.D_n);
            H.c.gro = (float)(I.dt * I.theta * I.kappa);
            H.c.upt = (float)(I.dt * I.kappa);
            H.c.chi2 = (float)(2.0 * I.chi);
            H.h = I.h;
            H.dt = I.dt;
            H.b_thr = I.b_thr;
            H.cx = isnan(I.cx) ? 0.5 * (I.nx - 1) : I.cx;
            H.cy = isnan(I.cy) ? 0.5 * (I.ny - 1) : I.cy;
            H.pad_ = 0;
            b->rows[k] = default_rows_for(inst, count, k);
        }
        hipLaunchKernelGGL(kc::series_zero, dim3(256), dim3(256), 0, b->stream, b->dseries,
                           (size_t)count * max_samples * 5);
        if (hipGetLastError() != hipSuccess)
            rc = KC_EHIP;
    }
    if (rc == KC_OK) {
        rc = layout(b, b->T);
        b->geom_T = b->T;
        b->geom_dirty = false;
    }
    if (rc != KC_OK) {
        kb_destroy(b);
        return rc;
    }
    *out = b;
    return KC_OK;
}

int kb_set_fields(kb_batch *b, int32_t k, const float *b0, const float *n0, const float *sigma,
                  int mem)
{
    if (!b)
        return KC_EINVAL;
    b->err.clear();
    if (k < 0 || k >= b->count || !b0 || !n0 || !sigma ||
        (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE))
        return bfail(b, KC_EINVAL, "bad arguments to kb_set_fields (instance %d)", k);
    const kb_instance &I = b->inst[k];
    const size_t cells = (size_t)I.nx * I.ny;
    double mx = 0.0, rate = 0.0;
    if (mem == KC_MEM_HOST) {
        const int rc = kc::host_check<float>(I.nx, I.ny, b0, n0, sigma, 1.0, I.chi, b->law, &mx,
                                             &rate);
        if (rc != KC_OK)
            return bfail(b, rc, "instance %d: input fields rejected: %s", k, kc_strerror(rc));
    } else {
        const int cp = kc::check_parts(cells);
        if (b->dcheck)
            (void)hipFree(b->dcheck);
        b->dcheck = nullptr;
        KB_HIP(b, hipMalloc((void **)&b->dcheck, 4 * (size_t)cp * sizeof(double)));
        if (ensure_pinned(b, 4 * (size_t)cp) != KC_OK)
            return KC_ENOMEM;
        KB_HIP(b, kc::launch_check<float>(b0, n0, sigma, I.nx, I.ny, 1.0, I.chi, b->law, b->dcheck,
                                          b->stream));
        KB_HIP(b, hipMemcpyAsync(b->hpin, b->dcheck, 4 * cp * sizeof(double),
                                 hipMemcpyDeviceToHost, b->stream));
        KB_HIP(b, hipStreamSynchronize(b->stream));
        double nbad = 0;
        for (int i = 0; i < cp; ++i) {
            nbad += b->hpin[4 * i];
            mx = b->hpin[4 * i + 1] > mx ? b->hpin[4 * i + 1] : mx;
            rate = b->hpin[4 * i + 2] > rate ? b->hpin[4 * i + 2] : rate;
        }
        if (nbad > 0)
            return bfail(b, KC_ENONFINITE, "instance %d: %.0f NaN/Inf/negative entries", k, nbad);
    }
    char msg[256];
    if (kc::stability(I.h, I.dt, I.D_n, mx, rate, msg, sizeof msg) != KC_OK)
        return bfail(b, KC_EUNSTABLE, "instance %d: %s", k, msg);
    const BInst &H = b->hinst[k];
    const hipMemcpyKind kind = mem == KC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const size_t sp = (size_t)I.nx * sizeof(float), dp = (size_t)H.pitch * sizeof(float);
    KB_HIP(b, kc::copy_rows(H.b[b->cur], dp, b0, sp, sp, I.ny, kind, b->stream));
    KB_HIP(b, kc::copy_rows(H.n[b->cur], dp, n0, sp, sp, I.ny, kind, b->stream));
    KB_HIP(b, kc::copy_rows(H.sg, dp, sigma, sp, sp, I.ny, kind, b->stream));
    KB_HIP(b, hipStreamSynchronize(b->stream));
    b->has_fields[k] = 1;
    b->nsamp = 0;
    b->steps = 0;
    hipLaunchKernelGGL(kc::series_zero, dim3(256), dim3(256), 0, b->stream, b->dseries,
                       (size_t)b->count * b->cap * 5);
    KB_HIP(b, hipGetLastError());
    return KC_OK;
}

int kb_run(kb_batch *b, int64_t nsteps, int32_t sample_every)
{
    if (!b)
        return KC_EINVAL;
    b->err.clear();
    if (nsteps < 0 || sample_every < 1 || nsteps % sample_every != 0)
        return bfail(b, KC_EINVAL, "nsteps (%lld) must be a multiple of sample_every (%d) >= 1",
                     (long long)nsteps, sample_every);
    for (int k = 0; k < b->count; ++k)
        if (!b->has_fields[k])
            return bfail(b, KC_ESTATE, "instance %d has no fields", k);
    const int64_t ns = nsteps / sample_every;
    if (b->nsamp + ns > b->cap)
        return bfail(b, KC_EINVAL, "run would record %lld samples, capacity left %d",
                     (long long)ns, b->cap - b->nsamp);
    if (nsteps == 0)
        return KC_OK;
    if (!b->persistent && b->row_cells > 0) {
        // every instance a single row: the whole run in one launch
        kc::Row1Args r;
        r.inst = b->dinst;
        r.series = b->dseries;
        r.cap = b->cap;
        r.sample_base = b->nsamp;
        r.parity0 = b->cur;
        r.sample_every = sample_every;
        r.nsamples = (int)ns;
        r.step_base = b->steps;
        const dim3 grid((unsigned)b->count), block(64);
        const int K = b->row_cells <= 256 ? 4 : 8;
        if (b->law == 0) {
            if (K == 4)
                hipLaunchKernelGGL((kc::batch_row_kernel<4, 0>), grid, block, 0, b->stream, r);
            else
                hipLaunchKernelGGL((kc::batch_row_kernel<8, 0>), grid, block, 0, b->stream, r);
        } else {
            if (K == 4)
                hipLaunchKernelGGL((kc::batch_row_kernel<4, 1>), grid, block, 0, b->stream, r);
            else
                hipLaunchKernelGGL((kc::batch_row_kernel<8, 1>), grid, block, 0, b->stream, r);
        }
        KB_HIP(b, hipGetLastError());
        b->cur ^= 1;
        b->steps += nsteps;
        b->nsamp += (int)ns;
        return KC_OK;
    }
    const int T = run_depth(b->T, sample_every);
    if (b->geom_dirty || T != b->geom_T) { // strip numbering depends on T and rows
        const int rc = layout(b, T);
        if (rc != KC_OK)
            return rc;
        b->geom_dirty = false;
        b->geom_T = T;
    }
    const long long blocks = nsteps / T;

    kc::BatchArgs a;
    a.inst = b->dinst;
    a.strip_inst = b->dstrip_inst;
    a.S = b->S;
    a.T = T;
    a.total_items = blocks * (long long)b->S;
    a.tau0 = 0;
    a.parity0 = b->cur;
    a.seb = sample_every / T;
    a.sample_base = b->nsamp;
    a.cap = b->cap;
    a.step_base = b->steps;
    a.flags = b->dflags;
    a.arrive = b->dcnt;
    a.fin = b->dcnt + b->count;
    a.abort_flag = b->dcnt + 2 * b->count;
    a.next = b->dnext;
    a.partials = b->dpartials;
    a.series = b->dseries;
    a.spin_limit = b->spin_limit;

    {
        const int nz = b->S > b->count ? b->S : b->count;
        hipLaunchKernelGGL(kc::batch_zero, dim3((nz + 255) / 256), dim3(256), 0, b->stream,
                           a.flags, b->S, a.arrive, a.fin, b->count, a.abort_flag, a.next);
    }
    KB_HIP(b, hipGetLastError());
    if (b->persistent) {
        const void *fn = nullptr;
        KB_HIP(b, dispatch(b->law, b->pf, true, T, a, dim3(1), b->stream, &fn));
        int per_cu = 0, dev = 0, cus = 0;
        KB_HIP(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0));
        KB_HIP(b, hipGetDevice(&dev));
        KB_HIP(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        // no more wavefronts than one time block has strips: extra ones would only
        // wait for the previous block
        long long g = (long long)(per_cu > 0 ? per_cu : 1) * cus;
        const long long need = ((long long)b->S + 3) / 4;
        if (g > need)
            g = need;
        KB_HIP(b, dispatch(b->law, b->pf, true, T, a, dim3((unsigned)g), b->stream));
    } else {
        const dim3 grid((unsigned)((b->S + 3) / 4));
        for (long long tau = 0; tau < blocks; ++tau) {
            a.tau0 = (int)tau;
            KB_HIP(b, dispatch(b->law, b->pf, false, T, a, grid, b->stream));
        }
    }
    if (b->persistent) {
        // abort flag back to the host (small, synchronous): a stopped launch is an error
        unsigned abort_h = 0;
        KB_HIP(b, hipMemcpyAsync(&abort_h, a.abort_flag, sizeof(unsigned),
                                 hipMemcpyDeviceToHost, b->stream));
        KB_HIP(b, hipStreamSynchronize(b->stream));
        if (abort_h) {
            // strips that finished a block have already overwritten a level: the
            // fields now mix different times and must be set again
            std::fill(b->has_fields.begin(), b->has_fields.end(), (char)0);
            return bfail(b, KC_EHIP,
                         "persistent batch launch stopped: a wait exceeded %lld polls; the "
                         "fields must be set again",
                         b->spin_limit);
        }
    }
    b->cur = (int)((b->cur + blocks) & 1);
    b->steps += nsteps;
    b->nsamp += (int)ns;
    return KC_OK;
}

int kb_series(kb_batch *b, double *out, int32_t *nsamples, int mem)
{
    if (!b)
        return KC_EINVAL;
    if (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE)
        return bfail(b, KC_EINVAL, "bad memory kind");
    if (nsamples)
        *nsamples = b->nsamp;
    if (out) {
        KB_HIP(b, hipMemcpyAsync(out, b->dseries, (size_t)b->count * b->cap * 5 * sizeof(double),
                                 mem == KC_MEM_HOST ? hipMemcpyDeviceToHost
                                                    : hipMemcpyDeviceToDevice,
                                 b->stream));
        KB_HIP(b, hipStreamSynchronize(b->stream));
    }
    return KC_OK;
}

int kb_get_fields(kb_batch *b, int32_t k, float *bo, float *no, int mem)
{
    if (!b)
        return KC_EINVAL;
    b->err.clear();
    if (k < 0 || k >= b->count || (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE))
        return bfail(b, KC_EINVAL, "bad arguments to kb_get_fields");
    if (!b->has_fields[k])
        return bfail(b, KC_ESTATE, "instance %d has no fields", k);
    const BInst &H = b->hinst[k];
    const hipMemcpyKind kind = mem == KC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    const size_t dp = (size_t)H.nx * sizeof(float), sp = (size_t)H.pitch * sizeof(float);
    if (bo)
        KB_HIP(b, kc::copy_rows(bo, dp, H.b[b->cur], sp, dp, H.ny, kind, b->stream));
    if (no)
        KB_HIP(b, kc::copy_rows(no, dp, H.n[b->cur], sp, dp, H.ny, kind, b->stream));
    KB_HIP(b, hipStreamSynchronize(b->stream));
    return KC_OK;
}

int kb_fit_velocity(kb_batch *b, int32_t radius, const double *r_lo, const double *r_hi,
                    double *v, int32_t *npoints)
{
    return kb_fit_velocity_until(b, radius, r_lo, r_hi, nullptr, v, npoints);
}

int kb_fit_velocity_until(kb_batch *b, int32_t radius, const double *r_lo, const double *r_hi,
                          const double *t_max, double *v, int32_t *npoints)
{
    if (!b)
        return KC_EINVAL;
    b->err.clear();
    if (!r_lo || !r_hi || !v)
        return bfail(b, KC_EINVAL, "null pointer");
    if (radius != KB_RADIUS_ENVELOPE && radius != KB_RADIUS_AREA)
        return bfail(b, KC_EINVAL, "bad radius selector %d", radius);
    if (t_max)
        for (int k = 0; k < b->count; ++k)
            if (isnan(t_max[k]))
                return bfail(b, KC_EINVAL, "t_max[%d] is NaN", k);
    if (ensure_pinned(b, 3 * (size_t)b->count) != KC_OK)
        return KC_ENOMEM;
    for (int k = 0; k < b->count; ++k) {
        b->hpin[3 * k] = r_lo[k];
        b->hpin[3 * k + 1] = r_hi[k];
        b->hpin[3 * k + 2] = t_max ? t_max[k] : (double)INFINITY;
    }
    KB_HIP(b, hipMemcpyAsync(b->dwin, b->hpin, 3 * b->count * sizeof(double),
                             hipMemcpyHostToDevice, b->stream));
    hipLaunchKernelGGL(kc::kb_fit, dim3(b->count), dim3(64), 0, b->stream, b->dseries, b->cap,
                       b->nsamp, radius == KB_RADIUS_AREA ? 4 : 3, b->dwin, b->dv, b->dnpts);
    KB_HIP(b, hipGetLastError());
    KB_HIP(b, hipMemcpyAsync(v, b->dv, b->count * sizeof(double), hipMemcpyDeviceToHost,
                             b->stream));
    std::vector<int> np(b->count);
    KB_HIP(b, hipMemcpyAsync(np.data(), b->dnpts, b->count * sizeof(int), hipMemcpyDeviceToHost,
                             b->stream));
    KB_HIP(b, hipStreamSynchronize(b->stream));
    if (npoints)
        for (int k = 0; k < b->count; ++k)
            npoints[k] = np[k];
    return KC_OK;
}

int kb_set_tuning(kb_batch *b, int32_t tsteps, const int32_t *rows, int32_t prefetch,
                  int32_t persistent)
{
    if (!b)
        return KC_EINVAL;
    b->err.clear();
    if (tsteps < 0 || tsteps > 8 || (prefetch != 0 && prefetch != 2 && prefetch != 4) ||
        persistent < -1 || persistent > 1)
        return bfail(b, KC_EINVAL, "bad tuning");
    if (rows)
        for (int k = 0; k < b->count; ++k)
            if (rows[k] < 1)
                return bfail(b, KC_EINVAL, "rows[%d] < 1", k);
    if (tsteps)
        b->T = kc::stream_depth_at_most(tsteps, kc::INTEG_EULER);
    if (rows) {
        for (int k = 0; k < b->count; ++k)
            b->rows[k] = rows[k];
        b->geom_dirty = true;
    }
    if (prefetch)
        b->pf = prefetch;
    if (persistent >= 0)
        b->persistent = persistent;
    return KC_OK;
}

int kb_get_tuning(const kb_batch *b, int32_t *tsteps, int32_t *rows, int32_t *prefetch,
                  int32_t *persistent)
{
    if (!b)
        return KC_EINVAL;
    if (tsteps)
        *tsteps = b->T;
    if (rows)
        for (int k = 0; k < b->count; ++k)
            rows[k] = b->rows[k];
    if (prefetch)
        *prefetch = b->pf;
    if (persistent)
        *persistent = b->persistent;
    return KC_OK;
}

int kb_autotune(kb_batch *b, int32_t effort, int32_t sample_every)
{
    if (!b)
        return KC_EINVAL;
    b->err.clear();
    if (effort < 0 || effort > 1 || sample_every < 1)
        return bfail(b, KC_EINVAL, "bad autotune arguments");
    for (int k = 0; k < b->count; ++k)
        if (!b->has_fields[k])
            return bfail(b, KC_ESTATE, "instance %d has no fields", k);
    // candidates: depth (dividing sample_every) x prefetch x one strip height for
    // every instance (clamped to its grid); each is timed on the batch itself
    // with per-block launches that read the current level and write the
    // scratch level, so the state is unchanged
    static const int quick_t[] = {2, 3, 4}, full_t[] = {1, 2, 3, 4, 6, 8};
    static const int quick_r[] = {16, 32, 64, 128, 256};
    static const int full_r[] = {8, 16, 24, 32, 48, 64, 96, 128, 192, 256};
    const int *ts = effort ? full_t : quick_t, nt = effort ? 6 : 3;
    const int *rs = effort ? full_r : quick_r, nr = effort ? 10 : 5;
    double cells = 0;
    for (int k = 0; k < b->count; ++k)
        cells += (double)b->inst[k].nx * b->inst[k].ny;
    const std::vector<int> saved_rows = b->rows;
    const int saved_T = b->T, saved_pf = b->pf;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    KB_HIP(b, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(b, KC_EHIP, "hipEventCreate failed");
    }
    double best = 1e300;
    int bT = saved_T, bpf = saved_pf, brows = -1;
    int rc = KC_OK;
    for (int it = 0; it < nt && rc == KC_OK; ++it) {
        const int T = ts[it];
        if (sample_every % T != 0)
            continue;
        for (int ir = 0; ir < nr && rc == KC_OK; ++ir) {
            for (int k = 0; k < b->count; ++k)
                b->rows[k] = rs[ir] < b->inst[k].ny ? rs[ir] : b->inst[k].ny;
            rc = layout(b, T);
            if (rc != KC_OK)
                break;
            kc::BatchArgs a;
            a.inst = b->dinst;
            a.strip_inst = b->dstrip_inst;
            a.S = b->S;
            a.T = T;
            a.total_items = b->S;
            a.tau0 = 0;
            a.parity0 = b->cur;
            a.seb = 1 << 30; // no sampling block among the timed ones
            a.sample_base = 0;
            a.cap = b->cap;
            a.step_base = b->steps;
            a.flags = b->dflags;
            a.arrive = b->dcnt;
            a.fin = b->dcnt + b->count;
            a.abort_flag = b->dcnt + 2 * b->count;
            a.next = b->dnext;
            a.partials = b->dpartials;
            a.series = b->dseries;
            a.spin_limit = b->spin_limit;
            const dim3 grid((unsigned)((b->S + 3) / 4));
            int reps = (int)(2e9 / (cells * T));
            reps = reps < 3 ? 3 : reps > 30 ? 30 : reps;
            for (int p = 0; p < (effort ? 2 : 1) && rc == KC_OK; ++p) {
                const int pf = p ? 2 : 4;
                hipError_t e = dispatch(b->law, pf, false, T, a, grid, b->stream); // warm-up
                if (e == hipSuccess)
                    e = hipEventRecord(e0, b->stream);
                for (int r = 0; r < reps && e == hipSuccess; ++r)
                    e = dispatch(b->law, pf, false, T, a, grid, b->stream);
                if (e == hipSuccess)
                    e = hipEventRecord(e1, b->stream);
                if (e == hipSuccess)
                    e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess)
                    e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc = bfail(b, KC_EHIP, "autotune launch: %s", hipGetErrorString(e));
                    break;
                }
                const double per_step = (double)ms / (reps * T);
                if (per_step < best) {
                    best = per_step;
                    bT = T;
                    bpf = pf;
                    brows = rs[ir];
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != KC_OK) {
        b->rows = saved_rows;
        b->geom_dirty = true;
        return rc;
    }
    if (brows < 0)
        return bfail(b, KC_EINVAL, "no compiled depth divides sample_every = %d", sample_every);
    b->T = bT;
    b->pf = bpf;
    for (int k = 0; k < b->count; ++k)
        b->rows[k] = brows < b->inst[k].ny ? brows : b->inst[k].ny;
    b->persistent = 0;
    b->geom_dirty = true;
    return KC_OK;
}

int kb_set_spin_limit(kb_batch *b, int64_t polls)
{
    if (!b || polls < 1)
        return KC_EINVAL;
    b->spin_limit = polls;
    return KC_OK;
}

int kb_steps(const kb_batch *b, int64_t *steps)
{
    if (!b || !steps)
        return KC_EINVAL;
    *steps = b->steps;
    return KC_OK;
}

} // extern "C"
