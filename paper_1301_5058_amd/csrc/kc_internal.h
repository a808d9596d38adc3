// kc_internal.h -- launch interface between the C ABI (kc_api.hip) and the
// kernels (kc_step.hip, kc_diag.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kc_device.h"

namespace kc {

// Padded device layout of one field: row y starts at y * pitch elements;
// pitch is nx rounded up to a multiple of 64 elements, padding kept at 0.
inline int pitch_for(int nx) { return (nx + 63) / 64 * 64; }

// Copy of `rows` rows of `width` bytes between buffers with row pitches
// dpitch and spitch, enqueued on s.  When both pitches equal the row width
// (nx a multiple of 64) it is one linear copy: the same bytes, and 2-D copies
// to pageable host memory have returned wrong data under rocprofv3 kernel
// tracing on this ROCm stack while linear ones did not.
inline hipError_t copy_rows(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width,
                            size_t rows, hipMemcpyKind kind, hipStream_t s)
{
    if (dpitch == width && spitch == width)
        return hipMemcpyAsync(dst, src, width * rows, kind, s);
    return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, kind, s);
}

template <typename R> struct Fields {
    const R *b_in, *n_in, *sg; // current level and agar field sigma
    R *b_out, *n_out;          // next level
    int nx, ny, pitch;
};

struct Tuning {
    int tsteps;    // time steps fused in one launch (Euler, or Runge-Kutta: 2 levels each)
    int rows;      // output rows per wavefront strip
    int prefetch;  // rows loaded ahead (2 or 4)
    int waves = 1; // wavefronts per strip: 1 (all levels) or 2 (levels split in halves)
};

// Integrators (kc.h's KC_EULER / KC_RK2).
enum { INTEG_EULER = 0, INTEG_RK2 = 1 };

// Largest fused depth (time steps) with a compiled kernel that is <= t.
int stream_depth_at_most(int t, int integrator);
// Levels (Euler stages) of a launch of `tsteps` steps: the halo width.
int stream_levels(int integrator, int tsteps);

// Launch geometry of the fused kernel (for the planner and the autotuner): a
// whole-strip launch packs four strips into a workgroup, a split launch (two
// wavefronts per strip) one strip.
// With fold, a last strip column that holds few output columns is folded
// (FP32 launches of at most four levels): fold_bands (>= 2) of its strips share
// one wavefront, fold_lanes lanes each (strips [0, nmain) are the first
// nsx_main columns row by row, the rest the folded last column); without,
// nsx_main = nsx, nmain = nstrips, fold_bands = 1.
struct StreamGeom {
    int nsx, nsy, nstrips, nblocks_padded, out_cols;
    int nsx_main, nmain, fold_bands, fold_lanes;
};
StreamGeom stream_geom(int precision, int levels, int nx, int ny, int rows, int waves = 1,
                       bool fold = false);
// Wavefronts per strip a launch of `levels` levels actually uses when `waves`
// are asked for: 2 only where the levels split into two halves of whole time
// steps (an even count; with Runge-Kutta an even number of steps per half).
int launch_waves(int integrator, int levels, int waves);

// Diagnostics fused into a fused-kernel launch: strip k folds the cells it
// stores into parts[4k .. 4k + 3] = {sum b, sum n, max squared distance from
// (cx, cy) of a cell with b >= b_thr (-1: none), count of such cells}.
struct DiagReq {
    double *parts;
    double b_thr, cx, cy;
};

// One launch advancing t.tsteps steps of `integrator` with the fused kernel;
// with z non-null the agar field is redrawn at every step (z's step words are
// the launch's first step) and f.sg is not read; with d non-null the launch
// also writes the diagnostics partials of the level it stores (4 doubles per
// strip, stream_geom(...).nstrips strips).
template <typename R>
hipError_t launch_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, int integrator,
                         const Tuning &t, hipStream_t s, const Noise<R> *z = nullptr,
                         const DiagReq *d = nullptr);
// One forward-Euler step with the global-memory reference kernel; with b_avg
// non-null the result is averaged with (b_avg, n_avg) (Runge-Kutta stage 2);
// with z non-null sigma is drawn for z's step.
template <typename R>
hipError_t launch_ref(const Fields<R> &f, const Coef<R> &c, int chi_law, hipStream_t s,
                      const R *b_avg = nullptr, const R *n_avg = nullptr,
                      const Noise<R> *z = nullptr);

// Average duration (ms) of one fused launch with tuning t, from `reps` launches
// after one warm-up launch, timed with HIP events on stream s.  The warm-up
// reads f's input level and writes its output level.  With tmp_b, tmp_n (a
// spare level of f's size) the timed launches then alternate between f's
// output level and the spare one, as a run's launches alternate between its
// two levels (the same working set; reading one level again and again would
// keep it in the 256 MB last-level cache and flatter the timing); without,
// they repeat the warm-up.  f's input level is never written.
template <typename R>
hipError_t time_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, int integrator,
                       const Tuning &t, hipStream_t s, int reps, double *ms,
                       const Noise<R> *z = nullptr, R *tmp_b = nullptr, R *tmp_n = nullptr);

// Wavefronts of the fused kernel (precision, law, integrator, depth, prefetch)
// that the device holds at once: blocks per compute unit x 4 x compute units
// (0 on error).
int resident_waves(int precision, int chi_law, int integrator, int tsteps, int prefetch,
                   bool noise = false, int waves = 1);
// Rows per strip such that the strips of a launch of `levels` levels fill at
// most `rounds` rounds of `strips` resident strips (0 when none does).
int round_fitted_rows(int precision, int levels, int nx, int ny, int strips, int rounds);

// Candidate configurations of the autotuner: effort 0 is a short list, 1 the
// full grid (tsteps in {1,2,3,4,6,8}, at most 3 for Runge-Kutta, rows in
// 8..256, prefetch 2 or 4), each with one wavefront per strip and, where the
// depth splits into halves of whole steps, two; both add, per depth and
// wavefront count, the rows that fill 1..8 whole rounds of resident strips.
void tuning_candidates(int effort, int precision, int chi_law, int integrator, bool noise,
                       int nx, int ny, Tuning *out, int *n, int cap);

// Autotune cache: one JSON object per line, keyed by device, grid, precision,
// sensitivity law and (for Runge-Kutta) integrator.  Path from KC_AUTOTUNE_CACHE, else none.
// The last entry for `key`; *gcells (if non-null) gets its stored rate (0 if none).
bool cache_lookup(const char *key, int integrator, Tuning *t, double *gcells = nullptr);
void cache_store(const char *key, const Tuning &t, double gcells);
int device_key(char *buf, size_t n, int nx, int ny, int precision, int chi_law, int integrator,
               bool noise = false);

// Diagnostics: partial sums over row blocks (4 doubles each), then one
// fixed-order final pass writing {t, mass, nutrient, envelope radius, area
// radius} to out5 (device doubles).
int diag_parts(int ny);
template <typename R>
hipError_t launch_diag(const R *b, const R *n, int nx, int ny, int pitch, double h, double t,
                       double b_thr, double cx, double cy, double *parts, double *out5,
                       hipStream_t s);
// The fixed-order final pass alone, over `nparts` partials of 4 doubles (those
// of launch_diag or of a launch_stream with diagnostics).
hipError_t launch_diag_fold(const double *parts, int nparts, double h, double t, double *out5,
                            hipStream_t s);

// Input check of dense device arrays [ny][nx]: block k writes
// parts[4k .. 4k + 3] = {number of NaN / Inf / negative entries it saw, its max
// of sigma n b, its max of the donor-cell outflow rate (see host_check), 0} for
// k < check_parts(nx * ny); a null sg counts as sigma = 1 everywhere, and
// sigma is multiplied by sscale.
int check_parts(size_t cells);
template <typename R>
hipError_t launch_check(const R *b, const R *n, const R *sg, int nx, int ny, double sscale,
                        double chi, int law, double *parts, hipStream_t s);

// The same check of dense host arrays: KC_OK or KC_ENONFINITE; *max_snb =
// max sigma n b and *max_rate = max over cells P of
//   sum_Q (D_P + D_Q) / 2 + chi sigma_P n_P b_P chihat(n_P) sum_{Q: n_Q > n_P} (n_Q - n_P)
// (D = sigma n b, Q over the existing neighbours), the outflow rate of b at P
// times h^2: the forward-Euler step keeps b >= 0 when dt max_rate <= h^2.
template <typename R>
int host_check(int nx, int ny, const R *b, const R *n, const R *s, double sscale, double chi,
               int law, double *max_snb, double *max_rate);

// Stability of dt for fields with max sigma n b = max_snb and outflow rate
// max_rate: KC_OK, or KC_EUNSTABLE with a message in msg.
int stability(double h, double dt, double D_n, double max_snb, double max_rate, char *msg,
              size_t msg_n);

} // namespace kc
