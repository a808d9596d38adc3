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

template <typename R> struct Fields {
    const R *b_in, *n_in, *sg; // current level and agar field sigma
    R *b_out, *n_out;          // next level
    int nx, ny, pitch;
};

struct Tuning {
    int tsteps;   // steps fused in one launch
    int rows;     // output rows per wavefront strip
    int prefetch; // rows loaded ahead (2 or 4)
};

// Largest fused depth with a compiled kernel that is <= t.
int stream_depth_at_most(int t);

// Launch geometry of the fused kernel (for the planner and the autotuner).
struct StreamGeom {
    int nsx, nsy, nstrips, nblocks_padded, out_cols;
};
StreamGeom stream_geom(int precision, int tsteps, int nx, int ny, int rows);

// One launch advancing `tsteps` steps with the fused kernel.
template <typename R>
hipError_t launch_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, const Tuning &t,
                         hipStream_t s);
// One launch advancing one step with the global-memory reference kernel.
template <typename R>
hipError_t launch_ref(const Fields<R> &f, const Coef<R> &c, int chi_law, hipStream_t s);

// Average duration (ms) of one fused launch with tuning t, from `reps` launches
// after one warm-up launch, timed with HIP events on stream s.  The launch
// reads f's input level and writes its output level; nothing else changes.
template <typename R>
hipError_t time_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, const Tuning &t,
                       hipStream_t s, int reps, double *ms);

// Wavefronts of the fused kernel (precision, law, depth, prefetch) that the
// device holds at once: blocks per compute unit x 4 x compute units (0 on error).
int resident_waves(int precision, int chi_law, int tsteps, int prefetch);
// Rows per strip such that the strips fill at most `rounds` rounds of `waves`
// resident wavefronts (0 when no such choice exists).
int round_fitted_rows(int precision, int tsteps, int nx, int ny, int waves, int rounds);

// Candidate configurations of the autotuner: effort 0 is a short list, 1 the
// full grid (tsteps in {1,2,3,4,6,8}, rows in 8..256, prefetch 2 or 4); both
// add, per depth, the rows that fill 1..8 whole rounds of resident wavefronts.
void tuning_candidates(int effort, int max_tsteps, int precision, int chi_law, int nx, int ny,
                       Tuning *out, int *n, int cap);

// Autotune cache: one JSON object per line, keyed by device, grid, precision
// and sensitivity law.  Path from KC_AUTOTUNE_CACHE, else none.
bool cache_lookup(const char *key, Tuning *t);
void cache_store(const char *key, const Tuning &t, double gcells);
int device_key(char *buf, size_t n, int nx, int ny, int precision, int chi_law);

// Diagnostics: partial sums over row blocks (4 doubles each), then one
// fixed-order final pass writing {t, mass, nutrient, envelope radius, area
// radius} to out5 (device doubles).
int diag_parts(int ny);
template <typename R>
hipError_t launch_diag(const R *b, const R *n, int nx, int ny, int pitch, double h, double t,
                       double b_thr, double cx, double cy, double *parts, double *out5,
                       hipStream_t s);

// Input check of dense device arrays: block k writes parts[2k] = number of
// NaN / Inf / negative entries it saw and parts[2k+1] = its max of sigma n b,
// for k < check_parts(cells).
int check_parts(size_t cells);
template <typename R>
hipError_t launch_check(const R *b, const R *n, const R *sg, size_t cells, double *parts,
                        hipStream_t s);

} // namespace kc
