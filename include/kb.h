/*
 * kb.h -- batched parameter sweeps of the chemotaxis system (see kc.h for the
 * equations and the discretisation): many independent instances, each with
 * its own grid, time step, rates, chemotactic strength and agar field, advanced
 * together by one kernel launch per time block of T steps.
 *
 * The paper varies the initial nutrient n0, the chemotactic strength chi0 and
 * the agar field (Sec. 3, table tabresparam) and compares the growth velocity
 * of the colony envelope with its asymptotic bound (Sec. 4.1-4.2).  A batch
 * runs such a sweep: every instance is a kc-style grid in FP32 whose
 * envelope radius R(t), mass and nutrient are sampled on the device at a fixed
 * step interval, and whose velocity is the least-squares slope of R(t) over a
 * radius window.
 *
 * Memory and streams follow kc.h: fields passed in or out are dense row-major
 * [ny][nx] float arrays in host or device memory (KC_MEM_HOST /
 * KC_MEM_DEVICE), the batch keeps padded copies in one device arena, and all
 * work is enqueued on the stream given at creation.  Status codes are kc.h's.
 *
 * Launches.  By default kb_run issues one launch per time block (T steps of
 * every instance); the kernel boundary orders block tau after block tau-1.
 * The optional persistent mode (kb_set_tuning) issues one launch whose
 * wavefronts pull work items (time block, instance, strip) from a global
 * counter in time-block order; an item of block tau waits until the strips of
 * block tau-1 whose output meets its halo window have published their progress
 * flags (device-scope release / acquire).  Every item waited on was handed out
 * earlier, to a running wavefront, so the launch always drains.  Each wait is
 * also bounded (kb_set_spin_limit): a wait that exceeds the bound stops the
 * launch (every other waiting wavefront sees the stop and leaves too) and
 * kb_run reports KC_EHIP; strips that had finished a block have then already
 * overwritten a level, so the fields of every instance must be set again
 * (kb_run and kb_get_fields return KC_ESTATE until kb_set_fields).  On gfx950 a device-scope release or
 * acquire writes back or invalidates the issuing XCD's L2, once per item, so
 * the persistent mode is slower than per-block launches at every batch size
 * measured; the autotuner always selects per-block launches.  A batch whose
 * instances are all single rows (ny = 1) of at most 512 cells, such as the
 * 1-D front experiment of Sec. 4.2, runs each kb_run in one launch outside
 * the persistent mode: one wavefront per instance keeps its row in registers
 * for every step and writes the samples; fields and radii are the same as
 * the per-block launches', mass and nutrient the same sums in another order.
 */
#ifndef KB_H
#define KB_H

#include <stdint.h>

#include "kc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kb_batch kb_batch;

typedef struct {
    int32_t nx, ny;   /* grid cells, >= 1 each                                      */
    double h, dt;     /* cell width, time step (> 0)                                */
    double D_n, theta, kappa, chi; /* rates and chemotactic strength, >= 0 (kc_params) */
    double b_thr;     /* envelope threshold                                         */
    double cx, cy;    /* envelope centre in cell units; NaN = grid centre           */
} kb_instance;

/* Create a batch of count >= 1 instances sharing chi_law (KC_CHI_*), able to
 * hold max_samples >= 1 diagnostic samples per instance.  Allocates one
 * device arena for all fields.  *out is NULL on failure. */
int kb_create(int32_t count, const kb_instance *inst, int32_t chi_law, int32_t max_samples,
              void *hip_stream, kb_batch **out);

/* Set the initial fields of instance k (0 <= k < count); checks and
 * stability bound as kc_set_fields.  Clears the recorded samples of the whole
 * batch and its step count. */
int kb_set_fields(kb_batch *bt, int32_t k, const float *b0, const float *n0, const float *sigma,
                  int mem);

/* Advance every instance by nsteps (a multiple of sample_every >= 1) and
 * record {t, mass, nutrient, envelope_radius, area_radius} (as
 * kc_diagnostics_device) of every instance after each sample_every steps.
 * Per-block launches are enqueued; the persistent mode reads its stop flag
 * back and so synchronises the stream.  Fails with KC_EINVAL when the samples
 * would exceed max_samples. */
int kb_run(kb_batch *bt, int64_t nsteps, int32_t sample_every);

/* Copy the samples out: out is [count][max_samples][5] doubles (unused
 * entries are zero); *nsamples (may be NULL) receives the number recorded.
 * Synchronous. */
int kb_series(kb_batch *bt, double *out, int32_t *nsamples, int mem);

/* Current fields of instance k (synchronous). */
int kb_get_fields(kb_batch *bt, int32_t k, float *b, float *n, int mem);

enum { KB_RADIUS_ENVELOPE = 0, KB_RADIUS_AREA = 1 };

/* Least-squares slope dR/dt of each instance's recorded radius (envelope or
 * area, `radius`) over the samples with r_lo[k] <= R <= r_hi[k] (host arrays
 * of count doubles).  v[k] is NaN when fewer than 3 samples qualify; npoints
 * (may be NULL) receives the sample counts.  Computed on the device;
 * synchronous. */
int kb_fit_velocity(kb_batch *bt, int32_t radius, const double *r_lo, const double *r_hi,
                    double *v, int32_t *npoints);

/* kb_fit_velocity over the samples recorded at times t <= t_max[k] only
 * (t_max: host array of count doubles, +infinity for no limit, or NULL for
 * none at all; a NaN entry is KC_EINVAL): the fit of a run cut at its own end
 * time, e.g. the 1-D experiment of Sec. 4.2, whose slow fronts stall long
 * before the batch's last step. */
int kb_fit_velocity_until(kb_batch *bt, int32_t radius, const double *r_lo, const double *r_hi,
                          const double *t_max, double *v, int32_t *npoints);

/* Kernel configuration.  tsteps: steps per time block (a compiled depth that
 * divides sample_every is used); rows: output rows per strip for each
 * instance (count entries, or NULL to keep); prefetch 2 or 4 (0 keeps);
 * persistent: 1 = one launch per kb_run, 0 = one launch per time block
 * (the default), -1 keeps.  Fields, sample times and radii are bitwise independent of all
 * of these; the double-precision mass and nutrient sums are folded per strip,
 * so a different strip partition changes them at the level of rounding. */
int kb_set_tuning(kb_batch *bt, int32_t tsteps, const int32_t *rows, int32_t prefetch,
                  int32_t persistent);
int kb_get_tuning(const kb_batch *bt, int32_t *tsteps, int32_t *rows, int32_t *prefetch,
                  int32_t *persistent);

/* Pick the time-block depth (a compiled depth dividing sample_every), the
 * prefetch depth and one strip height for all instances (clamped to each
 * grid) by timing per-block launches of the whole batch (current level in,
 * scratch level out: the state is unchanged), and select per-block launches.
 * effort 0 tries depths {2, 3, 4} x heights {16, 32, 64, 128, 256} with
 * prefetch 4; effort 1 depths {1, 2, 3, 4, 6, 8} x ten heights from 8 to 256 x
 * prefetch {2, 4}.  Requires fields on every instance.  Synchronous. */
int kb_autotune(kb_batch *bt, int32_t effort, int32_t sample_every);

/* Bound of each wait of the persistent kernel, in polls (default 2^23, a few
 * seconds).  A tiny bound makes a run stop early with KC_EHIP. */
int kb_set_spin_limit(kb_batch *bt, int64_t polls);

/* Steps done since kb_set_fields. */
int kb_steps(const kb_batch *bt, int64_t *steps);

void kb_destroy(kb_batch *bt);
const char *kb_last_error(const kb_batch *bt);

#ifdef __cplusplus
}
#endif

#endif /* KB_H */
