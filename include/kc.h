/*
 * kc.h -- C ABI of the MI355X (gfx950) solver for the normalised
 * nutrient / bacteria chemotaxis system of Leyva, Malaga and Plaza,
 * "The effects of nutrient chemotaxis on bacterial aggregation patterns with
 * non-linear degenerate cross diffusion" (arXiv:1301.5058):
 *
 *   n_t = D_n Lap(n) - kappa n b                                   Sec. 2.4, eq. eqnadim
 *   b_t = div(sigma n b grad b) + theta kappa n b
 *         - chi div(sigma n b^2 chihat(n) grad n)                  Sec. 2.4, eq. eqbadim
 *   chihat(n) = 1/(1+n)^2 (receptor law, eq. receptor_law with K_d = 1)
 *             or 1        (constant sensitivity, Sec. 4.1 eq. velo-system)
 *   no-flux boundaries                                              Sec. 2.4, eq. bconds
 *
 * The normalised system has D_n = theta = kappa = 1 and a free agar field
 * sigma = sigma0 (1 + Delta) (eq. CoefCrsDif); the three rates are kept as
 * parameters.  The paper integrates with an explicit finite-difference scheme
 * (Sec. 3).  This library advances the system with forward Euler, or the
 * two-stage Runge-Kutta method (KC_RK2), on nx * ny cell-centred finite
 * volumes of width h: the face diffusivity of the b-flux
 * is the mean of sigma n b over the two cells, the chemotactic coefficient
 * sigma n b^2 chihat(n) is taken from the donor cell (the cell the nutrient
 * gradient points away from), and every boundary face carries zero flux.
 *
 * Layout.  Fields passed in or out are dense row-major [ny][nx] arrays, x
 * fastest, of the context's precision (float for KC_FP32, double for
 * KC_FP64).  Host pointers (KC_MEM_HOST) are ordinary CPU memory; device
 * pointers (KC_MEM_DEVICE) are device memory of the current HIP device.  The
 * context keeps its own padded device copies; the caller keeps ownership of
 * every buffer it passes, and no call retains a caller pointer.
 *
 * Streams.  All device work of a context is enqueued on the hipStream_t
 * given at creation (NULL = the legacy default stream).  kc_step and
 * kc_diagnostics_device return after enqueueing; kc_set_fields,
 * kc_get_fields and kc_diagnostics return after the stream has drained the
 * work they need.
 *
 * Errors.  Every int-returning call returns KC_OK (0) or a negative code
 * below; a message for the last failure of a context is kept until its next
 * call (kc_last_error).  Invalid arguments are rejected before any device
 * work is enqueued.  A context is not thread-safe; distinct contexts are
 * independent.
 */
#ifndef KC_H
#define KC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KC_OK 0
#define KC_EINVAL -1     /* null pointer, nx or ny < 1, h <= 0, dt <= 0, negative rate, bad enum, size overflow */
#define KC_ENONFINITE -2 /* NaN / Inf or negative value in b0, n0 or sigma                               */
#define KC_EUNSTABLE -3  /* dt above the explicit bound of the fields given to kc_set_fields (kc_check_step) */
#define KC_ESTATE -4     /* step / diagnostics / get before kc_set_fields                                */
#define KC_ENOMEM -5     /* device or host allocation failed                                             */
#define KC_EHIP -6       /* no usable device, or a HIP runtime error                                     */

enum { KC_FP32 = 0, KC_FP64 = 1 };
enum { KC_CHI_RECEPTOR = 0, KC_CHI_CONSTANT = 1 };
enum { KC_MEM_HOST = 0, KC_MEM_DEVICE = 1 };
/* Time integrator.  KC_EULER: forward Euler.  KC_RK2: the explicit two-stage
 * Runge-Kutta method the paper integrates with (Sec. 3), read as Heun's method
 * in strong-stability-preserving form: with E one forward-Euler step,
 * u' = (u + E(E(u))) / 2.  Both have the same stability bound. */
enum { KC_EULER = 0, KC_RK2 = 1 };
/* Agar field.  KC_NOISE_STATIC: the sigma field given to kc_set_fields, fixed
 * for the run.  KC_NOISE_PER_STEP: the paper's hardness perturbed at every
 * point and time step (Sec. 3), sigma = sigma0 (1 + noise_amp Delta) with Delta
 * triangular on [-1, 1], drawn from the counter-based generator Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, SC 2011): counter (x / 4, y, step low word,
 * step high word), key (noise_seed low word, high word); cell x takes output
 * word x mod 4, whose 16-bit halves k1, k2 give Delta = (k1 + k2) 2^-16 - 1.
 * `step` is the global step count (step0 + steps taken); the two stages of a
 * KC_RK2 step share the step's field.  Fields are the same for any kernel
 * configuration and any split of a run into kc_step calls. */
enum { KC_NOISE_STATIC = 0, KC_NOISE_PER_STEP = 1 };

typedef struct kc_ctx kc_ctx;

typedef struct {
    int32_t nx; /* cells along x (fastest index), >= 1 */
    int32_t ny; /* cells along y, >= 1                 */
} kc_grid;

typedef struct {
    double D_n;        /* nutrient diffusivity (1 in the normalised system), >= 0           */
    double theta;      /* conversion of consumed nutrient into bacteria (1), >= 0           */
    double kappa;      /* uptake rate of f = kappa n b, eq. goodkinetics (1), >= 0         */
    double chi;        /* chemotactic strength chi_0 >= 0 (Sec. 2.4; 0 = Kawasaki model)   */
    int32_t chi_law;   /* KC_CHI_RECEPTOR or KC_CHI_CONSTANT                                */
    int32_t precision; /* KC_FP32 (fields float, reductions double) or KC_FP64              */
    double b_thr;      /* envelope threshold: cells with b >= b_thr count for the radius   */
    double cx, cy;     /* envelope centre in cell-index units (default (nx-1)/2, (ny-1)/2) */
    int64_t step0;     /* step count at which the given fields sit (time = steps * dt)     */
    int32_t integrator; /* KC_EULER or KC_RK2                                              */
    int32_t noise;      /* KC_NOISE_STATIC or KC_NOISE_PER_STEP                            */
    double sigma0;      /* per-step noise: mean hardness sigma0 > 0                        */
    double noise_amp;   /* per-step noise: amplitude a, 0 <= a <= 1 (a = 1: the paper's)   */
    uint64_t noise_seed; /* per-step noise: generator key                                  */
} kc_params;

/* Fill *p with the normalised defaults: D_n = theta = kappa = 1, chi = 0,
 * receptor law, FP32, b_thr = 0.5, centre unset (NaN -> grid centre), step0 = 0,
 * forward Euler, static agar field (sigma0 = 1, noise_amp = 0, seed 0). */
void kc_default_params(kc_params *p);

/* Create a context for grid g, cell width h > 0 and time step dt > 0 on the
 * current HIP device; hip_stream is a hipStream_t or NULL.  Allocates the
 * padded device fields.  *out receives the context (NULL on failure). */
int kc_create(const kc_grid *g, double h, double dt, const kc_params *p, void *hip_stream,
              kc_ctx **out);

/* Copy initial fields b0 (bacteria), n0 (nutrient) and sigma (agar field,
 * eq. CoefCrsDif) into the context; mem says where the three arrays live.
 * Rejects NaN / Inf / negative entries (KC_ENONFINITE) and a dt above the
 * explicit bounds of kc_check_step for these fields (KC_EUNSTABLE); on failure
 * the context keeps its previous state.  Resets the step count to p->step0.
 * With KC_NOISE_PER_STEP sigma is not used (may be NULL) and the bounds take
 * the largest sigma the noise can draw, sigma0 (1 + noise_amp). */
int kc_set_fields(kc_ctx *ctx, const void *b0, const void *n0, const void *sigma, int mem);

/* Advance nsteps >= 0 time steps of the context's integrator (enqueued,
 * asynchronous). */
int kc_step(kc_ctx *ctx, int64_t nsteps);

/* Diagnostics of the current level, synchronous:
 *   mass = h^2 sum b, nutrient = h^2 sum n (both accumulated in double),
 *   envelope_radius = h * max distance of a cell with b >= b_thr from (cx, cy)
 *   (0 when no cell qualifies).  Any output pointer may be NULL. */
int kc_diagnostics(kc_ctx *ctx, double *mass, double *nutrient, double *envelope_radius);

/* Same diagnostics, enqueued: writes 5 doubles {time, mass, nutrient,
 * envelope_radius, area_radius} to device memory dev_out5 when the stream
 * reaches it; area_radius = h sqrt(N / pi), N the number of cells with
 * b >= b_thr (the radius of a disc of the colony's area). */
int kc_diagnostics_device(kc_ctx *ctx, double *dev_out5);

/* kc_step(ctx, nsteps) followed by kc_diagnostics_device(ctx, dev_out5), with
 * the diagnostics fused into the last step launch: every wavefront strip folds
 * the cells it stores into double partials and one small pass folds those in a
 * fixed order, so no separate read of the fields is made (mass and nutrient
 * are the integrals whose sum the model conserves without growth, Sec. 4.1,
 * eq. mass-conser).  nsteps >= 1 (KC_EINVAL otherwise;
 * dev_out5 non-NULL).  Time and radii equal kc_diagnostics_device's; mass and
 * nutrient are the same sums in another order (equal to about 1e-15
 * relative).  Enqueued, asynchronous.  The first call for a strip count above
 * those seen before allocates a partials buffer of 32 bytes per strip.  With
 * the reference kernel selected it runs kc_step and kc_diagnostics_device. */
int kc_step_sample(kc_ctx *ctx, int64_t nsteps, double *dev_out5);

/* kc_step_sample for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same launches and results as kc_step_sample (fields, time and radii
 * bit for bit; mass and nutrient are the same sums in the same order), but the
 * per-strip partials of the last launch go to a fixed scratch array that the
 * library keeps in device memory (4 doubles per strip, at most
 * KC_NOALLOC_MAX_STRIPS strips: 4 MiB per device, held until the process
 * ends) instead of a buffer of the context, and the call allocates nothing.
 * Every strip writes its own partials before the final pass reads them, so
 * nothing has to be cleared between calls.  All calls on one device share
 * that array: calls that overlap in time on one device (other streams or
 * contexts) race and must be ordered by the caller.  KC_EINVAL when the last
 * launch would have more strips than that (taller strips, kc_set_tuning, fix
 * it) or when the reference kernel is selected; otherwise as kc_step_sample. */
#define KC_NOALLOC_MAX_STRIPS 131072
int kc_step_sample_noalloc(kc_ctx *ctx, int64_t nsteps, double *dev_out5);

/* Copy the current level out (synchronous).  Either pointer may be NULL. */
int kc_get_fields(kc_ctx *ctx, void *b, void *n, int mem);

/* Current time (step count times dt, in double) and step count. */
int kc_time(const kc_ctx *ctx, double *t, int64_t *steps);

/* 0.2 h^2 / max(D_n, max_sigma_n_b): a time step with a 5x margin over the
 * diffusive explicit limit h^2 / (4 max D). */
double kc_suggest_dt(double h, double D_n, double max_sigma_n_b);

/* Host-side check of dense host arrays (no device work): KC_OK, KC_EINVAL for
 * null pointers or bad sizes, KC_ENONFINITE for NaN / Inf / negative entries.
 * *max_sigma_n_b (may be NULL) receives max sigma n b over the cells. */
int kc_check_fields(int32_t nx, int32_t ny, int precision, const void *b0, const void *n0,
                    const void *sigma, double *max_sigma_n_b);

/* Host-side stability check of dense host arrays for a step dt on cells of
 * width h with the rates, sensitivity and noise of *p (no device work; sigma
 * may be NULL with KC_NOISE_PER_STEP, which takes sigma0 (1 + noise_amp)
 * everywhere).  With D = sigma n b, two bounds apply (eqs. eqnadim / eqbadim
 * discretised as in the header comment):
 *   diffusion:   dt <= h^2 / (4 max(D_n, max D)), the explicit limit of both
 *                fields (it keeps n >= 0 and n <= max n0);
 *   positivity:  dt <= h^2 / max_P [ sum_Q (D_P + D_Q) / 2
 *                  + chi sigma_P n_P b_P chihat(n_P) sum_{Q: n_Q > n_P} (n_Q - n_P) ],
 *                Q over the existing neighbours of P: b_P loses at most this
 *                fraction of itself per step through its faces (diffusion and
 *                the donor-cell chemotactic flux toward higher nutrient), so b
 *                stays >= 0.
 * Returns KC_OK, KC_EINVAL (bad arguments), KC_ENONFINITE (NaN / Inf /
 * negative entries) or KC_EUNSTABLE; *dt_max (may be NULL) receives the
 * largest dt both bounds allow for these fields.  The bounds hold for the
 * given fields; a run whose fields sharpen later may need a smaller step. */
int kc_check_step(int32_t nx, int32_t ny, int precision, const void *b0, const void *n0,
                  const void *sigma, double h, double dt, const kc_params *p, double *dt_max);

/* Kernel configuration: tsteps = time steps fused into one launch (1..8; 1..3
 * with KC_RK2, whose steps take two levels of the fused kernel each),
 * rows = output rows per wavefront strip (>= 1), prefetch = rows loaded ahead
 * (2 or 4).  0 keeps the current value.  Results do not depend on it. */
int kc_set_tuning(kc_ctx *ctx, int32_t tsteps, int32_t rows, int32_t prefetch);
int kc_get_tuning(const kc_ctx *ctx, int32_t *tsteps, int32_t *rows, int32_t *prefetch);

/* Wavefronts per strip of the fused kernel: 1 (one wavefront advances a strip
 * through all the levels of a launch) or 2 (two wavefronts of one workgroup
 * share the strip, the first running the first half of the levels and
 * handing each row to the second through LDS: each holds half the state, so
 * twice as many wavefronts fit on a SIMD for the same strips).  2 applies to
 * launches whose levels split into halves of whole time steps (an even number
 * of Euler steps, two Runge-Kutta steps); other launches use 1.  Results do
 * not depend on it.  KC_EINVAL for other values. */
int kc_set_strip_waves(kc_ctx *ctx, int32_t waves);
int kc_get_strip_waves(const kc_ctx *ctx, int32_t *waves);

/* Pick the fused-kernel configuration (as kc_set_tuning and
 * kc_set_strip_waves) by timing candidate launches on the context's own
 * fields: a candidate's first launch reads the current level and writes the
 * scratch level, and its timed launches alternate between the scratch level
 * and a temporary one (allocated for the call and freed before it returns;
 * when it cannot be allocated they repeat the first launch), as a run
 * alternates between its two levels; the current level is never written, so
 * the state is unchanged.  effort 0 tries 4 depths x 4 strip heights with
 * prefetch 4, effort 1 6 depths x 10 heights x prefetch 2 and 4; each with one
 * wavefront per strip and, where the depth splits, two; both add, per depth,
 * prefetch and wavefront count, the strip heights that fill 1..8 whole rounds
 * of the strips the device holds at once.  With use_cache != 0 a matching
 * entry of the file named by the environment variable KC_AUTOTUNE_CACHE (one
 * JSON object per line, keyed by device, grid, precision, law, integrator and
 * noise mode) is used instead of timing, and a new result is appended to it.
 * *gcell_s (may be NULL) receives the best measured rate in 1e9
 * cell-updates/s, or when the cache answered the rate stored with its entry
 * (0 if it has none).  Requires fields (KC_ESTATE).
 * Synchronous. */
int kc_autotune(kc_ctx *ctx, int32_t effort, int32_t use_cache, double *gcell_s);

/* Use the one-step-per-launch global-memory kernel (1) or the fused,
 * register-streaming kernel (0, default).  Both give bitwise equal fields. */
int kc_set_reference_kernel(kc_ctx *ctx, int32_t on);

void kc_destroy(kc_ctx *ctx);
const char *kc_strerror(int status);
const char *kc_last_error(const kc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* KC_H */
