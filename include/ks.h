/*
 * ks.h -- learned surrogate of the colony-envelope velocity.
 *
 * The paper estimates the envelope speed with the closed-form bound
 * cbar(n0, chi0) of Sec. 4.1 (eqs. c-bar-chi0, c-bar-0) and with 1-D
 * simulations (Sec. 4.2).  This surrogate instead learns the velocity that the
 * batched solver (kb.h) measures, as a function of (n0, chi, a) -- initial
 * nutrient, chemotactic strength and agar-noise amplitude -- and falls back to
 * the solver outside the convex hull of its training inputs.
 *
 * Network: 3 -> 64 -> 64 -> 64 -> 1, GELU (exact erf form) after each hidden
 * layer, weights and hidden activations rounded to bfloat16, every product
 * accumulated in float32 (the two 64 x 64 layers and their gradients on
 * MFMA).  Inputs and targets pass through caller-chosen affine maps:
 *   x' = (x - in_shift) / in_scale,   v = v' * out_scale + out_shift,
 * or, in log-target mode, v = exp(v' * out_scale + out_shift) (targets y are
 * mapped as (log y - out_shift) / out_scale, so the loss weighs relative
 * errors).  Training minimises the mean squared error of v' against the
 * mapped targets with Adam (float32 master weights and moments).
 *
 * Parameter vector (float32, 8641 entries, row-major [out][in] weights):
 *   W1[64][3] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4
 *
 * Memory: X is [n][3] float (n0, chi, a per row), targets and outputs are [n]
 * float; mem = KC_MEM_HOST or KC_MEM_DEVICE as in kc.h.  Work is enqueued on
 * the stream given at creation; calls that return values to the host are
 * synchronous.  Status codes are kc.h's.
 */
#ifndef KS_H
#define KS_H

#include <stdint.h>

#include "kc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define KS_NPARAM 8641

typedef struct ks_model ks_model;

/* Create a model with all parameters zero; max_points bounds n in every call. */
int ks_create(int32_t max_points, void *hip_stream, ks_model **out);

/* Set / read the float32 master parameters (host arrays of KS_NPARAM).
 * Setting also clears the Adam moments and step count. */
int ks_set_params(ks_model *m, const float *params);
int ks_get_params(ks_model *m, float *params);

/* Affine maps of inputs (3 shifts, 3 non-zero scales) and of the output;
 * log_target 1 selects log-target mode (targets must then be > 0). */
int ks_set_normalization(ks_model *m, const double *in_shift, const double *in_scale,
                         double out_shift, double out_scale, int32_t log_target);

/* iters Adam steps (learning rate lr > 0, beta1 0.9, beta2 0.999, eps 1e-8)
 * on minibatches of `batch` consecutive points, cycling through the n points.
 * *loss (may be NULL) receives the mean squared error of the last minibatch
 * in mapped units. */
int ks_train(ks_model *m, const float *X, const float *v, int32_t n, int32_t iters, int32_t batch,
             double lr, int mem, double *loss);

/* Gradient of the mean squared error over all n points with respect to the
 * parameters (host array of KS_NPARAM floats) and the loss; for checks. */
int ks_grad(ks_model *m, const float *X, const float *v, int32_t n, float *grad, double *loss,
            int mem);

/* Predicted velocities v[n] (in target units). */
int ks_predict(ks_model *m, const float *X, int32_t n, float *v, int mem);

/* Training hull: nf facets (a_f . x + b_f <= 0 inside), as rows
 * {a0, a1, a2, b} of facets[nf][4] (host doubles), with tolerance tol >= 0. */
int ks_hull_set(ks_model *m, const double *facets, int32_t nf, double tol);

/* inside[i] = 1 when X[i] satisfies every facet, else 0 (uint8 array in the
 * same memory kind as X). */
int ks_hull_test(ks_model *m, const float *X, int32_t n, uint8_t *inside, int mem);

/* cbar(n0, chi) sqrt(sigma0) of Sec. 4.1 for each row (n0, chi, .) of X:
 * 2 n0 sqrt(sigma0) sqrt(psi(b*)), psi(b) = b (1 - b/n0)^2 (1 + chi b). */
int ks_cbar(ks_model *m, const float *X, int32_t n, double sigma0, float *out, int mem);

/* Threshold speed c*(n0, chi0) of travelling fronts of the scalar equation
 * of Sec. 4.1, b_t = sigma0 (D-tilde b_x)_x + g(b) (eqs. scalar-eq-b-re,
 * D-tilde, reac-term), for each row (n0, chi0, .) of X: the infimum of the
 * speeds c for which dz/db = -c - sigma0 D-tilde g / z has a solution z < 0 on
 * (0, n0) with z(0+) = z(n0-) = 0 (the appendix: sets defAchi0 / defA0; the
 * paper bounds c* by c-bar, see ks_cbar).  Computed on the device by shooting
 * from the sharp-front start at b = 0 with an L-stable two-step implicit
 * integrator (16384 steps) and a 65-way multisection over [0, 1.05 c-bar]
 * (5 rounds); relative accuracy about 1e-7.  NaN for n0 <= 0 or chi0 < 0. */
int ks_cstar(ks_model *m, const float *X, int32_t n, double sigma0, float *out, int mem);

void ks_destroy(ks_model *m);
const char *ks_last_error(const ks_model *m);

#ifdef __cplusplus
}
#endif

#endif /* KS_H */
