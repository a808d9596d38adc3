/*
 * kc_oracle.c -- plain FP64 CPU oracle for the explicit time step of the
 * normalised nutrient / bacteria chemotaxis system.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP library.
 *
 * What it computes (Leyva, Malaga, Plaza, arXiv:1301.5058):
 *
 *   n_t = D_n Lap(n) - kappa n b                                 (Sec. 2.4, eq. eqnadim;
 *                                                                 D_n, kappa from eq. nutriente-dim)
 *   b_t = div(sigma n b grad b) + theta kappa n b
 *         - chi div( sigma n b^2 chihat(n) grad n )              (Sec. 2.4, eq. eqbadim)
 *
 *   chihat(n) = 1/(1+n)^2   receptor law after normalisation     (Sec. 2.2 eq. receptor_law, Sec. 2.4)
 *   chihat(n) = 1           constant sensitivity                 (Sec. 4.1 eq. velo-system)
 *   no-flux boundaries                                            (Sec. 2.4 eq. bconds)
 *
 * The normalised system has D_n = theta = kappa = 1; they are kept as
 * parameters so that special cases (theta = 0: pure transport of b;
 * kappa = D_n = 0: frozen nutrient) can be exercised.
 *
 * Discretisation (the paper only says "explicit scheme and finite
 * differences", Sec. 3; the reading taken here):
 *   - nx * ny cell-centred finite volumes of width h, row-major, x fastest.
 *   - every boundary face carries zero flux (eq. bconds).
 *   - face diffusivity: arithmetic mean of the two cell values of
 *     D = sigma n b (eq. CoefCrsDif).
 *   - face chemotactic coefficient X = sigma n b^2 chihat(n) (eq. chemflux)
 *     taken from the donor cell: the bacteria move up the nutrient gradient,
 *     so across a face with n_Q > n_P the donor is P, otherwise Q.
 *   - forward Euler in time; every right-hand side uses the old level
 *     (oracle_step), or the two-stage Runge-Kutta step built from it
 *     (oracle_rk2_step).
 *
 * All arithmetic is IEEE double, written term by term in the order of the
 * equations above; the file is compiled without FMA contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define OR_CHI_RECEPTOR 0
#define OR_CHI_CONSTANT 1

/* chihat(n): the normalised sensitivity (receptor law with K_d = 1, or 1). */
static double chihat(double n, int chi_law)
{
    if (chi_law == OR_CHI_CONSTANT)
        return 1.0;
    return 1.0 / ((1.0 + n) * (1.0 + n));
}

/*
 * One forward-Euler step.  b, n, sigma: input level (nx*ny each).
 * b_out, n_out: new level (must not alias the inputs).
 */
void oracle_step(int nx, int ny, double h, double dt,
                 double D_n, double theta, double kappa, double chi, int chi_law,
                 const double *b, const double *n, const double *sigma,
                 double *b_out, double *n_out)
{
    const double lam = dt / (h * h);
    /* neighbour offsets: east, west, north (j+1), south (j-1) */
    const int di[4] = {+1, -1, 0, 0};
    const int dj[4] = {0, 0, +1, -1};

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            const long p = (long)j * nx + i;
            const double bP = b[p], nP = n[p], sP = sigma[p];
            /* eq. CoefCrsDif: D = sigma n b */
            const double DP = sP * nP * bP;
            /* eq. chemflux (normalised): X = sigma n b^2 chihat(n) */
            const double XP = sP * nP * bP * bP * chihat(nP, chi_law);

            double Fb = 0.0; /* sum over faces of (flux into P) * h^2 for b */
            double Fn = 0.0; /* same for the nutrient Laplacian          */
            for (int k = 0; k < 4; ++k) {
                const int qi = i + di[k], qj = j + dj[k];
                if (qi < 0 || qi >= nx || qj < 0 || qj >= ny)
                    continue; /* boundary face: no flux (eq. bconds) */
                const long q = (long)qj * nx + qi;
                const double bQ = b[q], nQ = n[q], sQ = sigma[q];
                const double DQ = sQ * nQ * bQ;
                const double XQ = sQ * nQ * bQ * bQ * chihat(nQ, chi_law);
                /* donor cell for the chemotactic flux */
                const double Xup = (nQ > nP) ? XP : XQ;
                const double Dface = 0.5 * (DP + DQ);
                Fb += Dface * (bQ - bP) - chi * Xup * (nQ - nP);
                Fn += nQ - nP;
            }
            /* linear kinetics f = kappa n b (eq. goodkinetics) */
            const double r = kappa * nP * bP;
            b_out[p] = bP + lam * Fb + dt * theta * r;
            n_out[p] = nP + lam * D_n * Fn - dt * r;
        }
    }
}

/*
 * nsteps forward-Euler steps in place on (b, n).  Returns 0, or -5 when the
 * scratch level cannot be allocated.
 */
int oracle_run(int nx, int ny, double h, double dt,
               double D_n, double theta, double kappa, double chi, int chi_law,
               double *b, double *n, const double *sigma, long nsteps)
{
    const size_t cells = (size_t)nx * (size_t)ny;
    double *b2 = (double *)malloc(cells * sizeof(double));
    double *n2 = (double *)malloc(cells * sizeof(double));
    if (!b2 || !n2) {
        free(b2);
        free(n2);
        return -5;
    }
    double *bc = b, *nc = n, *bn = b2, *nn = n2;
    for (long s = 0; s < nsteps; ++s) {
        oracle_step(nx, ny, h, dt, D_n, theta, kappa, chi, chi_law, bc, nc, sigma, bn, nn);
        double *t;
        t = bc; bc = bn; bn = t;
        t = nc; nc = nn; nn = t;
    }
    if (bc != b) {
        for (size_t p = 0; p < cells; ++p) {
            b[p] = bc[p];
            n[p] = nc[p];
        }
    }
    free(b2);
    free(n2);
    return 0;
}

/*
 * One step of the explicit two-stage Runge-Kutta method.  The paper
 * integrates in time with an explicit second-order Runge-Kutta scheme
 * (Sec. 3) without naming it; the reading taken is Heun's method in its
 * strong-stability-preserving form: with E the forward-Euler step above,
 *
 *   u1 = E(u),   u2 = E(u1),   u' = (u + u2) / 2,
 *
 * i.e. the average of u and two chained Euler steps (algebraically the usual
 * u' = u + dt/2 (L(u) + L(u1))).  Every stage is an Euler step and u' a
 * convex combination, so b >= 0 and the stability bound of E carry over.
 * b1, n1, b2, n2: scratch levels (nx*ny each, not aliasing anything else).
 */
void oracle_rk2_step(int nx, int ny, double h, double dt,
                     double D_n, double theta, double kappa, double chi, int chi_law,
                     const double *b, const double *n, const double *sigma,
                     double *b1, double *n1, double *b2, double *n2,
                     double *b_out, double *n_out)
{
    oracle_step(nx, ny, h, dt, D_n, theta, kappa, chi, chi_law, b, n, sigma, b1, n1);
    oracle_step(nx, ny, h, dt, D_n, theta, kappa, chi, chi_law, b1, n1, sigma, b2, n2);
    const long cells = (long)nx * ny;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < cells; ++p) {
        b_out[p] = 0.5 * (b[p] + b2[p]);
        n_out[p] = 0.5 * (n[p] + n2[p]);
    }
}

/*
 * nsteps steps of oracle_rk2_step in place on (b, n).  Returns 0, or -5 when
 * the scratch levels cannot be allocated.
 */
int oracle_run_rk2(int nx, int ny, double h, double dt,
                   double D_n, double theta, double kappa, double chi, int chi_law,
                   double *b, double *n, const double *sigma, long nsteps)
{
    const size_t cells = (size_t)nx * (size_t)ny;
    double *buf = (double *)malloc(6 * cells * sizeof(double));
    if (!buf)
        return -5;
    double *b1 = buf, *n1 = buf + cells, *b2 = buf + 2 * cells, *n2 = buf + 3 * cells;
    double *bn = buf + 4 * cells, *nn = buf + 5 * cells;
    for (long s = 0; s < nsteps; ++s) {
        oracle_rk2_step(nx, ny, h, dt, D_n, theta, kappa, chi, chi_law, b, n, sigma,
                        b1, n1, b2, n2, bn, nn);
        for (size_t p = 0; p < cells; ++p) {
            b[p] = bn[p];
            n[p] = nn[p];
        }
    }
    free(buf);
    return 0;
}

/*
 * Per-step agar noise.  The paper perturbs the agar hardness at every point
 * and every time step, sigma = sigma0 (1 + Delta) with Delta triangular on
 * [-1, 1] (Sec. 3).  Reading: sigma = sigma0 (1 + a Delta), Delta = U1 + U2 - 1
 * with U1, U2 uniform, drawn from the counter-based generator Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC 2011): counter (i / 4, j, step low word, step high word), key (seed low
 * word, seed high word); cell i takes output word i mod 4, whose two 16-bit
 * halves k1, k2 give Delta = (k1 + k2) 2^-16 - 1 exactly (one generator call
 * serves four neighbouring cells).
 */
static void philox4x32_10(uint32_t ctr[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { /* key schedule: Weyl increments */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * ctr[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t x0 = hi1 ^ ctr[1] ^ k0, x2 = hi0 ^ ctr[3] ^ k1;
        ctr[0] = x0;
        ctr[1] = lo1;
        ctr[2] = x2;
        ctr[3] = lo0;
    }
}

/* The raw generator, for its known-answer tests. */
void oracle_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key, uint32_t *out)
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    philox4x32_10(c, key[0], key[1]);
    for (int i = 0; i < 4; ++i)
        out[i] = c[i];
}

/* Delta of cell (i, j) at time step `step` (see above). */
double oracle_noise_delta(uint64_t seed, int64_t step, int i, int j)
{
    uint32_t c[4] = {(uint32_t)i >> 2, (uint32_t)j, (uint32_t)((uint64_t)step & 0xffffffffu),
                     (uint32_t)((uint64_t)step >> 32)};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const uint32_t w = c[i & 3];
    const double u = (double)((w & 0xffffu) + (w >> 16)); /* integer < 2^17 */
    return u * (1.0 / 65536.0) - 1.0;                     /* 2^-16 */
}

/* sigma of every cell at time step `step`. */
static void noise_sigma(int nx, int ny, double sigma0, double amp, uint64_t seed, int64_t step,
                        double *sg)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            sg[(long)j * nx + i] = sigma0 * (1.0 + amp * oracle_noise_delta(seed, step, i, j));
}

/*
 * nsteps steps with a fresh agar field at every step (steps step0,
 * step0 + 1, ...): forward Euler (integrator 0) or the two-stage Runge-Kutta
 * step (1), whose two stages share the step's field.  Returns 0, or -5.
 */
int oracle_run_noise(int nx, int ny, double h, double dt,
                     double D_n, double theta, double kappa, double chi, int chi_law,
                     double *b, double *n, double sigma0, double amp, uint64_t seed,
                     int64_t step0, long nsteps, int integrator)
{
    const size_t cells = (size_t)nx * (size_t)ny;
    double *buf = (double *)malloc(7 * cells * sizeof(double));
    if (!buf)
        return -5;
    double *sg = buf, *b1 = buf + cells, *n1 = buf + 2 * cells, *b2 = buf + 3 * cells;
    double *n2 = buf + 4 * cells, *bn = buf + 5 * cells, *nn = buf + 6 * cells;
    for (long s = 0; s < nsteps; ++s) {
        noise_sigma(nx, ny, sigma0, amp, seed, step0 + s, sg);
        if (integrator == 0)
            oracle_step(nx, ny, h, dt, D_n, theta, kappa, chi, chi_law, b, n, sg, bn, nn);
        else
            oracle_rk2_step(nx, ny, h, dt, D_n, theta, kappa, chi, chi_law, b, n, sg, b1, n1,
                            b2, n2, bn, nn);
        for (size_t p = 0; p < cells; ++p) {
            b[p] = bn[p];
            n[p] = nn[p];
        }
    }
    free(buf);
    return 0;
}

/*
 * Diagnostics of one level:
 *   mass     = h^2 * sum b     (summed in row order)
 *   nutrient = h^2 * sum n
 *   radius   = h * max over cells with b >= b_thr of the distance of the
 *              cell index (i, j) from (cx, cy); 0 when no cell qualifies.
 *   area_radius = h * sqrt(count of cells with b >= b_thr / pi): the radius
 *              of the disc with the colony's area.
 * The paper tracks the front of b near a fixed level (Sec. 4.2); both radii
 * carry that idea to a two-dimensional colony.
 */
void oracle_diag(int nx, int ny, double h, const double *b, const double *n,
                 double b_thr, double cx, double cy,
                 double *mass, double *nutrient, double *radius, double *area_radius)
{
    double sb = 0.0, sn = 0.0, rmax = 0.0, count = 0.0;
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            const long p = (long)j * nx + i;
            sb += b[p];
            sn += n[p];
            if (b[p] >= b_thr) {
                count += 1.0;
                const double dx = (double)i - cx, dy = (double)j - cy;
                const double d = sqrt(dx * dx + dy * dy);
                if (d > rmax)
                    rmax = d;
            }
        }
    }
    *mass = h * h * sb;
    *nutrient = h * h * sn;
    *radius = h * rmax;
    *area_radius = h * sqrt(count / 3.14159265358979323846);
}

/* Threads for the following calls (n >= 1; no effect without OpenMP).  Only the
 * timing of the oracle depends on it: every cell is computed the same way. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads oracle_step runs with (1 without OpenMP). */
int oracle_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
