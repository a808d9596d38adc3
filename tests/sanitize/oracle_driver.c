/* The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_sanitizers.py with gcc, no OpenMP): every entry point
 * on degenerate and ragged grids (1 x 1, single rows and columns, odd sizes),
 * so that a read or write outside a field, an uninitialised scratch cell or an
 * undefined integer operation aborts the run.  Checks only that the results
 * are finite and non-negative; the numbers themselves are pinned elsewhere. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_step(int nx, int ny, double h, double dt, double D_n, double theta, double kappa,
                 double chi, int chi_law, const double *b, const double *n, const double *sigma,
                 double *b_out, double *n_out);
int oracle_run(int nx, int ny, double h, double dt, double D_n, double theta, double kappa,
               double chi, int chi_law, double *b, double *n, const double *sigma, long nsteps);
int oracle_run_rk2(int nx, int ny, double h, double dt, double D_n, double theta, double kappa,
                   double chi, int chi_law, double *b, double *n, const double *sigma, long nsteps);
int oracle_run_noise(int nx, int ny, double h, double dt, double D_n, double theta, double kappa,
                     double chi, int chi_law, double *b, double *n, double sigma0, double amp,
                     uint64_t seed, int64_t step0, long nsteps, int integrator);
void oracle_diag(int nx, int ny, double h, const double *b, const double *n, double b_thr,
                 double cx, double cy, double *mass, double *nutrient, double *radius,
                 double *area_radius);
void oracle_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key, uint32_t *out);
double oracle_noise_delta(uint64_t seed, int64_t step, int i, int j);

static int bad = 0;

static void check(const char *what, int nx, int ny, const double *b, const double *n)
{
    for (long p = 0; p < (long)nx * ny; ++p)
        if (!isfinite(b[p]) || !isfinite(n[p]) || b[p] < 0.0 || n[p] < 0.0) {
            fprintf(stderr, "%s %dx%d: cell %ld b %g n %g\n", what, nx, ny, p, b[p], n[p]);
            ++bad;
            return;
        }
}

int main(void)
{
    static const int shapes[][2] = {{1, 1}, {1, 7}, {7, 1}, {5, 3}, {16, 16}, {3, 40}, {33, 2}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
        const int nx = shapes[s][0], ny = shapes[s][1];
        const size_t cells = (size_t)nx * ny;
        double *b = malloc(cells * sizeof(double)), *n = malloc(cells * sizeof(double));
        double *sg = malloc(cells * sizeof(double)), *b2 = malloc(cells * sizeof(double));
        double *n2 = malloc(cells * sizeof(double));
        for (int law = 0; law < 2; ++law) {
            for (size_t p = 0; p < cells; ++p) {
                b[p] = 0.3 + 0.2 * sin(0.7 * (double)p);
                n[p] = 0.6 + 0.1 * cos(1.3 * (double)p);
                sg[p] = 1.0 + 0.4 * sin(2.1 * (double)p);
            }
            oracle_step(nx, ny, 1.0, 0.05, 1.0, 1.0, 1.0, 1.5, law, b, n, sg, b2, n2);
            check("step", nx, ny, b2, n2);
            if (oracle_run(nx, ny, 1.0, 0.05, 1.0, 1.0, 1.0, 1.5, law, b, n, sg, 7) != 0)
                ++bad;
            check("run", nx, ny, b, n);
            if (oracle_run_rk2(nx, ny, 1.0, 0.05, 1.0, 1.0, 1.0, 1.5, law, b, n, sg, 5) != 0)
                ++bad;
            check("rk2", nx, ny, b, n);
            for (int integ = 0; integ < 2; ++integ) {
                if (oracle_run_noise(nx, ny, 0.5, 0.01, 1.0, 1.0, 1.0, 2.0, law, b, n, 1.0, 1.0,
                                     (uint64_t)0x9E3779B97F4A7C15ull, (int64_t)4294967290ll, 9,
                                     integ) != 0)
                    ++bad;
                check("noise", nx, ny, b, n);
            }
            double m, nu, r, ra;
            oracle_diag(nx, ny, 1.0, b, n, 0.3, -0.5, (ny - 1) / 2.0, &m, &nu, &r, &ra);
            if (!isfinite(m) || !isfinite(nu) || !(r >= 0.0) || !(ra >= 0.0))
                ++bad;
        }
        free(b);
        free(n);
        free(sg);
        free(b2);
        free(n2);
    }
    const uint32_t ctr[4] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu};
    const uint32_t key[2] = {0xffffffffu, 0xffffffffu};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    const double d = oracle_noise_delta(UINT64_MAX, INT64_MAX, 0x7fffffff, 0x7fffffff);
    if (!(d >= -1.0 && d <= 1.0))
        ++bad;
    printf("oracle driver: %d failures\n", bad);
    return bad ? 1 : 0;
}
