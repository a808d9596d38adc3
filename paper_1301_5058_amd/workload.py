"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module holds input recipes only -- none of the time step's arithmetic --
so that the library and the CPU oracle can be fed identical data without
sharing any code with each other.

Recipe (the paper's set-up, Sec. 3, with the readings listed below):
  * nutrient      n0 uniform over the grid (eq. inicond);
  * bacteria      a centred Gaussian inoculum b_max exp(-d^2 / r0^2), d the
                  distance in cells from ((nx-1)/2, (ny-1)/2) (the paper uses
                  b_M exp(-(x^2+y^2)/6.25), eq. inibacexp), set to zero beyond
                  cut * r0 so that no denormal tail is seeded;
  * agar field    sigma = sigma0 (1 + a U), U ~ Uniform[-1, 1] i.i.d. per cell
                  from numpy's default_rng(seed) (the paper perturbs sigma0 by a
                  random Delta, Sec. 3; here the field is static per run and
                  its amplitude a is a parameter);
  * time step     dt = 0.2 h^2 / max(D_n, max sigma n b), rounded to FP32 so that
                  single- and double-precision runs use the same number.
Fields are generated in FP64 and rounded to FP32; both sides use the rounded
values.
"""
import numpy as np


def fields(nx, ny, n0, a, seed, b_max=0.7, r0=6.0, cut=3.0, sigma0=1.0, chunk_rows=1024):
    """Return (b0, n0_field, sigma) as float32 arrays of shape [ny, nx].

    The inoculum is evaluated only on the square patch that holds its support,
    and sigma is drawn in row chunks (the same stream of doubles as one draw of
    shape [ny, nx]), so that grids of 16384^2 cells stay cheap in host memory.
    """
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    rc = cut * r0
    i0, i1 = max(0, int(np.floor(cx - rc))), min(nx, int(np.ceil(cx + rc)) + 1)
    j0, j1 = max(0, int(np.floor(cy - rc))), min(ny, int(np.ceil(cy + rc)) + 1)
    b = np.zeros((ny, nx), dtype=np.float32)
    if i1 > i0 and j1 > j0:
        j, i = np.meshgrid(np.arange(j0, j1, dtype=np.float64), np.arange(i0, i1, dtype=np.float64),
                           indexing="ij")
        d2 = (i - cx) ** 2 + (j - cy) ** 2
        patch = b_max * np.exp(-d2 / (r0 * r0))
        patch[d2 > rc * rc] = 0.0
        b[j0:j1, i0:i1] = patch.astype(np.float32)
    n = np.full((ny, nx), np.float32(n0), dtype=np.float32)
    s = np.empty((ny, nx), dtype=np.float32)
    rng = np.random.default_rng(seed)
    for r in range(0, ny, chunk_rows):
        rows = min(chunk_rows, ny - r)
        u = rng.uniform(-1.0, 1.0, (rows, nx))
        s[r:r + rows] = (sigma0 * (1.0 + a * u)).astype(np.float32)
    return b, n, s


def config_dt(b, n, sigma, h=1.0, D_n=1.0, factor=0.2):
    """dt = factor h^2 / max(D_n, max sigma n b) on the given fields, FP32-rounded."""
    b = np.asarray(b)
    nz = b > 0
    m = 0.0
    if nz.any():
        m = float(np.max(np.asarray(sigma)[nz].astype(np.float64) * np.asarray(n)[nz].astype(np.float64)
                         * b[nz].astype(np.float64)))
    return float(np.float32(factor * h * h / max(D_n, m)))


# The parameter sets of the workloads (normalised units, h = 1, D_n = theta = kappa = 1,
# receptor-law sensitivity, envelope threshold b_thr = 0.5 n0).
SMALL_128 = dict(nx=128, ny=128, n0=0.8, a=0.5, seed=0, chi=0.5, steps=2000)
SINGLE_4096 = dict(nx=4096, ny=4096, n0=0.5, a=0.5, seed=0, chi=1.0, steps=50000, warmup=1000)
HIRES_16384 = dict(nx=16384, ny=16384, n0=0.35, a=0.5, seed=0, chi=2.0, steps=20000)
CROP_512 = dict(nx=512, ny=512, n0=0.35, a=0.5, seed=0, chi=2.0, steps=20000)


def sweep(count=256, meta_seed=2026, sides=(256, 512, 1024, 2048)):
    """Instance list of a parameter sweep: side ~ U{sides}, n0 ~ U[0.3, 1.2],
    chi ~ U[0, 2], a ~ U[0.1, 0.5], sigma seed = instance index."""
    rng = np.random.default_rng(meta_seed)
    out = []
    for k in range(count):
        side = int(sides[rng.integers(0, len(sides))])
        n0 = float(rng.uniform(0.3, 1.2))
        chi = float(rng.uniform(0.0, 2.0))
        a = float(rng.uniform(0.1, 0.5))
        out.append(dict(nx=side, ny=side, n0=n0, chi=chi, a=a, seed=k))
    return out


# ---------------------------------------------------------------------------
# The one-dimensional front experiment (Sec. 4.2, system velo-system-1d):
# n_t = n_xx - n b,  b_t = (sigma0 n b b_x - chi0 sigma0 n b^2 n_x)_x + n b on
# [0, 20] with n(x, 0) = n0 and b(x, 0) = b_M exp(-x^2 / 6.25), b_M = 0.71,
# sigma0 = 1, for n0 in {0.35, 0.71, 1.07, 2, 3, 4} and chi0 in
# {0, 1, 2.5, 5, 10} (constant sensitivity).  Readings: cell-centred cells
# x_i = (i + 1/2) h on [0, length]; the inoculum is cut beyond 3 r0 (r0 = 2.5),
# as in two dimensions, because logistic growth of an uncut tail would reach
# the threshold ahead of the front; the front is the largest x with
# b >= min(0.5, n0 / 2) (Sec. 4.2 follows the point where b is about one half;
# n0 / 2 where the plateau n0 stays below it), and its speed is fitted over
# x in [9, 17], beyond the initial support.
# ---------------------------------------------------------------------------
FRONT1D = dict(length=20.0, cells=400, b_max=0.71, r0=2.5, cut=3.0, sigma0=1.0,
               n0=(0.35, 0.71, 1.07, 2.0, 3.0, 4.0), chi=(0.0, 1.0, 2.5, 5.0, 10.0),
               window=(9.0, 17.0), threshold=0.5)


def front1d_threshold(n0, level=0.5):
    """Front threshold of the 1-D experiment: `level`, or n0 / 2 when smaller."""
    return min(level, 0.5 * n0)


def front1d_fields(cells, length, n0, b_max=0.71, r0=2.5, cut=3.0, sigma0=1.0):
    """(b0, n0_field, sigma) float32 arrays of shape [1, cells] on [0, length]."""
    h = length / cells
    x = (np.arange(cells, dtype=np.float64) + 0.5) * h
    b = b_max * np.exp(-x * x / (r0 * r0))
    b[x > cut * r0] = 0.0
    n = np.full((1, cells), np.float32(n0), dtype=np.float32)
    s = np.full((1, cells), np.float32(sigma0), dtype=np.float32)
    return b.astype(np.float32)[None, :], n, s


def front1d_dt(cells, length, n0, chi=0.0, b_max=0.71, sigma0=1.0, D_n=1.0, factor=0.2):
    """dt = factor h^2 / max(D_n, sigma0 n0 (n0 + b_max) (1 + chi n0)), FP32-rounded.

    n stays <= n0 and b <= n0 + b_max, so sigma n b stays below
    sigma0 n0 (n0 + b_max) for the whole run (the initial fields alone would
    under-estimate it); the factor (1 + chi n0) covers the chemotactic outflow,
    chi sigma n b times nutrient differences of up to n0, which the positivity
    bound of the donor-cell step counts next to the diffusive outflow."""
    h = length / cells
    return float(np.float32(factor * h * h / max(D_n, sigma0 * n0 * (n0 + b_max) * (1.0 + chi * n0))))


# ---------------------------------------------------------------------------
# The paper's two-dimensional runs (Sec. 3, Table tabresparam): a square of
# side L = 680 with N = 2048 cells per side, inoculum b_M exp(-(x^2+y^2)/6.25)
# (b_M = 0.71) about the centre of the square, uniform nutrient n0, and
# sigma = sigma0 (1 + Delta) redrawn at every cell and step (noise amplitude
# 1), integrated with the two-stage Runge-Kutta method.  Each figure set
# compares two sensitivities chi0 at the four times of its captions.
# Readings: the inoculum's radius sqrt(6.25) = 2.5 is a physical length
# (2.5 / h cells) and is cut beyond 3 r0 as everywhere else; the Set 1 and
# Set 2 step is 0.02315, the one their captions' times and iteration counts
# imply (the text rounds it to 0.0231); the sigma0 = 4 sets quote 0.0110.
# ---------------------------------------------------------------------------
PAPER_2D = dict(length=680.0, cells=2048, b_max=0.71, r0=2.5, cut=3.0, amp=1.0)

PAPER_SETS = {
    "set1": dict(sigma0=1.0, n0=0.71, chi=(0.0, 5.0), times=(694.5, 1389.0, 2083.5, 2824.0),
                 dt=0.02315),
    "set2": dict(sigma0=1.0, n0=1.07, chi=(0.0, 5.0), times=(115.7, 231.5, 370.4, 509.3),
                 dt=0.02315),
    "set3a": dict(sigma0=4.0, n0=0.71, chi=(0.0, 2.5), times=(92.6, 162.0, 231.5, 324.0),
                  dt=0.0110),
    "set3b": dict(sigma0=4.0, n0=0.71, chi=(5.0, 7.5), times=(92.6, 162.0, 231.5, 324.0),
                  dt=0.0110),
    "set4": dict(sigma0=4.0, n0=1.07, chi=(0.0, 7.5), times=(33.0, 66.0, 88.0, 110.2),
                 dt=0.0110),
}


def paper_fields(cells, length, n0, b_max=0.71, r0=2.5, cut=3.0):
    """(b0, n0_field) float32 arrays of shape [cells, cells]: the inoculum of
    physical radius r0 (r0 / h cells, h = length / cells) about the centre."""
    h = length / cells
    b, n, _ = fields(cells, cells, n0, 0.0, 0, b_max=b_max, r0=r0 / h, cut=cut, chunk_rows=cells)
    return b, n


def paper_dt(cells, length, sigma0, n0, dt_paper, amp=1.0, b_max=0.71, D_n=1.0, margin=0.95):
    """The paper's step where it keeps the explicit bound, else `margin` times
    the bound; FP32-rounded.

    Bound: h^2 / (4 max(D_n, sigma0 (1 + amp) B^2)) with B = (n0 + b_max) / 2.
    sigma n b is largest where nutrient has turned into bacteria up to b = n
    (local kinetics keep b + n <= n0 + b_max, so n b <= B^2), and the noise
    draws sigma up to sigma0 (1 + amp).  The paper's 0.0110 at sigma0 = 4 and
    its 0.02315 at (sigma0, n0) = (1, 1.07) exceed this bound; the runs then
    take the smaller step and keep the captions' physical times."""
    h = length / cells
    B = 0.5 * (n0 + b_max)
    bound = h * h / (4.0 * max(D_n, sigma0 * (1.0 + amp) * B * B))
    return float(np.float32(min(dt_paper, margin * bound)))
