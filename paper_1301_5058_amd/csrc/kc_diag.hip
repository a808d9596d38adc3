// kc_diag.hip -- reductions over one field level, accumulated in double.
//
// diag_partial: block k reduces rows k, k + G, k + 2G, ...: sum b, sum n,
//   the largest squared distance from (cx, cy) of a cell with b >= b_thr
//   (-1 when none) and the number of such cells.  Wavefront butterfly (xor
//   shuffles) then a fixed LDS tree, so the result is the same bits on every
//   run for a given grid.
// diag_final:   one block folds the partials in a fixed order and writes
//   {t, h^2 sum b, h^2 sum n, h sqrt(max d^2), h sqrt(count / pi)}; it also
//   folds the per-strip partials that a fused step launch writes.
// check_partial: input validation of dense device arrays: per block, the
//   count of NaN / Inf / negative entries, the max of sigma n b and the max of
//   the donor-cell outflow rate (cell_rate; sigma taken as 1 when its pointer
//   is null, and scaled by sscale).
#include "kc_internal.h"

namespace kc {

static constexpr int kDiagBlocks = 1024;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Reduce per-thread values over a 256-thread block (sums s0, s1, s3 and the
// maximum m2); thread 0 gets them.
__device__ __forceinline__ void block_reduce4(double &s0, double &s1, double &m2, double &s3)
{
    __shared__ double sh[4][4];
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    m2 = wave_max(m2);
    s3 = wave_sum(s3);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        sh[0][w] = s0;
        sh[1][w] = s1;
        sh[2][w] = m2;
        sh[3][w] = s3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s0 = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        s1 = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
        m2 = fmax(fmax(sh[2][0], sh[2][1]), fmax(sh[2][2], sh[2][3]));
        s3 = (sh[3][0] + sh[3][1]) + (sh[3][2] + sh[3][3]);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void diag_partial(const R *b, const R *n, int nx, int ny,
                                                     int pitch, double b_thr, double cx, double cy,
                                                     double *parts)
{
    double sb = 0.0, sn = 0.0, m2 = -1.0, cnt = 0.0;
    for (int y = blockIdx.x; y < ny; y += gridDim.x) {
        const R *rb = b + (size_t)y * pitch;
        const R *rn = n + (size_t)y * pitch;
        const double dy = (double)y - cy;
        for (int x = threadIdx.x; x < nx; x += 256) {
            const double bv = (double)rb[x];
            sb += bv;
            sn += (double)rn[x];
            if (bv >= b_thr) {
                const double dx = (double)x - cx;
                m2 = fmax(m2, dx * dx + dy * dy);
                cnt += 1.0;
            }
        }
    }
    block_reduce4(sb, sn, m2, cnt);
    if (threadIdx.x == 0) {
        parts[4 * blockIdx.x + 0] = sb;
        parts[4 * blockIdx.x + 1] = sn;
        parts[4 * blockIdx.x + 2] = m2;
        parts[4 * blockIdx.x + 3] = cnt;
    }
}

__global__ __launch_bounds__(256) void diag_final(const double *parts, int nparts, double h,
                                                   double t, double *out5)
{
    double sb = 0.0, sn = 0.0, m2 = -1.0, cnt = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) {
        sb += parts[4 * i + 0];
        sn += parts[4 * i + 1];
        m2 = fmax(m2, parts[4 * i + 2]);
        cnt += parts[4 * i + 3];
    }
    block_reduce4(sb, sn, m2, cnt);
    if (threadIdx.x == 0) {
        out5[0] = t;
        out5[1] = h * h * sb;
        out5[2] = h * h * sn;
        out5[3] = m2 < 0.0 ? 0.0 : h * sqrt(m2);
        out5[4] = h * sqrt(cnt / 3.14159265358979323846);
    }
}

int diag_parts(int ny) { return ny < kDiagBlocks ? ny : kDiagBlocks; }

hipError_t launch_diag_fold(const double *parts, int nparts, double h, double t, double *out5,
                            hipStream_t s)
{
    hipLaunchKernelGGL(diag_final, dim3(1), dim3(256), 0, s, parts, nparts, h, t, out5);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_diag(const R *b, const R *n, int nx, int ny, int pitch, double h, double t,
                       double b_thr, double cx, double cy, double *parts, double *out5,
                       hipStream_t s)
{
    const int np = diag_parts(ny);
    hipLaunchKernelGGL((diag_partial<R>), dim3(np), dim3(256), 0, s, b, n, nx, ny, pitch, b_thr, cx,
                       cy, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(diag_final, dim3(1), dim3(256), 0, s, parts, np, h, t, out5);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Input validation
// ---------------------------------------------------------------------------
static constexpr int kCheckBlocks = 1024;

// Per-cell outflow rate of the donor-cell step (times h^2), the quantity whose
// product with dt / h^2 must stay <= 1 for b' >= 0:
//   sum over the existing neighbours Q of (D_P + D_Q) / 2
//   + chi sigma_P n_P b_P chihat(n_P) sum over Q with n_Q > n_P of (n_Q - n_P),
// D = sigma n b (eq. eqbadim; the chemotactic flux leaves P through every face
// toward higher nutrient with the donor coefficient X_P = sigma n b^2 chihat).
template <typename R>
__device__ __forceinline__ double cell_rate(const R *b, const R *n, const R *sg, int nx, int ny,
                                            int x, int y, double sscale, double chi, int law)
{
    const size_t i = (size_t)y * nx + x;
    const double sP = (sg ? (double)sg[i] : 1.0) * sscale;
    const double nP = (double)n[i], bP = (double)b[i];
    const double DP = sP * nP * bP;
    double dsum = 0.0, up = 0.0;
    const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int xq = x + dx[q], yq = y + dy[q];
        if (xq < 0 || xq >= nx || yq < 0 || yq >= ny)
            continue;
        const size_t j = (size_t)yq * nx + xq;
        const double nQ = (double)n[j];
        const double DQ = (sg ? (double)sg[j] : 1.0) * sscale * nQ * (double)b[j];
        dsum += 0.5 * (DP + DQ);
        if (nQ > nP)
            up += nQ - nP;
    }
    const double ch = law == 0 ? 1.0 / ((1.0 + nP) * (1.0 + nP)) : 1.0;
    return dsum + chi * DP * ch * up;
}

template <typename R>
__global__ __launch_bounds__(256) void check_partial(const R *b, const R *n, const R *sg, int nx,
                                                      int ny, double sscale, double chi, int law,
                                                      double *parts)
{
    double nbad = 0.0, mx = 0.0, rate = 0.0, unused = 0.0;
    const size_t cells = (size_t)nx * ny;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < cells; i += stride) {
        const R bv = b[i], nv = n[i], sv = sg ? sg[i] : R(1);
        const bool ok = (bv >= R(0)) && (nv >= R(0)) && (sv >= R(0)) && __builtin_isfinite(bv) &&
                        __builtin_isfinite(nv) && __builtin_isfinite(sv);
        if (!ok)
            nbad += 1.0;
        else
            mx = fmax(mx, (double)sv * sscale * (double)nv * (double)bv);
    }
    if (nbad == 0.0) // neighbours may be non-finite otherwise; the block reports them
        for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < cells; i += stride)
            rate = fmax(rate, cell_rate<R>(b, n, sg, nx, ny, (int)(i % nx), (int)(i / nx), sscale,
                                           chi, law));
    // block_reduce4 sums its first, second and fourth values and takes the max of
    // the third: the two maxima go through the max slot one after the other
    double m1 = mx;
    block_reduce4(nbad, unused, m1, unused);
    __syncthreads();
    double z0 = 0.0, z1 = 0.0, z3 = 0.0, m2 = rate;
    block_reduce4(z0, z1, m2, z3);
    if (threadIdx.x == 0) {
        parts[4 * blockIdx.x + 0] = nbad;
        parts[4 * blockIdx.x + 1] = m1;
        parts[4 * blockIdx.x + 2] = m2;
        parts[4 * blockIdx.x + 3] = 0.0;
    }
}

int check_parts(size_t cells)
{
    const size_t nb = (cells + 255) / 256;
    return nb < (size_t)kCheckBlocks ? (int)(nb ? nb : 1) : kCheckBlocks;
}

template <typename R>
hipError_t launch_check(const R *b, const R *n, const R *sg, int nx, int ny, double sscale,
                        double chi, int law, double *parts, hipStream_t s)
{
    const size_t cells = (size_t)nx * ny;
    hipLaunchKernelGGL((check_partial<R>), dim3(check_parts(cells)), dim3(256), 0, s, b, n, sg, nx,
                       ny, sscale, chi, law, parts);
    return hipGetLastError();
}

template hipError_t launch_diag<float>(const float *, const float *, int, int, int, double, double,
                                       double, double, double, double *, double *, hipStream_t);
template hipError_t launch_diag<double>(const double *, const double *, int, int, int, double,
                                        double, double, double, double, double *, double *,
                                        hipStream_t);
template hipError_t launch_check<float>(const float *, const float *, const float *, int, int,
                                        double, double, int, double *, hipStream_t);
template hipError_t launch_check<double>(const double *, const double *, const double *, int, int,
                                         double, double, int, double *, hipStream_t);

} // namespace kc
