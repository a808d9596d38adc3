// kc_step.hip -- explicit time-step kernels for gfx950.
//
// step_ref     one step per launch, one thread per cell, neighbours read from
//              global memory.  The plain form of the stencil; every other
//              kernel must reproduce its bits.
// step_stream  T steps per launch ("temporal blocking").  One 64-lane
//              wavefront owns a strip of 64*VEC columns (VEC adjacent cells
//              per lane, loaded as one 16-byte vector) and walks it downwards
//              row by row.  Level s (1..T) of the time block trails level s-1
//              by one row, so the three rows a level needs sit in registers;
//              the horizontal neighbour across a lane boundary comes from the
//              adjacent lane through a DPP wave shift.  Each level loses one
//              valid column at either strip edge, so strips overlap by HX >= T
//              columns (a multiple of VEC) and by T rows above and below.  Rows
//              are prefetched PF rows ahead into a register ring.  HBM traffic
//              per launch: read b, n, sigma once, write b', n' once (plus the
//              halo re-reads, which mostly hit L2).
#include "kc_internal.h"

namespace kc {

template <typename R> struct StepArgs {
    const R *b_in, *n_in, *sg;
    R *b_out, *n_out;
    int nx, ny, pitch;
    int rows;           // output rows per strip
    int nsx, nstrips;   // strips along x, total strips
    int nblocks_padded; // grid size (multiple of 8)
    Coef<R> c;
};

// ---------------------------------------------------------------------------
// Reference kernel
// ---------------------------------------------------------------------------
template <typename R, int LAW>
__device__ __forceinline__ void ref_cell(const StepArgs<R> &a, int x, int y, R &b, R &n, R &D, R &X)
{
    if (x < 0 || x >= a.nx || y < 0 || y >= a.ny) {
        b = n = D = X = R(0);
        return;
    }
    const size_t p = (size_t)y * a.pitch + x;
    b = a.b_in[p];
    n = a.n_in[p];
    const R sh = R(0.5) * a.sg[p];
    coef<R, LAW>(sh, n, b, a.c.chi2, D, X);
}

template <typename R, int LAW>
__global__ __launch_bounds__(256) void step_ref(StepArgs<R> a)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.nx || y >= a.ny)
        return;
    R bP, nP, DP, XP, bE, nE, DE, XE, bW, nW, DW, XW, bN, nN, DN, XN, bS, nS, DS, XS;
    ref_cell<R, LAW>(a, x, y, bP, nP, DP, XP);
    ref_cell<R, LAW>(a, x + 1, y, bE, nE, DE, XE);
    ref_cell<R, LAW>(a, x - 1, y, bW, nW, DW, XW);
    ref_cell<R, LAW>(a, x, y + 1, bN, nN, DN, XN);
    ref_cell<R, LAW>(a, x, y - 1, bS, nS, DS, XS);
    R geb, gen, gwb, gwn, gnb, gnn, gsb, gsn;
    face<R>(bP, nP, DP, XP, bE, nE, DE, XE, x + 1 < a.nx, geb, gen);
    face<R>(bW, nW, DW, XW, bP, nP, DP, XP, x - 1 >= 0, gwb, gwn);
    face<R>(bP, nP, DP, XP, bN, nN, DN, XN, y + 1 < a.ny, gnb, gnn);
    face<R>(bS, nS, DS, XS, bP, nP, DP, XP, y - 1 >= 0, gsb, gsn);
    const R Fb = net<R>(geb, gwb, gnb, gsb);
    const R Fn = net<R>(gen, gwn, gnn, gsn);
    R bo, no;
    update<R>(bP, nP, Fb, Fn, a.c, bo, no);
    const size_t p = (size_t)y * a.pitch + x;
    a.b_out[p] = bo;
    a.n_out[p] = no;
}

// ---------------------------------------------------------------------------
// Fused register-streaming kernel
// ---------------------------------------------------------------------------
template <typename R, int VEC> struct VecT;
template <> struct VecT<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct VecT<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };

template <typename R> struct StreamShape;
template <> struct StreamShape<float> { static constexpr int VEC = 4; };
template <> struct StreamShape<double> { static constexpr int VEC = 2; };

template <int T, int VEC> struct Halo {
    static constexpr int HX = (T + VEC - 1) / VEC * VEC; // halo columns per side
    static constexpr int WC = 64 * VEC;                  // columns per wavefront
    static constexpr int OW = WC - 2 * HX;               // output columns per strip
};

template <typename R, int T, int LAW, int PF>
__global__ __launch_bounds__(256) void step_stream(StepArgs<R> a)
{
    constexpr int VEC = StreamShape<R>::VEC;
    constexpr int HX = Halo<T, VEC>::HX;
    constexpr int WC = Halo<T, VEC>::WC;
    constexpr int OW = Halo<T, VEC>::OW;
    typedef typename VecT<R, VEC>::type vec_t;

    const int lb = xcd_block(a.nblocks_padded);
    const int strip = lb * 4 + (int)(threadIdx.x >> 6);
    if (strip >= a.nstrips)
        return; // whole wavefront leaves together
    const int lane = threadIdx.x & 63;
    const int sx = strip % a.nsx, sy = strip / a.nsx;
    const int x0 = sx * OW - HX + lane * VEC; // first column of this lane
    const int y0 = sy * a.rows;
    const int y1 = min(y0 + a.rows, a.ny);
    const int rs = max(y0 - T, 0); // first input row
    const int re = y1 + T;         // one past the last input row needed
    const bool lane_in = (x0 >= 0) && (x0 < a.pitch);
    const bool lane_out = (lane * VEC >= HX) && (lane * VEC < WC - HX) && (x0 < a.nx);
    bool ve[VEC]; // east face of cell k is interior
#pragma unroll
    for (int k = 0; k < VEC; ++k)
        ve[k] = (x0 + k >= 0) && (x0 + k + 1 < a.nx);

    // level state: centre row of level L (= time level L within the block) and
    // the face flux G(S,P) below it
    R cb[T][VEC], cn[T][VEC], cD[T][VEC], cX[T][VEC], cs[T][VEC], fb[T][VEC], fn[T][VEC];
#pragma unroll
    for (int L = 0; L < T; ++L)
#pragma unroll
        for (int k = 0; k < VEC; ++k)
            cb[L][k] = cn[L][k] = cD[L][k] = cX[L][k] = cs[L][k] = fb[L][k] = fn[L][k] = R(0);

    // prefetch ring: slot (row - rs) % PF
    vec_t pb[PF], pn[PF], ps[PF];
    const vec_t zero = (vec_t)(R(0));
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int row = rs + u;
        if (row < a.ny && lane_in) {
            const size_t p = (size_t)row * a.pitch + x0;
            pb[u] = *reinterpret_cast<const vec_t *>(a.b_in + p);
            pn[u] = *reinterpret_cast<const vec_t *>(a.n_in + p);
            ps[u] = *reinterpret_cast<const vec_t *>(a.sg + p);
        } else {
            pb[u] = pn[u] = ps[u] = zero;
        }
    }

    for (int r0 = rs; r0 < re; r0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int row = r0 + u;
            // consume slot u (row), refill it with row + PF
            R ib[VEC], in[VEC], iD[VEC], iX[VEC], is[VEC];
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                ib[k] = pb[u][k];
                in[k] = pn[u][k];
                is[k] = R(0.5) * ps[u][k];
            }
            {
                const int nrow = row + PF;
                if (nrow < re && nrow < a.ny && lane_in) {
                    const size_t p = (size_t)nrow * a.pitch + x0;
                    pb[u] = *reinterpret_cast<const vec_t *>(a.b_in + p);
                    pn[u] = *reinterpret_cast<const vec_t *>(a.n_in + p);
                    ps[u] = *reinterpret_cast<const vec_t *>(a.sg + p);
                } else {
                    pb[u] = pn[u] = ps[u] = zero;
                }
            }
#pragma unroll
            for (int k = 0; k < VEC; ++k)
                coef<R, LAW>(is[k], in[k], ib[k], a.c.chi2, iD[k], iX[k]);

#pragma unroll
            for (int L = 0; L < T; ++L) {
                const int y = row - L - 1; // centre row of this level
                const bool vv = (y >= 0) && (y + 1 < a.ny);
                R gvb[VEC], gvn[VEC], geb[VEC], gen[VEC];
#pragma unroll
                for (int k = 0; k < VEC; ++k)
                    face<R>(cb[L][k], cn[L][k], cD[L][k], cX[L][k], ib[k], in[k], iD[k], iX[k], vv,
                            gvb[k], gvn[k]);
#pragma unroll
                for (int k = 0; k + 1 < VEC; ++k)
                    face<R>(cb[L][k], cn[L][k], cD[L][k], cX[L][k], cb[L][k + 1], cn[L][k + 1],
                            cD[L][k + 1], cX[L][k + 1], ve[k], geb[k], gen[k]);
                {
                    const R eb = from_next(cb[L][0]), en = from_next(cn[L][0]);
                    const R eD = from_next(cD[L][0]), eX = from_next(cX[L][0]);
                    face<R>(cb[L][VEC - 1], cn[L][VEC - 1], cD[L][VEC - 1], cX[L][VEC - 1], eb, en,
                            eD, eX, ve[VEC - 1], geb[VEC - 1], gen[VEC - 1]);
                }
                const R wb = from_prev(geb[VEC - 1]), wn = from_prev(gen[VEC - 1]);
                R ob[VEC], on[VEC], os[VEC];
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    const R Fb = net<R>(geb[k], k ? geb[k - 1] : wb, gvb[k], fb[L][k]);
                    const R Fn = net<R>(gen[k], k ? gen[k - 1] : wn, gvn[k], fn[L][k]);
                    update<R>(cb[L][k], cn[L][k], Fb, Fn, a.c, ob[k], on[k]);
                    os[k] = cs[L][k];
                }
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    fb[L][k] = gvb[k];
                    fn[L][k] = gvn[k];
                    cb[L][k] = ib[k];
                    cn[L][k] = in[k];
                    cD[L][k] = iD[k];
                    cX[L][k] = iX[k];
                    cs[L][k] = is[k];
                }
                if (L + 1 < T) {
#pragma unroll
                    for (int k = 0; k < VEC; ++k) {
                        ib[k] = ob[k];
                        in[k] = on[k];
                        is[k] = os[k];
                        coef<R, LAW>(is[k], in[k], ib[k], a.c.chi2, iD[k], iX[k]);
                    }
                } else if (y >= y0 && y < y1 && lane_out) {
                    vec_t vb, vn;
#pragma unroll
                    for (int k = 0; k < VEC; ++k) {
                        vb[k] = ob[k];
                        vn[k] = on[k];
                    }
                    const size_t p = (size_t)y * a.pitch + x0;
                    *reinterpret_cast<vec_t *>(a.b_out + p) = vb;
                    *reinterpret_cast<vec_t *>(a.n_out + p) = vn;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static const int kDepths[] = {1, 2, 3, 4, 6, 8};

int stream_depth_at_most(int t)
{
    int best = 1;
    for (int d : kDepths)
        if (d <= t)
            best = d;
    return best;
}

StreamGeom stream_geom(int precision, int tsteps, int nx, int ny, int rows)
{
    const int vec = precision == 0 ? 4 : 2;
    const int hx = (tsteps + vec - 1) / vec * vec;
    StreamGeom g;
    g.out_cols = 64 * vec - 2 * hx;
    g.nsx = (nx + g.out_cols - 1) / g.out_cols;
    g.nsy = (ny + rows - 1) / rows;
    g.nstrips = g.nsx * g.nsy;
    const int nblocks = (g.nstrips + 3) / 4;
    g.nblocks_padded = (nblocks + 7) / 8 * 8;
    return g;
}

template <typename R>
static StepArgs<R> make_args(const Fields<R> &f, const Coef<R> &c)
{
    StepArgs<R> a;
    a.b_in = f.b_in;
    a.n_in = f.n_in;
    a.sg = f.sg;
    a.b_out = f.b_out;
    a.n_out = f.n_out;
    a.nx = f.nx;
    a.ny = f.ny;
    a.pitch = f.pitch;
    a.rows = 1;
    a.nsx = a.nstrips = a.nblocks_padded = 0;
    a.c = c;
    return a;
}

template <typename R, int T, int LAW>
static hipError_t launch_stream_pf(const StepArgs<R> &a, int pf, dim3 grid, hipStream_t s)
{
    if (pf == 4)
        hipLaunchKernelGGL((step_stream<R, T, LAW, 4>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((step_stream<R, T, LAW, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename R, int LAW>
static hipError_t launch_stream_t(const StepArgs<R> &a, int T, int pf, dim3 grid, hipStream_t s)
{
    switch (T) {
    case 1: return launch_stream_pf<R, 1, LAW>(a, pf, grid, s);
    case 2: return launch_stream_pf<R, 2, LAW>(a, pf, grid, s);
    case 3: return launch_stream_pf<R, 3, LAW>(a, pf, grid, s);
    case 4: return launch_stream_pf<R, 4, LAW>(a, pf, grid, s);
    case 6: return launch_stream_pf<R, 6, LAW>(a, pf, grid, s);
    case 8: return launch_stream_pf<R, 8, LAW>(a, pf, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_stream(const Fields<R> &f, const Coef<R> &c, int chi_law, const Tuning &t,
                         hipStream_t s)
{
    StepArgs<R> a = make_args(f, c);
    const StreamGeom g = stream_geom(sizeof(R) == 4 ? 0 : 1, t.tsteps, f.nx, f.ny, t.rows);
    a.rows = t.rows;
    a.nsx = g.nsx;
    a.nstrips = g.nstrips;
    a.nblocks_padded = g.nblocks_padded;
    const dim3 grid(g.nblocks_padded);
    if (chi_law == 0)
        return launch_stream_t<R, 0>(a, t.tsteps, t.prefetch, grid, s);
    return launch_stream_t<R, 1>(a, t.tsteps, t.prefetch, grid, s);
}

template <typename R>
hipError_t launch_ref(const Fields<R> &f, const Coef<R> &c, int chi_law, hipStream_t s)
{
    const StepArgs<R> a = make_args(f, c);
    const dim3 grid((f.nx + 63) / 64, (f.ny + 3) / 4);
    if (chi_law == 0)
        hipLaunchKernelGGL((step_ref<R, 0>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((step_ref<R, 1>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_stream<float>(const Fields<float> &, const Coef<float> &, int,
                                         const Tuning &, hipStream_t);
template hipError_t launch_stream<double>(const Fields<double> &, const Coef<double> &, int,
                                          const Tuning &, hipStream_t);
template hipError_t launch_ref<float>(const Fields<float> &, const Coef<float> &, int, hipStream_t);
template hipError_t launch_ref<double>(const Fields<double> &, const Coef<double> &, int,
                                       hipStream_t);

} // namespace kc
