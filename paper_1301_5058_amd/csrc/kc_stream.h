// kc_stream.h -- one wavefront advancing one strip of the grid by T steps.
//
// A 64-lane wavefront owns a strip of 64*VEC columns (VEC adjacent cells per
// lane, loaded as one 16-byte vector) and walks it downwards row by row.
// Level s (1..T) of the time block trails level s-1 by one row, so the three
// rows a level needs are held in registers; the horizontal neighbour across a
// lane boundary comes from the adjacent lane through a DPP wave shift.  Each
// level loses one valid column at either strip edge, so strips overlap by
// HX >= T columns (a multiple of VEC) and by T rows above and below.  Input
// rows are prefetched PF rows ahead into a register ring.  HBM traffic per
// launch: read b, n, sigma once, write b', n' once, plus halo re-reads that
// mostly hit L2.
//
// With NOISE the agar field is redrawn at every time step (noise_half_sigma,
// kc_device.h): each level computes sigma of its incoming row for the step it
// advances instead of loading it (the two Runge-Kutta levels of a step share
// the step's field, passed along as before).
//
// With RK, each time step is two levels of the two-stage Runge-Kutta method
// u' = (u + E(E(u))) / 2 (E = one forward-Euler step): an even level hands the
// u of its centre row to the next level together with its Euler output, and
// the odd level averages that u with its own Euler output.  A block of T
// levels then advances T / 2 steps.
//
// Level L (0-based) computes only the centre rows [y0 - T + L, y1 + T - 1 - L):
// the rows that the T-th level's output rows [y0, y1) depend on, plus one lead-in
// row whose only purpose is the face flux below the first needed row.  The test
// is wave-uniform, so skipped rows cost a scalar branch, and a group of PF rows
// on which every level is active (the steady state between the first T - 1 + T
// and the last rows) runs a straight-line body without it.  A strip whose halo
// window lies strictly inside the domain (CHECK = false) needs no boundary-face
// masks and no load predicates; edge strips run the checked code.
//
// strip_diag reads back the cells a strip has just stored (each lane its own
// addresses, so program order makes the stores visible) and folds them into a
// per-lane accumulator: sum b, sum n in double, the largest squared distance
// from the envelope centre of a cell with b >= b_thr, and the count of such
// cells, rows ascending and columns ascending within a lane.
#pragma once

#include "kc_device.h"

namespace kc {

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

template <typename R> struct StripArgs {
    const R *b_in, *n_in, *sg;
    R *b_out, *n_out;
    int nx, ny, pitch;
    int rows; // output rows per strip
    Coef<R> c;
    Noise<R> z;           // per-step agar noise (NOISE only; sg unused then)
    double b_thr, cx, cy; // envelope diagnostics (strip_diag only)
};

template <bool B> struct BoolTag {
    static constexpr bool value = B;
};

struct DiagAcc {
    double sb, sn, m2, cnt;
};

// True when every face and load of strip (sx, sy) lies inside the domain.
template <typename R, int T>
__device__ __forceinline__ bool strip_interior(const StripArgs<R> &a, int sx, int sy)
{
    constexpr int VEC = StreamShape<R>::VEC;
    constexpr int HX = Halo<T, VEC>::HX;
    constexpr int OW = Halo<T, VEC>::OW;
    constexpr int WC = Halo<T, VEC>::WC;
    const int xl = sx * OW - HX;
    const int y0 = sy * a.rows, y1 = min(y0 + a.rows, a.ny);
    return xl >= 0 && xl + WC <= a.nx - 1 && y0 >= T && y1 + T <= a.ny;
}

template <typename R, int T, int LAW, int PF, bool CHECK, bool RK = false, bool NOISE = false>
__device__ __forceinline__ void stream_strip(const StripArgs<R> &a, int sx, int sy)
{
    static_assert(!RK || T % 2 == 0, "a two-stage Runge-Kutta block has an even level count");
    constexpr int VEC = StreamShape<R>::VEC;
    constexpr int HX = Halo<T, VEC>::HX;
    constexpr int WC = Halo<T, VEC>::WC;
    constexpr int OW = Halo<T, VEC>::OW;
    typedef typename VecT<R, VEC>::type vec_t;

    const int lane = threadIdx.x & 63;
    const int x0 = sx * OW - HX + lane * VEC; // first column of this lane
    const int y0 = sy * a.rows;
    const int y1 = min(y0 + a.rows, a.ny);
    const int rs = max(y0 - T, 0); // first input row
    const int re = y1 + T;         // one past the last input row needed
    const bool lane_out = (lane * VEC >= HX) && (lane * VEC < WC - HX) && (x0 < a.nx);
    bool ve[VEC]; // east face of cell k is interior
#pragma unroll
    for (int k = 0; k < VEC; ++k)
        ve[k] = !CHECK || ((x0 + k >= 0) && (x0 + k + 1 < a.nx));

    // level state: centre row of level L and the face inflow G(S,P) below it;
    // with RK, the second level of each step also holds the step's input u of
    // its centre row (cub, cun)
    R cb[T][VEC], cn[T][VEC], cD[T][VEC], cX[T][VEC], cs[T][VEC], fb[T][VEC], fn[T][VEC];
    R cub[T][VEC], cun[T][VEC];
#pragma unroll
    for (int L = 0; L < T; ++L)
#pragma unroll
        for (int k = 0; k < VEC; ++k)
            cb[L][k] = cn[L][k] = cD[L][k] = cX[L][k] = cs[L][k] = fb[L][k] = fn[L][k] =
                cub[L][k] = cun[L][k] = R(0);

    // Prefetch ring: slot (row - rs) % PF.  Loads are unconditional, from
    // addresses clamped into the array: a row past the last input row or a
    // column outside [0, pitch) yields some in-bounds value that only ever
    // meets a zero (masked) face or a skipped level, never a stored cell.
    // (A conditional load would make the compiler merge the two arms through
    // a register copy, which waits for the load it was meant to hide.)
    vec_t pb[PF], pn[PF], ps[PF];
    const int last_row = min(re, a.ny) - 1;
    const int xc = min(max(x0, 0), a.pitch - VEC);
    auto load_row = [&](int row, vec_t &vb, vec_t &vn, vec_t &vs) __attribute__((always_inline)) {
        const size_t p = (size_t)min(row, last_row) * a.pitch + xc;
        vb = *reinterpret_cast<const vec_t *>(a.b_in + p);
        vn = *reinterpret_cast<const vec_t *>(a.n_in + p);
        if constexpr (!NOISE)
            vs = *reinterpret_cast<const vec_t *>(a.sg + p);
        else
            vs = vec_t{};
    };
    // time step (after the launch's first) that level L advances
    auto level_step = [](int L) { return RK ? L / 2 : L; };
#pragma unroll
    for (int u = 0; u < PF; ++u)
        load_row(rs + u, pb[u], pn[u], ps[u]);

    // One group of PF rows.  With FULL every level is active on every row of
    // the group (the steady state), so the body is one straight-line block.
    auto group = [&](int r0, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int row = r0 + u;
            // consume slot u (row), refill it with row + PF
            R ib[VEC], in[VEC], iD[VEC], iX[VEC], is[VEC];
            R iub[VEC], iun[VEC]; // RK: u of the incoming row of an odd level
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                ib[k] = pb[u][k];
                in[k] = pn[u][k];
                is[k] = R(0.5) * ps[u][k];
                iub[k] = iun[k] = R(0);
            }
            if (NOISE) // sigma of the incoming row at the first level's step
                noise_half_sigma<R, VEC>(a.z, level_step(0), x0, row, is);
            load_row(row + PF, pb[u], pn[u], ps[u]);
#pragma unroll
            for (int k = 0; k < VEC; ++k)
                coef<R, LAW>(is[k], in[k], ib[k], a.c.chi2, iD[k], iX[k]);

#pragma unroll
            for (int L = 0; L < T; ++L) {
                const int y = row - L - 1; // centre row of this level
                if (!FULL && (y < y0 - T + L || y >= y1 + T - 1 - L)) {
                    // outside this level's rows: only move the incoming row in
#pragma unroll
                    for (int k = 0; k < VEC; ++k) {
                        if (RK && L % 2 == 0) {
                            iub[k] = cb[L][k];
                            iun[k] = cn[L][k];
                        }
                        if (RK && L % 2 == 1) {
                            cub[L][k] = iub[k];
                            cun[L][k] = iun[k];
                        }
                        cb[L][k] = ib[k];
                        cn[L][k] = in[k];
                        cD[L][k] = iD[k];
                        cX[L][k] = iX[k];
                        cs[L][k] = is[k];
                    }
                    continue;
                }
                const bool vv = !CHECK || ((y >= 0) && (y + 1 < a.ny));
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
                if (RK && L % 2 == 1) {
                    // second stage: the step's result is the average of its input u
                    // and the two chained Euler stages
#pragma unroll
                    for (int k = 0; k < VEC; ++k) {
                        ob[k] = rk2_average<R>(cub[L][k], ob[k]);
                        on[k] = rk2_average<R>(cun[L][k], on[k]);
                        cub[L][k] = iub[k];
                        cun[L][k] = iun[k];
                    }
                }
                if (RK && L % 2 == 0) {
#pragma unroll
                    for (int k = 0; k < VEC; ++k) {
                        iub[k] = cb[L][k];
                        iun[k] = cn[L][k];
                    }
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
                    if (NOISE && level_step(L + 1) != level_step(L)) {
                        // the next level advances a later step: fresh sigma of row y
                        noise_half_sigma<R, VEC>(a.z, level_step(L + 1), x0, y, os);
                    }
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
    };

    // every level is active on rows [y0 + T - 1, re): lead-in groups, the
    // steady state, then the tail (three loops, so that the steady loop
    // carries its state in the same registers from one trip to the next)
    const int full_lo = y0 + T - 1;
    int r0 = rs;
    for (; r0 < re && r0 < full_lo; r0 += PF)
        group(r0, BoolTag<false>());
    for (; r0 + PF <= re; r0 += PF)
        group(r0, BoolTag<true>());
    for (; r0 < re; r0 += PF)
        group(r0, BoolTag<false>());
}

// Diagnostics of the output block of strip (sx, sy) after stream_strip<.., T, ..>
// stored it (see the header comment).
template <typename R, int T>
__device__ __forceinline__ void strip_diag(const StripArgs<R> &a, int sx, int sy, DiagAcc &acc)
{
    constexpr int VEC = StreamShape<R>::VEC;
    constexpr int HX = Halo<T, VEC>::HX;
    constexpr int WC = Halo<T, VEC>::WC;
    constexpr int OW = Halo<T, VEC>::OW;
    typedef typename VecT<R, VEC>::type vec_t;
    const int lane = threadIdx.x & 63;
    const int x0 = sx * OW - HX + lane * VEC;
    const int y0 = sy * a.rows;
    const int y1 = min(y0 + a.rows, a.ny);
    const bool lane_out = (lane * VEC >= HX) && (lane * VEC < WC - HX) && (x0 < a.nx);
    if (!lane_out)
        return;
    for (int y = y0; y < y1; ++y) {
        const size_t p = (size_t)y * a.pitch + x0;
        const vec_t vb = *reinterpret_cast<const vec_t *>(a.b_out + p);
        const vec_t vn = *reinterpret_cast<const vec_t *>(a.n_out + p);
        const double dy = (double)y - a.cy;
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            if (x0 + k < a.nx) {
                const double bv = (double)vb[k];
                acc.sb += bv;
                acc.sn += (double)vn[k];
                if (bv >= a.b_thr) {
                    const double dx = (double)(x0 + k) - a.cx;
                    acc.m2 = fmax(acc.m2, dx * dx + dy * dy);
                    acc.cnt += 1.0;
                }
            }
        }
    }
}

// Butterfly reductions over the 64 lanes of a wavefront (fixed order).
__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max64(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

} // namespace kc
