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
// launch: read b, n, sigma once, write b', n' once, plus the halo: the 2 T
// rows a strip shares with its vertical neighbours are read by both, at
// opposite ends of their walks, so L2 rarely still holds them.
//
// No-flux walls by reflection: cells outside the grid are ghost cells holding
// the values of their mirror images (row -1 mirrors row 0, row -2 row 1, ...,
// column nx mirrors column nx - 1, ...; the even extension of period 2 nx, 2 ny).
// A face between a cell and its mirror then carries exactly +0 (equal values
// on both sides), which is what a masked boundary face contributes, and a
// ghost cell's update is bit for bit its mirror's: the face fluxes on the
// mirrored side are exact negations (x - y = -(y - x), the donor choice and
// the fused multiply-add are symmetric under the reflection).  So the kernel
// needs no face masks and no boundary-specific arithmetic; its cells are the
// same bits as the masked one-step reference kernel's.  A strip whose cells
// all lie in the grid (EDGE = false) loads 16-byte vectors; an edge strip
// loads cell by cell from the mirrored columns (the rows are mirrored in both).
//
// With NOISE the agar field is redrawn at every time step (noise_half_sigma,
// kc_device.h): each level computes sigma of its incoming row for the step it
// advances instead of loading it (the two Runge-Kutta levels of a step share
// the step's field, passed along as before).  A ghost cell draws its mirror's
// sigma.
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
// and the last rows) runs a straight-line body without it.
//
// A folded strip (FOLD) serves the last strip column of a grid whose last
// column holds few output cells: its wavefront holds several bands of
// fold_lanes lanes, band j advancing the strip of row sy * fold_bands + j of
// that column (each band a narrow strip with its own halo lanes; what the DPP
// exchange brings in across a band boundary stays in the halo).  The walk runs
// in coordinates relative to each band's first output row, so the loops and
// the level tests stay wave-uniform; rows in memory are per lane.  The last
// strip row may be short: its band computes the nominal rows (ghost rows below
// the grid, mirrored like any) and stores only those inside.
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
    int nsy;  // strip rows (FOLD only)
    int fold_bands, fold_lanes; // bands of a folded strip and lanes per band (FOLD only)
    uint32_t field_bytes;       // bytes of one field, pitch * ny (FOLD only)
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

// Index r reflected into [0, n): the even extension of period 2 n (row -1 is
// row 0, row n is row n - 1).  Uniform or per lane; a few steps at most.
__device__ __forceinline__ int mirror_index(int r, int n)
{
    while (r < 0 || r >= n)
        r = r < 0 ? -1 - r : 2 * n - 1 - r;
    return r;
}

// Buffer resource of one row of a field (base, size in bytes): loads and
// stores through it take the row base in scalar registers and a 32-bit byte
// offset per lane, so no per-lane 64-bit address arithmetic is issued; an
// offset past the row reads 0 and writes nothing.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *row, int nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(row), (short)0, nbytes,
                                             0x00020000);
}

template <typename V> __device__ __forceinline__ V buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <typename V> __device__ __forceinline__ V buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    static_assert(sizeof(V) == 16, "16-byte vector");
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <typename V>
__device__ __forceinline__ void buf_store16(V v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    static_assert(sizeof(V) == 16, "16-byte vector");
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, off, 0, 0);
}

// (a & m) | (b & ~m) bit for bit, m all ones or all zeros.
__device__ __forceinline__ float select_bits(uint32_t m, float a, float b)
{
    return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}
__device__ __forceinline__ double select_bits(uint32_t m, double a, double b)
{
    const uint64_t mm = ((uint64_t)m << 32) | m;
    return __longlong_as_double((int64_t)(((uint64_t)__double_as_longlong(a) & mm) |
                                          ((uint64_t)__double_as_longlong(b) & ~mm)));
}

// The same for 0 <= r < 2 n (one reflection at the far wall, no branch).
__device__ __forceinline__ int mirror_high(int r, int n) { return r >= n ? 2 * n - 1 - r : r; }

// True when every cell of strip (sx, sy) lies inside the columns of the grid
// (the vectorised loads need no reflection).
template <typename R, int T>
__device__ __forceinline__ bool strip_inside(const StripArgs<R> &a, int sx)
{
    constexpr int VEC = StreamShape<R>::VEC;
    constexpr int HX = Halo<T, VEC>::HX;
    constexpr int OW = Halo<T, VEC>::OW;
    constexpr int WC = Halo<T, VEC>::WC;
    const int xl = sx * OW - HX;
    return xl >= 0 && xl + WC <= a.nx;
}

// Roles of a wavefront in a strip: the whole block of T levels (WHOLE), or
// half of it with the other half in a second wavefront of the same workgroup
// (SPLIT_FIRST: levels [0, T/2), input rows from memory, its last level's rows
// handed over through a ring of LDS slots; SPLIT_SECOND: levels [T/2, T),
// input rows from that ring, output rows to memory).
enum { WHOLE = 0, SPLIT_FIRST = 1, SPLIT_SECOND = 2 };

// LDS ring between the two wavefronts of a split strip: 2 PF row slots of b
// and n (two groups of PF rows, double-buffered), 64 lanes of VEC cells each.
template <typename R, int PF> struct SplitRing {
    typedef typename VecT<R, StreamShape<R>::VEC>::type vec_t;
    vec_t v[2 * PF][2][64];
};

template <typename R, int T, int LAW, int PF, bool EDGE, bool RK = false, bool NOISE = false,
          bool GEN = false, int ROLE = WHOLE, bool FOLD = false>
__device__ __forceinline__ void stream_strip(const StripArgs<R> &a, int sx, int sy,
                                             SplitRing<R, PF> *ring = nullptr)
{
    static_assert(!FOLD || (EDGE && !GEN), "a folded strip is an edge strip of a grid whose "
                                           "width is a multiple of the vector width");
    static_assert(!RK || T % 2 == 0, "a two-stage Runge-Kutta block has an even level count");
    static_assert(ROLE == WHOLE || (T % 2 == 0 && (!RK || (T / 2) % 2 == 0)),
                  "a split strip hands over whole time steps");
    constexpr int L0 = ROLE == SPLIT_SECOND ? T / 2 : 0; // first level of this wavefront
    constexpr int L1 = ROLE == SPLIT_FIRST ? T / 2 : T;  // one past its last level
    constexpr int VEC = StreamShape<R>::VEC;
    constexpr int HX = Halo<T, VEC>::HX;
    constexpr int WC = Halo<T, VEC>::WC;
    constexpr int OW = Halo<T, VEC>::OW;
    typedef typename VecT<R, VEC>::type vec_t;

    const int lane = threadIdx.x & 63;
    // FOLD: the lane's band and its lane within the band; a lane past the last
    // band (or whose strip row does not exist) follows band 0 and stores nothing
    int lb = lane, sy_l = sy;
    bool band_ok = true;
    if constexpr (FOLD) {
        const int band = lane / a.fold_lanes;
        lb = lane - band * a.fold_lanes;
        band_ok = band < a.fold_bands && sy * a.fold_bands + band < a.nsy;
        sy_l = sy * a.fold_bands + (band_ok ? band : 0);
    }
    const int x0 = sx * OW - HX + lb * VEC; // first column of this lane
    // rows: absolute (y0 = first output row), or with FOLD relative to the
    // lane's band (ybase its first output row, ylim one past its last in the grid)
    const int ybase = FOLD ? sy_l * a.rows : 0;
    const int ylim = FOLD ? min(ybase + a.rows, a.ny) : 0;
    const int y0 = FOLD ? 0 : sy * a.rows;
    const int y1 = FOLD ? a.rows : min(y0 + a.rows, a.ny);
    const int rs = y0 - T; // first input row (rows outside the grid are mirrored)
    const int re = y1 + T; // one past the last input row needed
    const bool lane_out =
        band_ok && (lb * VEC >= HX) && (lb * VEC < WC - HX) && (x0 < a.nx);

    // Edge strips: the mirrored column of each of the lane's cells.  When nx is
    // a multiple of VEC (GEN = false) the reflections map every aligned block of
    // VEC cells onto an aligned block, forward or reversed, so a lane's noise is
    // one generator call for that block; otherwise (GEN) each cell draws its own.
    int xm[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k)
        xm[k] = EDGE ? mirror_index(x0 + k, a.nx) : x0 + k;
    const bool nrev = EDGE && xm[VEC - 1] < xm[0]; // the block is reversed
    const int nbx = nrev ? xm[VEC - 1] : xm[0];     // its first column
    const uint32_t rmask = nrev ? 0xffffffffu : 0u; // bit mask of the reversal

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

    // Prefetch ring: slot (row - rs) % PF.  Rows are reflected into the grid;
    // rows past the strip's last input row re - 1 are never used and load row
    // re - 1 again (a cache hit) instead of the next strip's rows; interior
    // strips load one 16-byte vector per field, edge strips one cell at a time
    // from the mirrored columns.
    // In the steady state (FULL groups) every row is >= 0 and below 2 ny, so one
    // branch-free reflection suffices; the lead-in and tail groups reflect in
    // general.
    vec_t pb[PF], pn[PF], ps[PF];
    auto mrow = [&](int row, auto full_tag) __attribute__((always_inline)) {
        const int r = FOLD ? ybase + row : row;
        if constexpr (decltype(full_tag)::value)
            return mirror_high(r, a.ny);
        else
            return mirror_index(r, a.ny);
    };
    auto load_row = [&](int row, vec_t &vb, vec_t &vn, vec_t &vs, auto full_tag)
                        __attribute__((always_inline)) {
        if constexpr (FOLD) {
            // the row differs per lane: the whole field through one buffer
            // resource, row and column in the lane's byte offset
            const uint32_t rowoff = (uint32_t)mrow(row, full_tag) * (uint32_t)a.pitch;
            const __amdgpu_buffer_rsrc_t rb = row_rsrc(a.b_in, (int)a.field_bytes);
            const __amdgpu_buffer_rsrc_t rn = row_rsrc(a.n_in, (int)a.field_bytes);
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                const uint32_t o = (rowoff + (uint32_t)xm[k]) * (uint32_t)sizeof(R);
                vb[k] = buf_load<R>(rb, o);
                vn[k] = buf_load<R>(rn, o);
                vs[k] = NOISE ? R(0) : buf_load<R>(row_rsrc(a.sg, (int)a.field_bytes), o);
            }
            return;
        }
        // the row (uniform) through a buffer resource, the lane's byte offset
        const size_t base = (size_t)mrow(row, full_tag) * a.pitch;
        const int nbytes = a.pitch * (int)sizeof(R);
        const __amdgpu_buffer_rsrc_t rb = row_rsrc(a.b_in + base, nbytes);
        const __amdgpu_buffer_rsrc_t rn = row_rsrc(a.n_in + base, nbytes);
        if constexpr (!EDGE) {
            const uint32_t o = (uint32_t)x0 * (uint32_t)sizeof(R);
            vb = buf_load16<vec_t>(rb, o);
            vn = buf_load16<vec_t>(rn, o);
            if constexpr (!NOISE)
                vs = buf_load16<vec_t>(row_rsrc(a.sg + base, nbytes), o);
            else
                vs = vec_t{};
        } else {
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                const uint32_t o = (uint32_t)xm[k] * (uint32_t)sizeof(R);
                vb[k] = buf_load<R>(rb, o);
                vn[k] = buf_load<R>(rn, o);
                vs[k] = NOISE ? R(0) : buf_load<R>(row_rsrc(a.sg + base, nbytes), o);
            }
        }
    };
    // sigma / 2 of the lane's cells in row `row` at step ds after the launch's
    // first (the mirror images' for ghost cells)
    auto draw = [&](int ds, int row, R *out, auto full_tag) __attribute__((always_inline)) {
        const int yr = mrow(row, full_tag);
        if (!EDGE) {
            noise_half_sigma<R, VEC>(a.z, ds, x0, yr, out);
        } else if (!GEN) {
            R t[VEC];
            noise_half_sigma<R, VEC>(a.z, ds, nbx, yr, t);
            // cell k takes word VEC - 1 - k of a reversed block: one bitwise
            // select per 32 bits (v_bfi_b32), not a dynamic index
#pragma unroll
            for (int k = 0; k < VEC; ++k)
                out[k] = select_bits(rmask, t[VEC - 1 - k], t[k]);
        } else {
#pragma unroll
            for (int k = 0; k < VEC; ++k)
                out[k] = noise_half_sigma1<R>(a.z, ds, xm[k], yr);
        }
    };
    // time step (after the launch's first) that level L advances
    auto level_step = [](int L) { return RK ? L / 2 : L; };
    // the second wavefront of a split strip loads only sigma (static field),
    // for its incoming rows (row - L0 at iteration row)
    auto load_sigma = [&](int row, vec_t &vs, auto full_tag) __attribute__((always_inline)) {
        if constexpr (!NOISE && FOLD) {
            const uint32_t rowoff = (uint32_t)mrow(row, full_tag) * (uint32_t)a.pitch;
            const __amdgpu_buffer_rsrc_t rsg = row_rsrc(a.sg, (int)a.field_bytes);
#pragma unroll
            for (int k = 0; k < VEC; ++k)
                vs[k] = buf_load<R>(rsg, (rowoff + (uint32_t)xm[k]) * (uint32_t)sizeof(R));
        } else if constexpr (!NOISE) {
            const size_t base = (size_t)mrow(row, full_tag) * a.pitch;
            const int nbytes = a.pitch * (int)sizeof(R);
            const __amdgpu_buffer_rsrc_t rsg = row_rsrc(a.sg + base, nbytes);
            if constexpr (!EDGE) {
                vs = buf_load16<vec_t>(rsg, (uint32_t)x0 * (uint32_t)sizeof(R));
            } else {
#pragma unroll
                for (int k = 0; k < VEC; ++k)
                    vs[k] = buf_load<R>(rsg, (uint32_t)xm[k] * (uint32_t)sizeof(R));
            }
        } else {
            vs = vec_t{};
        }
    };
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        if constexpr (ROLE == SPLIT_SECOND)
            load_sigma(min(rs - L0 + u, re - 1 - L0), ps[u], BoolTag<false>());
        else
            load_row(min(rs + u, re - 1), pb[u], pn[u], ps[u], BoolTag<false>());
    }

    // One group of PF rows.  With FULL every level is active on every row of
    // the group (the steady state), so the body is one straight-line block.
    auto group = [&](int r0, int slot0, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int row = r0 + u;
            // consume slot u (row), refill it with row + PF
            R ib[VEC], in[VEC], iD[VEC], iX[VEC], is[VEC];
            R iub[VEC], iun[VEC]; // RK: u of the incoming row of an odd level
            if constexpr (ROLE == SPLIT_SECOND) {
                // incoming row of level L0: what the first wavefront handed over
                const vec_t vb = ring->v[slot0 + u][0][lane];
                const vec_t vn = ring->v[slot0 + u][1][lane];
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    ib[k] = vb[k];
                    in[k] = vn[k];
                    is[k] = R(0.5) * ps[u][k];
                    iub[k] = iun[k] = R(0);
                }
                if (NOISE) // sigma of row - L0 at the step of level L0
                    draw(level_step(L0), row - L0, is, full_tag);
                load_sigma(min(row - L0 + PF, re - 1 - L0), ps[u], full_tag);
            } else {
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    ib[k] = pb[u][k];
                    in[k] = pn[u][k];
                    is[k] = R(0.5) * ps[u][k];
                    iub[k] = iun[k] = R(0);
                }
                if (NOISE) // sigma of the incoming row at the first level's step
                    draw(level_step(0), row, is, full_tag);
                load_row(min(row + PF, re - 1), pb[u], pn[u], ps[u], full_tag);
            }
#pragma unroll
            for (int k = 0; k < VEC; ++k)
                coef<R, LAW>(is[k], in[k], ib[k], a.c.chi2, iD[k], iX[k]);

#pragma unroll
            for (int L = L0; L < L1; ++L) {
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
                R gvb[VEC], gvn[VEC], geb[VEC], gen[VEC];
#pragma unroll
                for (int k = 0; k < VEC; ++k)
                    face<R>(cb[L][k], cn[L][k], cD[L][k], cX[L][k], ib[k], in[k], iD[k], iX[k], true,
                            gvb[k], gvn[k]);
#pragma unroll
                for (int k = 0; k + 1 < VEC; ++k)
                    face<R>(cb[L][k], cn[L][k], cD[L][k], cX[L][k], cb[L][k + 1], cn[L][k + 1],
                            cD[L][k + 1], cX[L][k + 1], true, geb[k], gen[k]);
                {
                    const R eb = from_next(cb[L][0]), en = from_next(cn[L][0]);
                    const R eD = from_next(cD[L][0]), eX = from_next(cX[L][0]);
                    face<R>(cb[L][VEC - 1], cn[L][VEC - 1], cD[L][VEC - 1], cX[L][VEC - 1], eb, en,
                            eD, eX, true, geb[VEC - 1], gen[VEC - 1]);
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
                if (L + 1 < L1) {
                    if (NOISE && level_step(L + 1) != level_step(L)) {
                        // the next level advances a later step: fresh sigma of row y
                        draw(level_step(L + 1), y, os, full_tag);
                    }
#pragma unroll
                    for (int k = 0; k < VEC; ++k) {
                        ib[k] = ob[k];
                        in[k] = on[k];
                        is[k] = os[k];
                        coef<R, LAW>(is[k], in[k], ib[k], a.c.chi2, iD[k], iX[k]);
                    }
                } else if (L1 < T) {
                    // the next level runs in the second wavefront: hand over b, n of
                    // row y (it takes sigma and the coefficients itself)
#pragma unroll
                    for (int k = 0; k < VEC; ++k) {
                        ib[k] = ob[k];
                        in[k] = on[k];
                    }
                } else if (y >= y0 && y < y1 && lane_out && (!FOLD || ybase + y < ylim)) {
                    vec_t vb, vn;
#pragma unroll
                    for (int k = 0; k < VEC; ++k) {
                        vb[k] = ob[k];
                        vn[k] = on[k];
                    }
                    if constexpr (FOLD) {
                        const uint32_t o =
                            ((uint32_t)(ybase + y) * (uint32_t)a.pitch + (uint32_t)x0) *
                            (uint32_t)sizeof(R);
                        buf_store16<vec_t>(vb, row_rsrc(a.b_out, (int)a.field_bytes), o);
                        buf_store16<vec_t>(vn, row_rsrc(a.n_out, (int)a.field_bytes), o);
                    } else {
                        const size_t rowp = (size_t)y * a.pitch;
                        const int nbytes = a.pitch * (int)sizeof(R);
                        const uint32_t o = (uint32_t)x0 * (uint32_t)sizeof(R);
                        buf_store16<vec_t>(vb, row_rsrc(a.b_out + rowp, nbytes), o);
                        buf_store16<vec_t>(vn, row_rsrc(a.n_out + rowp, nbytes), o);
                    }
                }
            }
            if constexpr (ROLE == SPLIT_FIRST) {
                // the incoming row of level L1 (computed, or passed through where
                // the last level skipped this row) into the ring
                vec_t vb, vn;
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    vb[k] = ib[k];
                    vn[k] = in[k];
                }
                ring->v[slot0 + u][0][lane] = vb;
                ring->v[slot0 + u][1][lane] = vn;
            }
        }
    };
    // Split strips: the first wavefront writes group g into ring half g % 2 and
    // then meets the second at a barrier; the second meets it there before
    // reading group g.  Both walk the same groups, so both pass the same number
    // of barriers, and a half is rewritten only after the barrier that follows
    // its last read.
    auto run_group = [&](int r0, auto full_tag) __attribute__((always_inline)) {
        const int slot0 = ((((r0 - rs) / PF) & 1) != 0) ? PF : 0;
        if constexpr (ROLE == SPLIT_SECOND) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        group(r0, slot0, full_tag);
        if constexpr (ROLE == SPLIT_FIRST) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
    };

    // every level is active on rows [y0 + T - 1, re): lead-in groups, the
    // steady state, then the tail (three loops, so that the steady loop
    // carries its state in the same registers from one trip to the next).  The
    // steady rows, the rows they load ahead and those they draw noise for lie
    // in [0, ny + T + PF): below 2 ny when ny >= T + PF; smaller grids run every
    // group as a tail group.
    const int full_lo = y0 + T - 1;
    const bool steady_ok = a.ny >= T + PF;
    // Wavefronts that share a SIMD issue oldest first, so the first strip
    // dispatched to a SIMD would finish long before the second, which then
    // runs alone at single-wavefront issue rate.  The strip's issue priority
    // instead falls in four steps as it advances (3 on its first quarter of
    // groups, 0 on its last): a wavefront that is ahead yields to one that is
    // behind, and the strips of a SIMD end nearly together.
    const int q1 = rs + (re - rs) / 4, q2 = rs + (re - rs) / 2, q3 = rs + 3 * (re - rs) / 4;
    auto set_priority = [&](int r0) __attribute__((always_inline)) {
        if (r0 >= q3)
            __builtin_amdgcn_s_setprio(0);
        else if (r0 >= q2)
            __builtin_amdgcn_s_setprio(1);
        else if (r0 >= q1)
            __builtin_amdgcn_s_setprio(2);
        else
            __builtin_amdgcn_s_setprio(3);
    };
    int r0 = rs;
    for (; r0 < re && r0 < full_lo; r0 += PF) {
        set_priority(r0);
        run_group(r0, BoolTag<false>());
    }
    for (; steady_ok && r0 + PF <= re; r0 += PF) {
        set_priority(r0);
        run_group(r0, BoolTag<true>());
    }
    for (; r0 < re; r0 += PF) {
        set_priority(r0);
        run_group(r0, BoolTag<false>());
    }
}

// Diagnostics of the output block of strip (sx, sy) after stream_strip<.., T, ..>
// stored it (see the header comment); FOLD: of every band of a folded strip,
// each lane its own band's rows.
template <typename R, int T, bool FOLD = false>
__device__ __forceinline__ void strip_diag(const StripArgs<R> &a, int sx, int sy, DiagAcc &acc)
{
    constexpr int VEC = StreamShape<R>::VEC;
    constexpr int HX = Halo<T, VEC>::HX;
    constexpr int WC = Halo<T, VEC>::WC;
    constexpr int OW = Halo<T, VEC>::OW;
    typedef typename VecT<R, VEC>::type vec_t;
    const int lane = threadIdx.x & 63;
    int lb = lane, sy_l = sy;
    bool band_ok = true;
    if constexpr (FOLD) {
        const int band = lane / a.fold_lanes;
        lb = lane - band * a.fold_lanes;
        band_ok = band < a.fold_bands && sy * a.fold_bands + band < a.nsy;
        sy_l = sy * a.fold_bands + (band_ok ? band : 0);
    }
    const int x0 = sx * OW - HX + lb * VEC;
    const int y0 = sy_l * a.rows;
    const int y1 = min(y0 + a.rows, a.ny);
    const bool lane_out =
        band_ok && (lb * VEC >= HX) && (lb * VEC < WC - HX) && (x0 < a.nx);
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
