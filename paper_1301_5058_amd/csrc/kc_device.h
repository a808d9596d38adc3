// kc_device.h -- per-cell arithmetic of the explicit step, shared by every
// kernel of the library so that all launch shapes produce identical bits.
//
// Discrete operator (finite volumes of width h, forward Euler; Sec. 2.4
// eqs. eqnadim / eqbadim with no-flux faces, eq. bconds):
//
//   G(P,Q)  = inflow into P across the face shared with Q, times h^2:
//             gb = (Dh_P + Dh_Q)(b_Q - b_P) - X_up (n_Q - n_P)
//             gn = n_Q - n_P
//     Dh    = sigma n b / 2            (half the Kawasaki diffusivity, eq. CoefCrsDif)
//     X     = chi sigma n b^2 chihat(n) (chemotactic coefficient, eq. chemflux
//                                        normalised as in eq. eqbadim)
//     X_up  = X_P if n_Q > n_P else X_Q (donor cell of the chemotactic flux)
//   F(P)    = (G(P,E) - G(W,P)) + (G(P,N) - G(S,P))   (E/W along x, N = row+1)
//   b'      = b + lam F_b + dt theta kappa n b
//   n'      = n + lam D_n F_n - dt kappa n b          (lam = dt / h^2)
//
// A boundary face contributes exactly zero.  The library is compiled without
// FMA contraction; the FMAs below are explicit, so every kernel that calls
// these functions on the same inputs produces the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kc {

// Constants of one run, in the field precision R.
template <typename R> struct Coef {
    R lam;   // dt / h^2
    R lamDn; // dt D_n / h^2
    R gro;   // dt theta kappa
    R upt;   // dt kappa
    R chi2;  // 2 chi   (X = chi2 * Dh * b * chihat)
};

template <typename R> __device__ __forceinline__ R rcp(R x);
// v_rcp_f32: 1 ulp reciprocal; (1+n)^2 >= 1 so no denormal or overflow case.
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
// v_rcp_f64 refined by two Newton-Raphson steps r <- r + r (1 - x r), each an
// FMA pair: within an ulp of 1/x for the arguments here ((1+n)^2 in [1, 16]),
// five instructions instead of the correctly rounded division's ten.
template <> __device__ __forceinline__ double rcp<double>(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Per-cell coefficients from (sigma/2, n, b).
template <typename R, int LAW>
__device__ __forceinline__ void coef(R sh, R n, R b, R chi2, R &Dh, R &X)
{
    Dh = (sh * n) * b;
    const R xb = (chi2 * Dh) * b;
    if (LAW == 0) {
        const R t = R(1) + n;
        X = xb * rcp<R>(t * t);
    } else {
        X = xb;
    }
}

// Face inflow G(P,Q); `valid` false for a boundary face (zero flux).
template <typename R>
__device__ __forceinline__ void face(R bP, R nP, R DP, R XP, R bQ, R nQ, R DQ, R XQ, bool valid,
                                     R &gb, R &gn)
{
    const R dn = nQ - nP;
    const R db = bQ - bP;
    // donor: dn > 0 exactly when nQ > nP (gradual underflow keeps the sign of a
    // non-zero difference; the kernels keep denormals), and it lets the
    // neighbour's nQ arrive through a DPP operand of the subtraction alone
    const R xu = (dn > R(0)) ? XP : XQ;
    const R g = fmaR(-xu, dn, (DP + DQ) * db);
    gb = valid ? g : R(0);
    gn = valid ? dn : R(0);
}

// Net inflow from the four face values, in one fixed order.
template <typename R>
__device__ __forceinline__ R net(R ge, R gw, R gnorth, R gsouth)
{
    return (ge - gw) + (gnorth - gsouth);
}

// Forward-Euler update of one cell.
template <typename R>
__device__ __forceinline__ void update(R b, R n, R Fb, R Fn, const Coef<R> &c, R &bo, R &no)
{
    const R nb = n * b;
    bo = fmaR(c.gro, nb, fmaR(c.lam, Fb, b));
    no = fmaR(-c.upt, nb, fmaR(c.lamDn, Fn, n));
}

// Result of a step of the two-stage Runge-Kutta method (Sec. 3): the average of
// the step's input u and the two chained Euler stages E(E(u)).
template <typename R> __device__ __forceinline__ R rk2_average(R u, R e2)
{
    return R(0.5) * (u + e2);
}

// ---------------------------------------------------------------------------
// Per-step agar noise (Sec. 3): sigma = sigma0 (1 + a Delta), Delta triangular
// on [-1, 1], redrawn for every cell and time step from the counter-based
// generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011).  Counter (x / 4, y, step low word,
// step high word), key (seed low word, seed high word); cell x takes output
// word x mod 4, and its two 16-bit halves k1, k2 give Delta = (k1 + k2) 2^-16
// - 1.  sigma / 2 is affine in k = k1 + k2 (an integer below 2^17, exact in
// either precision): sigma / 2 = h0 + h1 k with h0 = sigma0 (1 - a) / 2 and
// h1 = sigma0 a 2^-17, one FMA per cell.
// ---------------------------------------------------------------------------
template <typename R> struct Noise {
    R h0, h1;            // sigma / 2 = h0 + h1 (k1 + k2)
    uint32_t k0, k1;     // seed words
    uint32_t s_lo, s_hi; // time step of the launch's first step
};

// a ^ b ^ k in one v_bitop3_b32 (truth table 0x96 = 0xF0 ^ 0xCC ^ 0xAA); k is
// wave-uniform (a key word).  The compiler emits two XORs for this chain.
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t x0 = xor3_uniform((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t x2 = xor3_uniform((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = x0;
        c2 = x2;
        k0 += 0x9E3779B9u; // Weyl key schedule
        k1 += 0xBB67AE85u;
    }
}

// Step `ds` after the launch's first step, as (low, high) words.
template <typename R>
__device__ __forceinline__ void noise_step(const Noise<R> &z, int ds, uint32_t &lo, uint32_t &hi)
{
    lo = z.s_lo + (uint32_t)ds;
    hi = z.s_hi + (lo < z.s_lo ? 1u : 0u);
}

// sigma / 2 of one generator word.
template <typename R> __device__ __forceinline__ R noise_half(const Noise<R> &z, uint32_t w)
{
    return fmaR(z.h1, (R)((w & 0xffffu) + (w >> 16)), z.h0);
}

// sigma / 2 of cells x4 .. x4 + VEC - 1 of row y at step ds (x4 a multiple of VEC;
// VEC = 4: one generator call, VEC = 2: the matching half of one).
template <typename R, int VEC>
__device__ __forceinline__ void noise_half_sigma(const Noise<R> &z, int ds, int x4, int y, R *out)
{
    uint32_t lo, hi;
    noise_step<R>(z, ds, lo, hi);
    uint32_t c0 = (uint32_t)x4 >> 2, c1 = (uint32_t)y, c2 = lo, c3 = hi;
    philox4x32_10(c0, c1, c2, c3, z.k0, z.k1);
    if (VEC == 4) { // x4 is a multiple of 4: the whole call
        out[0] = noise_half<R>(z, c0);
        out[1] = noise_half<R>(z, c1);
        out[2 % VEC] = noise_half<R>(z, c2);
        out[3 % VEC] = noise_half<R>(z, c3);
    } else { // VEC = 2: words 0, 1 or 2, 3
        const bool upper = (x4 & 2) != 0;
        out[0] = noise_half<R>(z, upper ? c2 : c0);
        out[1 % VEC] = noise_half<R>(z, upper ? c3 : c1);
    }
}

// sigma / 2 of the single cell (x, y) at step ds (the reference kernel).
template <typename R>
__device__ __forceinline__ R noise_half_sigma1(const Noise<R> &z, int ds, int x, int y)
{
    uint32_t lo, hi;
    noise_step<R>(z, ds, lo, hi);
    uint32_t c0 = (uint32_t)x >> 2, c1 = (uint32_t)y, c2 = lo, c3 = hi;
    philox4x32_10(c0, c1, c2, c3, z.k0, z.k1);
    const int q = x & 3;
    const uint32_t w = q == 0 ? c0 : q == 1 ? c1 : q == 2 ? c2 : c3;
    return noise_half<R>(z, w);
}

// ---------------------------------------------------------------------------
// Cross-lane moves inside a 64-lane wavefront (DPP wave shifts, GFX9 family).
//   from_next(v): lane i receives lane i+1's v (lane 63 receives 0)
//   from_prev(v): lane i receives lane i-1's v (lane 0 receives 0)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dpp_next_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false); }

__device__ __forceinline__ float from_next(float v) { return __int_as_float(dpp_next_i(__float_as_int(v))); }
__device__ __forceinline__ float from_prev(float v) { return __int_as_float(dpp_prev_i(__float_as_int(v))); }
__device__ __forceinline__ double from_next(double v)
{
    const int64_t u = __double_as_longlong(v);
    const int lo = dpp_next_i((int)(uint32_t)u), hi = dpp_next_i((int)(u >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double from_prev(double v)
{
    const int64_t u = __double_as_longlong(v);
    const int lo = dpp_prev_i((int)(uint32_t)u), hi = dpp_prev_i((int)(u >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Workgroup index remapped so that each of the 8 XCDs (which receive
// workgroups round-robin) owns one contiguous range of logical tiles and its
// L2 sees the halo rows that neighbouring tiles share.
__device__ __forceinline__ int xcd_block(int nblocks_padded)
{
    const int per = nblocks_padded >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

} // namespace kc
