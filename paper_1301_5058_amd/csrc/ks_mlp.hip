// ks_mlp.hip -- velocity surrogate: 3 -> 64 -> 64 -> 64 -> 1 MLP on gfx950.
//
// mlp_kernel<TRAIN>: each wavefront runs tiles of 16 points.  Layer 1 (K = 3)
//   and layer 4 (N = 1) are VALU dot products; the two 64 x 64 layers, the
//   activation gradients through them and their weight gradients are MFMA:
//     forward   Z[p][f]  = sum_k H[p][k] W[f][k]        v_mfma_f32_16x16x32_bf16
//     backward  dH[p][k] = sum_f dZ[p][f] W[f][k]       v_mfma_f32_16x16x32_bf16
//     weights   dW[f][k] += sum_p dZ[p][f] H[p][k]     v_mfma_f32_16x16x16_bf16
//                                                       (K = the 16 points of a tile)
//   Operand layouts of both instructions: lane l = 16 g + c holds row c of A
//   and column c of B, K elements 8g..8g+7 (x32) or 4g..4g+3 (x16); the 4
//   accumulator values of lane l are rows 4g..4g+3 of column c.  Activations
//   are written to LDS both as [point][feature] and [feature][point] so that
//   every operand is one contiguous 8- or 16-byte LDS read.  Weight gradients
//   accumulate in float32 registers over all tiles of a wave and are written
//   as one per-wave partial vector (no atomics).
// adam_reduce: sums the per-wave partials in wave order (deterministic) and
//   applies one Adam step to the float32 master parameters.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "ks.h"

namespace ks {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short4v __attribute__((ext_vector_type(4)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort4v __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int OW1 = 0, OB1 = 192, OW2 = 256, OB2 = 4352, OW3 = 4416, OB3 = 8512, OW4 = 8576,
              OB4 = 8640, NP = KS_NPARAM;
constexpr int HS = 72; // row stride (elements) of [16][64] and [64][64] LDS tiles
constexpr int TS = 20; // row stride of [64][16] LDS tiles

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float f)
{
    const unsigned u = __float_as_uint(f);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short b) { return __uint_as_float((unsigned)b << 16); }
__device__ __forceinline__ float bf16_round(float f) { return bf16_val(bf16_bits(f)); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// LDS ordering inside one wavefront: wait for its LDS traffic, no code motion across
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ bf16x8 ld8(const unsigned short *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(p));
}
__device__ __forceinline__ short4v ld4(const unsigned short *p)
{
    return __builtin_bit_cast(short4v, *reinterpret_cast<const ushort4v *>(p));
}

struct MlpArgs {
    const float *params;
    const float *X; // [ntot][3]
    const float *y; // [ntot] targets (TRAIN)
    float *v;       // [ntot] outputs (inference)
    int n;          // points in this pass
    int start;      // first point; point i of the pass is (start + i) % ntot
    int ntot;
    float in_shift[3], in_inv[3];
    float out_shift, out_scale, out_inv;
    int log_target; // targets and outputs in log space: v = exp(v' scale + shift)
    float inv_b;    // 1 / n (mean of the squared error)
    float *gpart; // [waves][NP]
    float *lpart; // [waves]
};

template <bool TRAIN>
__global__ __launch_bounds__(256) void mlp_kernel(MlpArgs a)
{
    __shared__ __align__(16) unsigned short sW2[64 * HS], sW3[64 * HS];
    __shared__ __align__(16) unsigned short sW2t[TRAIN ? 64 * HS : 8], sW3t[TRAIN ? 64 * HS : 8];
    __shared__ float sW1[192], sb1[64], sb2[64], sb3[64], sW4[64], sb4;
    __shared__ __align__(16) unsigned short sH1[4][16 * HS], sH2[4][16 * HS];
    __shared__ __align__(16) unsigned short sH1t[TRAIN ? 4 : 1][64 * TS], sH2t[TRAIN ? 4 : 1][64 * TS];
    __shared__ __align__(16) unsigned short sDZ3[TRAIN ? 4 : 1][16 * HS], sDZ2[TRAIN ? 4 : 1][16 * HS];
    __shared__ __align__(16) unsigned short sDZ3t[TRAIN ? 4 : 1][64 * TS], sDZ2t[TRAIN ? 4 : 1][64 * TS];

    const int tid = threadIdx.x;
    for (int i = tid; i < 4096; i += 256) {
        const int f = i >> 6, k = i & 63;
        const unsigned short w2 = bf16_bits(a.params[OW2 + i]);
        const unsigned short w3 = bf16_bits(a.params[OW3 + i]);
        sW2[f * HS + k] = w2;
        sW3[f * HS + k] = w3;
        if (TRAIN) {
            sW2t[k * HS + f] = w2;
            sW3t[k * HS + f] = w3;
        }
    }
    if (tid < 192)
        sW1[tid] = bf16_round(a.params[OW1 + tid]);
    if (tid < 64) {
        sb1[tid] = a.params[OB1 + tid];
        sb2[tid] = a.params[OB2 + tid];
        sb3[tid] = a.params[OB3 + tid];
        sW4[tid] = bf16_round(a.params[OW4 + tid]);
    }
    if (tid == 0)
        sb4 = a.params[OB4];
    __syncthreads();

    const int w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
    const int gw = blockIdx.x * 4 + w, nw = gridDim.x * 4;
    unsigned short *H1 = sH1[w], *H2 = sH2[w];
    unsigned short *H1t = sH1t[TRAIN ? w : 0], *H2t = sH2t[TRAIN ? w : 0];
    unsigned short *DZ3 = sDZ3[TRAIN ? w : 0], *DZ2 = sDZ2[TRAIN ? w : 0];
    unsigned short *DZ3t = sDZ3t[TRAIN ? w : 0], *DZ2t = sDZ2t[TRAIN ? w : 0];

    floatx4 dW2[4][4], dW3[4][4];
    float dW1[4][3], db1[4], db2[4], db3[4], dW4[4], db4 = 0.f, lsum = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            dW2[i][j] = dW3[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
        dW1[i][0] = dW1[i][1] = dW1[i][2] = 0.f;
        db1[i] = db2[i] = db3[i] = dW4[i] = 0.f;
    }

    const int ntiles = (a.n + 15) >> 4;
    for (int tile = gw; tile < ntiles; tile += nw) {
        // my points: p = 4g + r of this tile
        float xs[4][3];
        bool valid[4];
        int idx[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = tile * 16 + 4 * g + r;
            valid[r] = i < a.n;
            idx[r] = valid[r] ? (a.start + i) % a.ntot : 0;
#pragma unroll
            for (int j = 0; j < 3; ++j)
                xs[r][j] = valid[r] ? (a.X[3 * idx[r] + j] - a.in_shift[j]) * a.in_inv[j] : 0.f;
        }
        // ---- layer 1 (VALU), feature f = 16 nb + c ----
        float g1[4][4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int f = 16 * nb + c;
            ushort4v t;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float z = sb1[f];
                z = fmaf(sW1[3 * f + 0], xs[r][0], z);
                z = fmaf(sW1[3 * f + 1], xs[r][1], z);
                z = fmaf(sW1[3 * f + 2], xs[r][2], z);
                if (TRAIN)
                    g1[nb][r] = gelu_grad(z);
                const unsigned short hb = bf16_bits(gelu(z));
                H1[(4 * g + r) * HS + f] = hb;
                t[r] = hb;
            }
            if (TRAIN)
                *reinterpret_cast<ushort4v *>(&H1t[f * TS + 4 * g]) = t;
        }
        wave_lds_sync();
        // ---- layer 2 (MFMA) ----
        float g2[4][4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&H1[c * HS + 32 * kb + 8 * g]),
                                                              ld8(&sW2[(16 * nb + c) * HS + 32 * kb + 8 * g]),
                                                              acc, 0, 0, 0);
            const int f = 16 * nb + c;
            ushort4v t;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[r] + sb2[f];
                if (TRAIN)
                    g2[nb][r] = gelu_grad(z);
                const unsigned short hb = bf16_bits(gelu(z));
                H2[(4 * g + r) * HS + f] = hb;
                t[r] = hb;
            }
            if (TRAIN)
                *reinterpret_cast<ushort4v *>(&H2t[f * TS + 4 * g]) = t;
        }
        wave_lds_sync();
        // ---- layer 3 (MFMA) ----
        float g3[4][4], h3[4][4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&H2[c * HS + 32 * kb + 8 * g]),
                                                              ld8(&sW3[(16 * nb + c) * HS + 32 * kb + 8 * g]),
                                                              acc, 0, 0, 0);
            const int f = 16 * nb + c;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[r] + sb3[f];
                if (TRAIN)
                    g3[nb][r] = gelu_grad(z);
                h3[nb][r] = bf16_round(gelu(z));
            }
        }
        // ---- layer 4 (VALU + lane reduction over the 16 feature lanes) ----
        float vp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s = 0.f;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                s = fmaf(sW4[16 * nb + c], h3[nb][r], s);
#pragma unroll
            for (int o = 1; o < 16; o <<= 1)
                s += __shfl_xor(s, o, 64);
            vp[r] = s + sb4;
        }
        if (!TRAIN) {
            if (c == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (valid[r]) {
                        const float o = vp[r] * a.out_scale + a.out_shift;
                        a.v[idx[r]] = a.log_target ? expf(o) : o;
                    }
            }
            continue;
        }
        // ---- loss and layer-4 gradients ----
        float dv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float yv = valid[r] ? a.y[idx[r]] : 1.f;
            if (a.log_target)
                yv = logf(yv);
            const float yt = valid[r] ? (yv - a.out_shift) * a.out_inv : 0.f;
            const float e = valid[r] ? vp[r] - yt : 0.f;
            dv[r] = 2.0f * e * a.inv_b;
            if (c == 0) {
                lsum = fmaf(e, e, lsum);
                db4 += dv[r];
            }
        }
        // dz3 = dv W4 gelu'(z3)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int f = 16 * nb + c;
            ushort4v t;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dW4[nb] = fmaf(dv[r], h3[nb][r], dW4[nb]);
                const float dz = dv[r] * sW4[f] * g3[nb][r];
                db3[nb] += dz;
                const unsigned short zb = bf16_bits(dz);
                DZ3[(4 * g + r) * HS + f] = zb;
                t[r] = zb;
            }
            *reinterpret_cast<ushort4v *>(&DZ3t[f * TS + 4 * g]) = t;
        }
        wave_lds_sync();
        // dW3 += dZ3^T H2 over the 16 points of the tile
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                dW3[mb][kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                    ld4(&DZ3t[(16 * mb + c) * TS + 4 * g]), ld4(&H2t[(16 * kb + c) * TS + 4 * g]),
                    dW3[mb][kb], 0, 0, 0);
        // dH2 = dZ3 W3, then dz2 = dH2 gelu'(z2)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&DZ3[c * HS + 32 * mb + 8 * g]),
                                                              ld8(&sW3t[(16 * kb + c) * HS + 32 * mb + 8 * g]),
                                                              acc, 0, 0, 0);
            const int f = 16 * kb + c;
            ushort4v t;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float dz = acc[r] * g2[kb][r];
                db2[kb] += dz;
                const unsigned short zb = bf16_bits(dz);
                DZ2[(4 * g + r) * HS + f] = zb;
                t[r] = zb;
            }
            *reinterpret_cast<ushort4v *>(&DZ2t[f * TS + 4 * g]) = t;
        }
        wave_lds_sync();
        // dW2 += dZ2^T H1
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                dW2[mb][kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                    ld4(&DZ2t[(16 * mb + c) * TS + 4 * g]), ld4(&H1t[(16 * kb + c) * TS + 4 * g]),
                    dW2[mb][kb], 0, 0, 0);
        // dH1 = dZ2 W2, dz1 = dH1 gelu'(z1); layer-1 gradients on VALU
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&DZ2[c * HS + 32 * mb + 8 * g]),
                                                              ld8(&sW2t[(16 * kb + c) * HS + 32 * mb + 8 * g]),
                                                              acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float dz = acc[r] * g1[kb][r];
                db1[kb] += dz;
                dW1[kb][0] = fmaf(dz, xs[r][0], dW1[kb][0]);
                dW1[kb][1] = fmaf(dz, xs[r][1], dW1[kb][1]);
                dW1[kb][2] = fmaf(dz, xs[r][2], dW1[kb][2]);
            }
        }
        wave_lds_sync();
    }
    if (!TRAIN)
        return;

    // ---- per-wave gradient partial ----
    float *P = a.gpart + (size_t)gw * NP;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = 16 * mb + 4 * g + r, k = 16 * kb + c;
                P[OW3 + f * 64 + k] = dW3[mb][kb][r];
                P[OW2 + f * 64 + k] = dW2[mb][kb][r];
            }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        float q[7] = {dW1[nb][0], dW1[nb][1], dW1[nb][2], db1[nb], db2[nb], db3[nb], dW4[nb]};
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            q[i] += __shfl_xor(q[i], 16, 64);
            q[i] += __shfl_xor(q[i], 32, 64);
        }
        if (g == 0) {
            const int f = 16 * nb + c;
            P[OW1 + 3 * f + 0] = q[0];
            P[OW1 + 3 * f + 1] = q[1];
            P[OW1 + 3 * f + 2] = q[2];
            P[OB1 + f] = q[3];
            P[OB2 + f] = q[4];
            P[OB3 + f] = q[5];
            P[OW4 + f] = q[6];
        }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        db4 += __shfl_xor(db4, o, 64);
        lsum += __shfl_xor(lsum, o, 64);
    }
    if (l == 0) {
        P[OB4] = db4;
        a.lpart[gw] = lsum;
    }
}

// Sum of the per-wave partials (wave order) and, when update != 0, one Adam step.
__global__ __launch_bounds__(256) void adam_reduce(float *params, float *m1, float *m2,
                                                    const float *gpart, int nwaves,
                                                    const float *lpart, float lr, float bc1,
                                                    float bc2, int update, float *grad,
                                                    double *loss, float inv_n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < NP) {
        float gs = 0.f;
        for (int w = 0; w < nwaves; ++w)
            gs += gpart[(size_t)w * NP + i];
        grad[i] = gs;
        if (update) {
            const float mm = 0.9f * m1[i] + 0.1f * gs;
            const float vv = 0.999f * m2[i] + 0.001f * gs * gs;
            m1[i] = mm;
            m2[i] = vv;
            params[i] -= lr * (mm * bc1) / (sqrtf(vv * bc2) + 1e-8f);
        }
    } else if (i == NP) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w)
            s += (double)lpart[w];
        *loss = s * (double)inv_n;
    }
}

__global__ void fill_zero(float *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0.f;
}

__global__ void hull_test(const float *X, int n, const double *facets, int nf, double tol,
                          unsigned char *inside)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double x0 = X[3 * i], x1 = X[3 * i + 1], x2 = X[3 * i + 2];
    unsigned char in = 1;
    for (int f = 0; f < nf; ++f) {
        const double *F = facets + 4 * f;
        if (F[0] * x0 + F[1] * x1 + F[2] * x2 + F[3] > tol)
            in = 0;
    }
    inside[i] = in;
}

__global__ void cbar_kernel(const float *X, int n, double sigma0, float *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double n0 = X[3 * i], chi = X[3 * i + 1];
    const double p = 3.0 - 2.0 * chi * n0;
    const double bs = 2.0 * n0 / (p + sqrt(p * p + 16.0 * chi * n0));
    const double q = 1.0 - bs / n0;
    const double psi = bs * q * q * (1.0 + chi * bs);
    out[i] = (float)(2.0 * n0 * sqrt(sigma0) * sqrt(psi));
}

// ---------------------------------------------------------------------------
// Threshold speed c* of travelling fronts of the scalar equation of Sec. 4.1,
// b_t = sigma0 (D-tilde(b, chi0) b_x)_x + g(b) (eqs. scalar-eq-b-re, D-tilde,
// reac-term), on [0, n0]: the infimum of the speeds c for which
//   dz/db = -c - H(b) / z,  H = sigma0 D-tilde g = sigma0 n0^2 b^2 q^2 (1 + chi0 b),
//   q = 1 - b / n0,  with z < 0 on (0, n0) and z(0+) = z(n0-) = 0
// has a solution (the appendix, sets defAchi0 / defA0).  Shooting: the sharp
// front leaves b = 0 along z = -c b + sigma0 n0^2 b^2 / (2c); followed upwards
// from b = eps n0, the trajectory of a c < c* meets z = 0 before b = n0, that of
// a c > c* reaches b = n0 (1 - eps) with z < 0.  Each step is one BDF2 step
// (L-stable: the problem is stiff where z -> 0), which for this equation is a
// quadratic in the new z with a closed-form root; a negative discriminant
// means no negative continuation, i.e. z has met 0.  One wavefront per point:
// its 64 lanes try 64 speeds spread over the current bracket [lo, hi]
// (initially [0, 1.05 c-bar], c* <= c-bar by Sec. 4.1), and the bracket
// shrinks 65-fold per round.
// ---------------------------------------------------------------------------
constexpr int CSTAR_STEPS = 16384;
constexpr int CSTAR_ROUNDS = 5;

__device__ double cbar_of(double n0, double chi, double sigma0)
{
    const double p = 3.0 - 2.0 * chi * n0;
    const double bs = 2.0 * n0 / (p + sqrt(p * p + 16.0 * chi * n0));
    const double q = 1.0 - bs / n0;
    return 2.0 * n0 * sqrt(sigma0) * sqrt(bs * q * q * (1.0 + chi * bs));
}

__global__ __launch_bounds__(256) void cstar_kernel(const float *X, int n, double sigma0,
                                                     float *out)
{
    const int lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (int)(threadIdx.x >> 6));
    if (i >= n)
        return; // whole wavefront
    const double n0 = X[3 * i], chi = X[3 * i + 1];
    if (!(n0 > 0.0) || !(chi >= 0.0) || !isfinite(n0) || !isfinite(chi)) {
        if (lane == 0)
            out[i] = NAN;
        return;
    }
    const double eps = 1e-6;
    const double u0 = eps * n0, u1 = n0 * (1.0 - eps);
    const double du = (u1 - u0) / CSTAR_STEPS;
    const double h2 = sigma0 * n0 * n0;
    auto H = [&](double u) {
        const double q = 1.0 - u / n0;
        return h2 * u * u * q * q * (1.0 + chi * u);
    };
    double lo = 0.0, hi = 1.05 * cbar_of(n0, chi, sigma0);
    for (int r = 0; r < CSTAR_ROUNDS; ++r) {
        const double c = lo + (lane + 1) * (hi - lo) / 65.0;
        double zm = -c * u0 + h2 * u0 * u0 / (2.0 * c);
        // first step: backward Euler, z1^2 - (z0 - du c) z1 + du H1 = 0
        const double A = zm - du * c;
        const double D1 = A * A - 4.0 * du * H(u0 + du);
        double zc = D1 >= 0.0 ? 0.5 * (A - sqrt(fmax(D1, 0.0))) : 0.0;
        bool alive = D1 >= 0.0 && zc < 0.0;
        for (int k = 2; k <= CSTAR_STEPS; ++k) {
            // BDF2: 3/2 z2 - 2 z1 + 1/2 z0 = du (-c - H / z2)
            const double B = du * c - 2.0 * zc + 0.5 * zm;
            const double D2 = B * B - 6.0 * du * H(u0 + k * du);
            const double zn = (-B - sqrt(fmax(D2, 0.0))) / 3.0;
            alive = alive && D2 >= 0.0 && zn < 0.0;
            zm = alive ? zc : zm;
            zc = alive ? zn : zc;
        }
        const unsigned long long below = __ballot(!alive);
        const int last = below ? 63 - __clzll(below) : -1;
        const double nlo = last >= 0 ? lo + (last + 1) * (hi - lo) / 65.0 : lo;
        const double nhi = last < 63 ? lo + (last + 2) * (hi - lo) / 65.0 : hi;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0)
        out[i] = (float)(0.5 * (lo + hi));
}

} // namespace ks

struct ks_model {
    int maxp = 0;
    hipStream_t stream = nullptr;
    float *params = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
    float *gpart = nullptr, *lpart = nullptr;
    double *loss = nullptr;
    float *dX = nullptr, *dy = nullptr, *dv = nullptr, *dcb = nullptr;
    unsigned char *din = nullptr;
    double *dfacets = nullptr;
    int nf = 0;
    double tol = 0;
    double in_shift[3] = {0, 0, 0}, in_scale[3] = {1, 1, 1}, out_shift = 0, out_scale = 1;
    int log_target = 0;
    long long t = 0;
    int maxwaves = 256;
    std::string err;
};

namespace {

int kfail(ks_model *m, int code, const char *fmt, ...)
{
    if (m) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        m->err = buf;
    }
    return code;
}

#define KS_HIP(mm, expr)                                                                           \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return kfail((mm), e_ == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP, "%s: %s", #expr,   \
                         hipGetErrorString(e_));                                                   \
    } while (0)

ks::MlpArgs base_args(const ks_model *m)
{
    ks::MlpArgs a;
    a.params = m->params;
    a.X = nullptr;
    a.y = nullptr;
    a.v = nullptr;
    a.n = a.start = 0;
    a.ntot = 1;
    for (int j = 0; j < 3; ++j) {
        a.in_shift[j] = (float)m->in_shift[j];
        a.in_inv[j] = (float)(1.0 / m->in_scale[j]);
    }
    a.out_shift = (float)m->out_shift;
    a.out_scale = (float)m->out_scale;
    a.out_inv = (float)(1.0 / m->out_scale);
    a.log_target = m->log_target;
    a.inv_b = 1.f;
    a.gpart = m->gpart;
    a.lpart = m->lpart;
    return a;
}

// Stage a [n][3] input (and optional [n] targets) in device memory.
int stage(ks_model *m, const float *X, const float *y, int32_t n, int mem, const float **dX,
          const float **dy)
{
    if (mem == KC_MEM_DEVICE) {
        *dX = X;
        if (dy)
            *dy = y;
        return KC_OK;
    }
    KS_HIP(m, hipMemcpyAsync(m->dX, X, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice,
                             m->stream));
    *dX = m->dX;
    if (dy) {
        KS_HIP(m, hipMemcpyAsync(m->dy, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice,
                                 m->stream));
        *dy = m->dy;
    }
    return KC_OK;
}

int waves_for(const ks_model *m, int n)
{
    const int tiles = (n + 15) / 16;
    int blocks = (tiles + 3) / 4;
    const int maxb = m->maxwaves / 4;
    if (blocks > maxb)
        blocks = maxb;
    return blocks < 1 ? 1 : blocks;
}

// One forward/backward pass over n points starting at `start` plus the reduce
// (and an Adam step when update != 0).
int train_pass(ks_model *m, const float *dX, const float *dy, int n, int start, int ntot,
               int update, double lr)
{
    ks::MlpArgs a = base_args(m);
    a.X = dX;
    a.y = dy;
    a.n = n;
    a.start = start;
    a.ntot = ntot;
    a.inv_b = (float)(1.0 / n);
    const int blocks = waves_for(m, n);
    hipLaunchKernelGGL(ks::mlp_kernel<true>, dim3(blocks), dim3(256), 0, m->stream, a);
    KS_HIP(m, hipGetLastError());
    float bc1 = 1.f, bc2 = 1.f;
    if (update) {
        ++m->t;
        bc1 = (float)(1.0 / (1.0 - pow(0.9, (double)m->t)));
        bc2 = (float)(1.0 / (1.0 - pow(0.999, (double)m->t)));
    }
    hipLaunchKernelGGL(ks::adam_reduce, dim3((ks::NP + 1 + 255) / 256), dim3(256), 0, m->stream,
                       m->params, m->m1, m->m2, m->gpart, blocks * 4, m->lpart, (float)lr, bc1,
                       bc2, update, m->grad, m->loss, (float)(1.0 / n));
    KS_HIP(m, hipGetLastError());
    return KC_OK;
}

} // namespace

extern "C" {

const char *ks_last_error(const ks_model *m) { return m ? m->err.c_str() : "null model"; }

void ks_destroy(ks_model *m)
{
    if (!m)
        return;
    (void)hipStreamSynchronize(m->stream);
    void *ptrs[] = {m->params, m->m1, m->m2, m->grad, m->gpart, m->lpart, m->loss, m->dX,
                    m->dy, m->dv, m->dcb, m->din, m->dfacets};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    delete m;
}

int ks_create(int32_t max_points, void *hip_stream, ks_model **out)
{
    if (!out)
        return KC_EINVAL;
    *out = nullptr;
    if (max_points < 1 || max_points > (1 << 26))
        return KC_EINVAL;
    int dev;
    if (hipGetDevice(&dev) != hipSuccess)
        return KC_EHIP;
    ks_model *m = new (std::nothrow) ks_model;
    if (!m)
        return KC_ENOMEM;
    m->maxp = max_points;
    m->stream = (hipStream_t)hip_stream;
    const size_t P = ks::NP * sizeof(float);
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess)
            e = hipMalloc(p, bytes);
        if (e == hipSuccess)
            e = hipMemset(*p, 0, bytes);
    };
    alloc((void **)&m->params, P);
    alloc((void **)&m->m1, P);
    alloc((void **)&m->m2, P);
    alloc((void **)&m->grad, P);
    alloc((void **)&m->gpart, (size_t)m->maxwaves * P);
    alloc((void **)&m->lpart, (size_t)m->maxwaves * sizeof(float));
    alloc((void **)&m->loss, sizeof(double));
    alloc((void **)&m->dX, (size_t)max_points * 3 * sizeof(float));
    alloc((void **)&m->dy, (size_t)max_points * sizeof(float));
    alloc((void **)&m->dv, (size_t)max_points * sizeof(float));
    alloc((void **)&m->dcb, (size_t)max_points * sizeof(float));
    alloc((void **)&m->din, (size_t)max_points);
    if (e != hipSuccess) {
        const int rc = e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
        ks_destroy(m);
        return rc;
    }
    *out = m;
    return KC_OK;
}

int ks_set_params(ks_model *m, const float *params)
{
    if (!m || !params)
        return KC_EINVAL;
    for (int i = 0; i < ks::NP; ++i)
        if (!isfinite(params[i]))
            return kfail(m, KC_ENONFINITE, "parameter %d is not finite", i);
    KS_HIP(m, hipMemcpyAsync(m->params, params, ks::NP * sizeof(float), hipMemcpyHostToDevice,
                             m->stream));
    hipLaunchKernelGGL(ks::fill_zero, dim3((ks::NP + 255) / 256), dim3(256), 0, m->stream, m->m1,
                       ks::NP);
    hipLaunchKernelGGL(ks::fill_zero, dim3((ks::NP + 255) / 256), dim3(256), 0, m->stream, m->m2,
                       ks::NP);
    KS_HIP(m, hipGetLastError());
    KS_HIP(m, hipStreamSynchronize(m->stream));
    m->t = 0;
    return KC_OK;
}

int ks_get_params(ks_model *m, float *params)
{
    if (!m || !params)
        return KC_EINVAL;
    KS_HIP(m, hipMemcpyAsync(params, m->params, ks::NP * sizeof(float), hipMemcpyDeviceToHost,
                             m->stream));
    KS_HIP(m, hipStreamSynchronize(m->stream));
    return KC_OK;
}

int ks_set_normalization(ks_model *m, const double *in_shift, const double *in_scale,
                         double out_shift, double out_scale, int32_t log_target)
{
    if (!m || !in_shift || !in_scale)
        return KC_EINVAL;
    for (int j = 0; j < 3; ++j)
        if (!isfinite(in_shift[j]) || !isfinite(in_scale[j]) || in_scale[j] == 0.0)
            return kfail(m, KC_EINVAL, "bad input map %d", j);
    if (!isfinite(out_shift) || !isfinite(out_scale) || out_scale == 0.0)
        return kfail(m, KC_EINVAL, "bad output map");
    for (int j = 0; j < 3; ++j) {
        m->in_shift[j] = in_shift[j];
        m->in_scale[j] = in_scale[j];
    }
    if (log_target != 0 && log_target != 1)
        return kfail(m, KC_EINVAL, "log_target must be 0 or 1");
    m->out_shift = out_shift;
    m->out_scale = out_scale;
    m->log_target = log_target;
    return KC_OK;
}

int ks_train(ks_model *m, const float *X, const float *v, int32_t n, int32_t iters, int32_t batch,
             double lr, int mem, double *loss)
{
    if (!m)
        return KC_EINVAL;
    m->err.clear();
    if (!X || !v || n < 1 || n > m->maxp || iters < 0 || batch < 1 || !(lr > 0) ||
        (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE))
        return kfail(m, KC_EINVAL, "bad arguments to ks_train");
    if (batch > n)
        batch = n;
    const float *dX, *dy;
    int rc = stage(m, X, v, n, mem, &dX, &dy);
    if (rc != KC_OK)
        return rc;
    long long start = 0;
    for (int it = 0; it < iters; ++it) {
        rc = train_pass(m, dX, dy, batch, (int)start, n, 1, lr);
        if (rc != KC_OK)
            return rc;
        start = (start + batch) % n;
    }
    double h = 0.0;
    KS_HIP(m, hipMemcpyAsync(&h, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->stream));
    KS_HIP(m, hipStreamSynchronize(m->stream));
    if (loss)
        *loss = h;
    return KC_OK;
}

int ks_grad(ks_model *m, const float *X, const float *v, int32_t n, float *grad, double *loss,
            int mem)
{
    if (!m)
        return KC_EINVAL;
    m->err.clear();
    if (!X || !v || !grad || n < 1 || n > m->maxp || (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE))
        return kfail(m, KC_EINVAL, "bad arguments to ks_grad");
    const float *dX, *dy;
    int rc = stage(m, X, v, n, mem, &dX, &dy);
    if (rc != KC_OK)
        return rc;
    rc = train_pass(m, dX, dy, n, 0, n, 0, 0.0);
    if (rc != KC_OK)
        return rc;
    double h = 0.0;
    KS_HIP(m, hipMemcpyAsync(grad, m->grad, ks::NP * sizeof(float), hipMemcpyDeviceToHost,
                             m->stream));
    KS_HIP(m, hipMemcpyAsync(&h, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->stream));
    KS_HIP(m, hipStreamSynchronize(m->stream));
    if (loss)
        *loss = h;
    return KC_OK;
}

int ks_predict(ks_model *m, const float *X, int32_t n, float *v, int mem)
{
    if (!m)
        return KC_EINVAL;
    m->err.clear();
    if (!X || !v || n < 1 || n > m->maxp || (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE))
        return kfail(m, KC_EINVAL, "bad arguments to ks_predict");
    const float *dX;
    int rc = stage(m, X, nullptr, n, mem, &dX, nullptr);
    if (rc != KC_OK)
        return rc;
    ks::MlpArgs a = base_args(m);
    a.X = dX;
    a.n = n;
    a.ntot = n;
    a.v = mem == KC_MEM_DEVICE ? v : m->dv;
    int blocks = ((n + 15) / 16 + 3) / 4;
    if (blocks > 2048)
        blocks = 2048;
    hipLaunchKernelGGL(ks::mlp_kernel<false>, dim3(blocks), dim3(256), 0, m->stream, a);
    KS_HIP(m, hipGetLastError());
    if (mem == KC_MEM_HOST) {
        KS_HIP(m, hipMemcpyAsync(v, m->dv, (size_t)n * sizeof(float), hipMemcpyDeviceToHost,
                                 m->stream));
        KS_HIP(m, hipStreamSynchronize(m->stream));
    }
    return KC_OK;
}

int ks_hull_set(ks_model *m, const double *facets, int32_t nf, double tol)
{
    if (!m || !facets || nf < 1 || nf > (1 << 20) || !(tol >= 0) || !isfinite(tol))
        return KC_EINVAL;
    for (int i = 0; i < 4 * nf; ++i)
        if (!isfinite(facets[i]))
            return kfail(m, KC_EINVAL, "non-finite facet entry %d", i);
    if (m->dfacets)
        (void)hipFree(m->dfacets);
    m->dfacets = nullptr;
    KS_HIP(m, hipMalloc((void **)&m->dfacets, (size_t)nf * 4 * sizeof(double)));
    KS_HIP(m, hipMemcpyAsync(m->dfacets, facets, (size_t)nf * 4 * sizeof(double),
                             hipMemcpyHostToDevice, m->stream));
    KS_HIP(m, hipStreamSynchronize(m->stream));
    m->nf = nf;
    m->tol = tol;
    return KC_OK;
}

int ks_hull_test(ks_model *m, const float *X, int32_t n, uint8_t *inside, int mem)
{
    if (!m)
        return KC_EINVAL;
    m->err.clear();
    if (!X || !inside || n < 1 || n > m->maxp || (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE))
        return kfail(m, KC_EINVAL, "bad arguments to ks_hull_test");
    if (!m->nf)
        return kfail(m, KC_ESTATE, "no hull set");
    const float *dX;
    int rc = stage(m, X, nullptr, n, mem, &dX, nullptr);
    if (rc != KC_OK)
        return rc;
    unsigned char *o = mem == KC_MEM_DEVICE ? inside : m->din;
    hipLaunchKernelGGL(ks::hull_test, dim3((n + 255) / 256), dim3(256), 0, m->stream, dX, n,
                       m->dfacets, m->nf, m->tol, o);
    KS_HIP(m, hipGetLastError());
    if (mem == KC_MEM_HOST) {
        KS_HIP(m, hipMemcpyAsync(inside, m->din, (size_t)n, hipMemcpyDeviceToHost, m->stream));
        KS_HIP(m, hipStreamSynchronize(m->stream));
    }
    return KC_OK;
}

int ks_cbar(ks_model *m, const float *X, int32_t n, double sigma0, float *out, int mem)
{
    if (!m)
        return KC_EINVAL;
    m->err.clear();
    if (!X || !out || n < 1 || n > m->maxp || !(sigma0 > 0) ||
        (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE))
        return kfail(m, KC_EINVAL, "bad arguments to ks_cbar");
    const float *dX;
    int rc = stage(m, X, nullptr, n, mem, &dX, nullptr);
    if (rc != KC_OK)
        return rc;
    float *o = mem == KC_MEM_DEVICE ? out : m->dcb;
    hipLaunchKernelGGL(ks::cbar_kernel, dim3((n + 255) / 256), dim3(256), 0, m->stream, dX, n,
                       sigma0, o);
    KS_HIP(m, hipGetLastError());
    if (mem == KC_MEM_HOST) {
        KS_HIP(m, hipMemcpyAsync(out, m->dcb, (size_t)n * sizeof(float), hipMemcpyDeviceToHost,
                                 m->stream));
        KS_HIP(m, hipStreamSynchronize(m->stream));
    }
    return KC_OK;
}

int ks_cstar(ks_model *m, const float *X, int32_t n, double sigma0, float *out, int mem)
{
    if (!m)
        return KC_EINVAL;
    m->err.clear();
    if (!X || !out || n < 1 || n > m->maxp || !(sigma0 > 0) || !isfinite(sigma0) ||
        (mem != KC_MEM_HOST && mem != KC_MEM_DEVICE))
        return kfail(m, KC_EINVAL, "bad arguments to ks_cstar");
    const float *dX;
    int rc = stage(m, X, nullptr, n, mem, &dX, nullptr);
    if (rc != KC_OK)
        return rc;
    float *o = mem == KC_MEM_DEVICE ? out : m->dcb;
    hipLaunchKernelGGL(ks::cstar_kernel, dim3((n + 3) / 4), dim3(256), 0, m->stream, dX, n,
                       sigma0, o);
    KS_HIP(m, hipGetLastError());
    if (mem == KC_MEM_HOST) {
        KS_HIP(m, hipMemcpyAsync(out, m->dcb, (size_t)n * sizeof(float), hipMemcpyDeviceToHost,
                                 m->stream));
        KS_HIP(m, hipStreamSynchronize(m->stream));
    }
    return KC_OK;
}

} // extern "C"
