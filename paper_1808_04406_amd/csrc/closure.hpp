// Learned closure for D3Q27: a per-node MLP chooses the relaxation rates of
// central-moment orders 3..6 (the omega_n of eq:omega for n >= 3).
//
// Network: x (27) -> GELU(W1 x + b1) (32) -> GELU(W2 h1 + b2) (32) -> z (4),
// omega_{3+j} = 0.5 + 1.45 sigmoid(z_j).  Inputs are the non-equilibrium
// central moments x_p = (kappa_p - kappa_eq,p) / (rho sigma_p).  FP32
// parameters are packed W1[32][27], b1[32], W2[32][32], b2[32], W3[4][32],
// b3[4] (2084 values).
//
// Inference runs on the matrix cores: v_mfma_f32_16x16x32_bf16, BF16
// operands, FP32 accumulation, one wavefront = 64 nodes.  Each layer is
// computed transposed, H^T = W X^T, with the hidden units as M and the nodes
// as N; the accumulator of tile (mt, nt) holds hidden 16 mt + 4 g + j of node
// 16 nt + r in lane 16 g + r, element j.  Ordering the K index of W2 and W3
// as k(8 g + j') = 4 g + j' (j' < 4) or 16 + 4 g + j' - 4 (j' >= 4) makes the
// two accumulators (mt = 0, 1) of a lane exactly the B operand of the next
// layer, so only the inputs pass through LDS (one transpose) and only the
// outputs move between lanes (16 shuffles).
#pragma once

#include "collide_tp.hpp"

namespace cmlb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNIn = 27, kNH = 32, kNOut = 4;
constexpr int kOW1 = 0, kOb1 = kOW1 + kNH * kNIn, kOW2 = kOb1 + kNH, kOb2 = kOW2 + kNH * kNH;
constexpr int kOW3 = kOb2 + kNH, kOb3 = kOW3 + kNOut * kNH, kNParam = kOb3 + kNOut;
static_assert(kNParam == 2084, "closure parameter count");

// Packed network used by the kernels (built on the device from FP32 params).
struct ClosureNet {
    bf16x8 w1[2][64];   // layer-1 A fragments: W1[16 mt + r][8 g + j'] (inputs >= 27 are 0)
    bf16x8 w2[2][64];   // layer-2 A fragments: W2[16 mt + r][k(8 g + j')]
    bf16x8 w3[64];      // layer-3 A fragments: W3[r][k(8 g + j')], rows r >= 4 are 0
    float b1[kNH], b2[kNH], b3[kNOut];
    float inv_norm[kNIn];
    float w2f[kNH][kNH];   // BF16-rounded weights as FP32, for the backward pass
    float w3f[kNOut][kNH];
    int tie_even;          // orders 4 and 6 relax at omega_2 (network outputs 1 and 3 unused)
};

// K order of layers 2 and 3 (see the header comment).
__host__ __device__ constexpr int kperm(int k) {
    return (k % 8) < 4 ? 4 * (k / 8) + (k % 8) : 16 + 4 * (k / 8) + (k % 8) - 4;
}

// Normal CDF Phi(a) and density factor exp(-a^2 / 2), branch-free.  Phi uses
// the rational approximation of Hastings as printed by Abramowitz and Stegun
// (formula 7.1.26: erf(y) = 1 - t (a1 + t (a2 + ... + t a5)) exp(-y^2),
// t = 1 / (1 + p y), |error| <= 1.5e-7), applied at y = |a| / sqrt(2).
__device__ __forceinline__ float normal_cdf_f(float a, float& e) {
    const float y = fabsf(a) * 0.70710678118654752f;
    const float t = recip<float>(fmaf(0.3275911f, y, 1.0f));
    float poly = fmaf(t, 1.061405429f, -1.453152027f);
    poly = fmaf(t, poly, 1.421413741f);
    poly = fmaf(t, poly, -0.284496736f);
    poly = fmaf(t, poly, 0.254829592f);
    poly *= t;
    e = __expf(-y * y);
    const float q = 0.5f * poly * e;   // Phi(-|a|)
    return a >= 0.0f ? 1.0f - q : q;
}
// GELU(a) = a Phi(a) = max(a, 0) - |a| Phi(-|a|), with no branch and no
// transcendental instruction: Phi(-x) for x = min(|a|, 4.5) is a degree-11
// polynomial in u = 2 x / 4.5 - 1 (the Chebyshev interpolant on [0, 4.5] in
// power form, evaluated by Horner's rule; paper_1808_04406_amd/gelu_poly.py
// writes the coefficients and checks the error).  Beyond 4.5 the correction
// stays at its value there, Phi(-4.5) = 3.4e-6 times 4.5.  In FP32,
// |GELU_f(a) - GELU(a)| <= 4.6e-6 |a| everywhere, far below the BF16 rounding
// of the activations (relative 2^-9).  GELU_f(+inf) = +inf; a NaN input gives
// a finite output (the state it came from is non-finite and is detected
// there).
constexpr float kGeluPoly[12] = {
    1.222619885e-02f, -7.141333294e-02f, 1.806419585e-01f, -2.448524967e-01f,
    1.588103216e-01f, 2.736721357e-02f, -1.356795843e-01f, 7.390512033e-02f,
    3.677727454e-02f, -4.407159648e-02f, -2.773498561e-03f, 9.067683363e-03f};
__device__ __forceinline__ float gelu_f(float a) {
    const float x = fminf(fabsf(a), 4.5f);
    const float u = fmaf(x, 2.0f / 4.5f, -1.0f);
    float p = kGeluPoly[11];
    static_for<0, 11>([&](auto K) { p = fmaf(p, u, kGeluPoly[10 - decltype(K)::value]); });
    return fmaf(-x, p, fmaxf(a, 0.0f));
}
__device__ __forceinline__ float gelu_grad_f(float a) {
    float e;
    const float phi = normal_cdf_f(a, e);
    return phi + a * 0.39894228040143268f * e;
}
__device__ __forceinline__ float sigmoid_f(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Pre-activations of the two hidden layers in accumulator layout (kept for
// the backward pass): a[l][mt][nt][j] = hidden 16 mt + 4 g + j of node 16 nt + r.
struct MlpTrace {
    f32x4 a1[2][4];
    f32x4 a2[2][4];
};

// Forward pass for the 64 nodes of this wavefront.  x: this lane's inputs;
// xs: this wavefront's LDS staging area (64 rows of 40 bf16); z: this lane's
// network outputs.  All 64 lanes must be active.  The caller separates
// successive uses of xs with a barrier.
template <bool KEEP>
__device__ __forceinline__ void mlp_forward_wave(const ClosureNet* __restrict__ net, const float (&x)[kNIn],
                                                 __bf16* xs, float (&z)[kNOut], MlpTrace* tr) {
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    // inputs as BF16 rows [node][k], k padded to 32 (row stride 40 keeps 16-byte alignment)
    __bf16* row = xs + lane * 40;
#pragma unroll
    for (int k = 0; k < 32; ++k) row[k] = (__bf16)(k < kNIn ? x[k] : 0.0f);
    __syncthreads();
    bf16x8 xb[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) xb[nt] = *reinterpret_cast<const bf16x8*>(xs + (16 * nt + r) * 40 + 8 * g);

    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    bf16x8 hb[4];
    // layer 1
    {
        const bf16x8 wa0 = net->w1[0][lane], wa1 = net->w1[1][lane];
        f32x4 bias[2];   // the accumulator input: W x + b in one instruction
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) bias[mt][j] = net->b1[16 * mt + 4 * g + j];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa0, xb[nt], bias[0], 0, 0, 0);
            f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa1, xb[nt], bias[1], 0, 0, 0);
            if constexpr (KEEP) {
                tr->a1[0][nt] = d0;
                tr->a1[1][nt] = d1;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                hb[nt][j] = (__bf16)gelu_f(d0[j]);
                hb[nt][4 + j] = (__bf16)gelu_f(d1[j]);
            }
        }
    }
    // layer 2
    {
        const bf16x8 wa0 = net->w2[0][lane], wa1 = net->w2[1][lane];
        f32x4 bias[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) bias[mt][j] = net->b2[16 * mt + 4 * g + j];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa0, hb[nt], bias[0], 0, 0, 0);
            f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa1, hb[nt], bias[1], 0, 0, 0);
            if constexpr (KEEP) {
                tr->a2[0][nt] = d0;
                tr->a2[1][nt] = d1;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                hb[nt][j] = (__bf16)gelu_f(d0[j]);
                hb[nt][4 + j] = (__bf16)gelu_f(d1[j]);
            }
        }
    }
    // layer 3: lanes of group 0 hold outputs 0..3 of node 16 nt + r
    const bf16x8 w3 = net->w3[lane];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3, hb[nt], zero, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float v = __shfl(d[j], r, 64);
            if (g == nt) z[j] = v + net->b3[j];
        }
    }
}

// Non-equilibrium central moments kappa'_p - kappa'_eq,p of one node (after
// tp_raw_to_central), with 0 for the conserved orders 0 and 1.
__device__ __forceinline__ void tp3_noneq(const float (&k)[27], float drho, float rho0, const float (&u)[3],
                                          float (&neq)[27]) {
    float uu[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};
    static_for<0, 27>([&](auto Pc) {
        constexpr int p = decltype(Pc)::value;
        constexpr int order = p % 3 + (p / 3) % 3 + p / 9;
        if constexpr (order >= 2) neq[p] = k[p] - tp_keq<3, p, float>(drho, rho0, u, uu);
        else neq[p] = 0.0f;
    });
}

// Transpose of tp_inverse (adjoint): population-space vector -> central-moment
// space, sweeping the axes in reverse order with the transposed 3x3 maps.
__device__ __forceinline__ void tp3_inverse_adjoint(float (&v)[27], const float (&u)[3]) {
    static_for<0, 3>([&](auto Dr) {
        constexpr int d = 2 - decltype(Dr)::value;
        constexpr int s = (d == 0) ? 1 : (d == 1 ? 3 : 9);
        static_for<0, 27>([&](auto B) {
            constexpr int base = decltype(B)::value;
            if constexpr ((base / s) % 3 == 0) {
                const float rm = v[base], r0 = v[base + s], rp = v[base + 2 * s];
                const float S = 0.5f * (rm + rp), Dd = 0.5f * (rp - rm);
                const float g2 = S - r0;
                const float g1 = Dd + 2.0f * u[d] * g2;
                const float g0 = r0 + u[d] * (u[d] * g2 + Dd);
                v[base] = g0;
                v[base + s] = g1;
                v[base + 2 * s] = g2;
            }
        });
    });
}

}  // namespace cmlb
