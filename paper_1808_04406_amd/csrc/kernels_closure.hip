// Learned-closure kernels (D3Q27, FP32 storage): weight packing, the fused
// stream + collide step with network rates, the training forward/backward
// pass, the deterministic gradient reduction and the Adam update.
#include <cmath>

#include "closure.hpp"
#include "launch.hpp"

namespace cmlb {

// ---------------------------------------------------------------------------
// FP32 parameters -> packed BF16 MFMA fragments (one block of 256 threads)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_closure_pack(const float* __restrict__ P, const float* __restrict__ norm,
                                                      int tie_even, ClosureNet* __restrict__ net) {
    const int t = threadIdx.x;
    if (t == 0) net->tie_even = tie_even;
    auto bf = [](float v) { return (__bf16)v; };
    if (t < 128) {  // layer-1 and layer-2 fragments: (mt, lane)
        const int mt = t >> 6, lane = t & 63, g = lane >> 4, r = lane & 15;
        bf16x8 a1, a2;
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            a1[j] = bf(k < kNIn ? P[kOW1 + (16 * mt + r) * kNIn + k] : 0.0f);
            a2[j] = bf(P[kOW2 + (16 * mt + r) * kNH + kperm(k)]);
        }
        net->w1[mt][lane] = a1;
        net->w2[mt][lane] = a2;
    } else if (t < 192) {  // layer-3 fragment
        const int lane = t - 128, g = lane >> 4, r = lane & 15;
        bf16x8 a3;
        for (int j = 0; j < 8; ++j) a3[j] = bf(r < kNOut ? P[kOW3 + r * kNH + kperm(8 * g + j)] : 0.0f);
        net->w3[lane] = a3;
    }
    if (t < kNH) {
        net->b1[t] = P[kOb1 + t];
        net->b2[t] = P[kOb2 + t];
    }
    if (t < kNOut) net->b3[t] = P[kOb3 + t];
    if (t < kNIn) net->inv_norm[t] = 1.0f / norm[t];
    for (int e = t; e < kNH * kNH; e += 256) net->w2f[e / kNH][e % kNH] = (float)bf(P[kOW2 + e]);
    if (t < kNOut * kNH) net->w3f[t / kNH][t % kNH] = (float)bf(P[kOW3 + t]);
}

// Relaxation rates of orders 3..6 for this lane's node (central moments k
// after tp_raw_to_central); the non-equilibrium parts are not kept.
template <bool KEEP>
__device__ __forceinline__ void closure_rates(const ClosureNet* net, const float (&k)[27], float drho, float rho0,
                                              const float (&u)[3], __bf16* xs, float (&om)[8], MlpTrace* tr,
                                              float (&z)[kNOut]) {
    float x[kNIn];
    {
        float neq[27];
        tp3_noneq(k, drho, rho0, u, neq);
        const float inv_rho = recip<float>(rho0 + drho);
#pragma unroll
        for (int p = 0; p < kNIn; ++p) x[p] = neq[p] * inv_rho * net->inv_norm[p];
    }
    mlp_forward_wave<KEEP>(net, x, xs, z, tr);
#pragma unroll
    for (int j = 0; j < kNOut; ++j) om[3 + j] = 0.5f + 1.45f * sigmoid_f(z[j]);
    if (net->tie_even) om[4] = om[6] = om[2];
}

// ---------------------------------------------------------------------------
// Fused stream + collide with network rates.  Every lane of every wave runs
// the network (the matrix instructions need full wavefronts), lanes past the
// end of a row compute on a clamped node and do not store.
// ---------------------------------------------------------------------------
// Four waves per SIMD: the compiler then keeps the MFMA accumulators in
// VGPRs (128, two of them spilled) instead of 84 VGPRs and 48 AGPRs at three
// waves, which removes 80 accumulator reads per wave; measured 5 % faster at
// 128^3.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_step_closure(StepArgs a, const ClosureNet* __restrict__ net) {
    using T = float;
    __shared__ __bf16 xs_all[4][64 * 40];
    const uint32_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const uint32_t chunk = blockIdx.x % a.g.nchunks;
    const uint32_t row = blockIdx.x / a.g.nchunks;
    const uint32_t xr = chunk * blockDim.x + threadIdx.x;
    const bool active = xr < nx;
    const uint32_t x = active ? xr : nx - 1;
    const uint32_t y = row % ny, z = row / ny;
    const char* __restrict__ src = static_cast<const char*>(a.src);
    char* __restrict__ dst = static_cast<char*>(a.dst);
    const uint64_t plane_bytes = a.g.plane * sizeof(T);
    const uint32_t xoff[3] = {(x + 1 == nx ? 0 : x + 1) * 4u, x * 4u, (x == 0 ? nx - 1 : x - 1) * 4u};
    const uint32_t ysrc[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const uint32_t zsrc[3] = {z + 1 == nz ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
    float h[27];
    static_for<0, 27>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = TP<3>::ex(i), ey = TP<3>::ey(i), ez = TP<3>::ez(i);
        const char* rowp = src + i * plane_bytes + ((uint64_t)zsrc[ez + 1] * ny + ysrc[ey + 1]) * a.pitch * 4;
        h[i] = *reinterpret_cast<const T*>(rowp + xoff[ex + 1]);
    });
    const float rho0 = (float)a.rho0;
    tp_raw<3, float>(h);
    const TPMacro<3, float> m = tp_macro_raw<3, float>(h, rho0);
    tp_raw_to_central<3, float>(h, m.u);
    float om[8];
    static_for<0, 8>([&](auto N) { om[decltype(N)::value] = (float)a.omega[decltype(N)::value]; });
    float zz[kNOut];
    closure_rates<false>(net, h, m.drho, rho0, m.u, xs_all[threadIdx.x >> 6], om, nullptr, zz);
    tp_relax<3, float>(h, m.drho, rho0, m.u, om);
    tp_inverse<3, float>(h, m.u);
    if (!active) return;
    char* outrow = dst + ((uint64_t)z * ny + y) * a.pitch * 4;
    static_for<0, 27>([&](auto I) {
        constexpr int i = decltype(I)::value;
        Store<kF32>::store(reinterpret_cast<T*>(outrow + i * plane_bytes + xoff[1]), h[i]);
    });
}

// ---------------------------------------------------------------------------
// Training.  Mode 0: objective (1/N) sum_nodes sum_i (f*_i - fbar_i)^2 / w_i
// over pairs (state, target); f* is the closure collision of the pulled
// state.  Mode 1 (momentum two steps ahead): target holds the field
// D = (2/N)(j2 - jbar) [pair][3][nodes] of k_closure_momentum, the adjoint of
// f*_i at node y is lam_i(y) = e_i . D(y + e_i), and the objective share of a
// node is |D|^2 N / 4.  One wavefront per block; each processes 64
// consecutive nodes of a row per tile, and each lane accumulates 34 fixed
// gradient entries over its tiles.
// ---------------------------------------------------------------------------
struct TrainArgs {
    const float* state;   // [pair][27][nodes], rows unpadded
    const float* target;  // mode 0: [pair][27][nodes]; mode 1: [pair][3][nodes]
    GridArgs g;
    int64_t n_pairs;
    float rho0;
    float omega2;
    float inv_count;      // 1 / (n_pairs * nodes)
    int mode;
};

constexpr int kGradPerLane = 34;   // 14 (W1, b1) + 17 (W2, b2) + 3 (W3, b3) entries of 64 lanes
constexpr int kPartialStride = kNParam + 1;  // gradient + objective

// D3Q27 weight 1/w_i: products of (6, 3/2, 6).
__device__ __forceinline__ float inv_w27(int i) {
    const float a = (i % 3 == 1) ? 1.5f : 6.0f, b = ((i / 3) % 3 == 1) ? 1.5f : 6.0f, c = (i / 9 == 1) ? 1.5f : 6.0f;
    return a * b * c;
}

// Gradient entry owned by a lane: section (0: W1|b1, 1: W2|b2, 2: W3|b3),
// output unit j and input m (m == fan-in means the bias).
__device__ __forceinline__ bool grad_entry(int q, int lane, int& sec, int& j, int& m) {
    if (q < 14) { const int e = lane + 64 * q; sec = 0; j = e / 28; m = e % 28; return true; }
    if (q < 31) { const int e = lane + 64 * (q - 14); sec = 1; j = e / 33; m = e % 33; return e < kNH * 33; }
    const int e = lane + 64 * (q - 31); sec = 2; j = e / 33; m = e % 33; return e < kNOut * 33;
}

__device__ __forceinline__ int grad_index(int sec, int j, int m) {
    if (sec == 0) return m < kNIn ? kOW1 + j * kNIn + m : kOb1 + j;
    if (sec == 1) return m < kNH ? kOW2 + j * kNH + m : kOb2 + j;
    return m < kNH ? kOW3 + j * kNH + m : kOb3 + j;
}

__global__ __launch_bounds__(64) void k_closure_train(TrainArgs t, const ClosureNet* __restrict__ net,
                                                      float* __restrict__ partials) {
    __shared__ __bf16 xs[64 * 40];
    __shared__ float H1[64][33], H2[64][33], D1[64][33], D2[64][33], DZ[64][4];
    __shared__ float ACC[kGradPerLane][64];
    const int lane = threadIdx.x;
    const uint32_t nx = t.g.nx, ny = t.g.ny, nz = t.g.nz;
    const uint64_t plane = nodes_of(t.g);   // the batch arrays are unpadded
    const uint64_t tiles_per_pair = plane / 64;
    const uint64_t ntiles = tiles_per_pair * (uint64_t)t.n_pairs;
    for (int q = 0; q < kGradPerLane; ++q) ACC[q][lane] = 0.0f;
    float loss = 0.0f;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t pair = tile / tiles_per_pair;
        const uint64_t node = (tile % tiles_per_pair) * 64 + lane;
        {
            const uint32_t x = node % nx, y = (node / nx) % ny, z = node / ((uint64_t)nx * ny);
            const float* S = t.state + pair * 27 * plane;
            const float* Tg = t.target + pair * 27 * plane;
            const uint32_t xs3[3] = {x + 1 == nx ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
            const uint32_t ys3[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
            const uint32_t zs3[3] = {z + 1 == nz ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
            float h[27];
            static_for<0, 27>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int ex = TP<3>::ex(i), ey = TP<3>::ey(i), ez = TP<3>::ez(i);
                h[i] = S[i * plane + ((uint64_t)zs3[ez + 1] * ny + ys3[ey + 1]) * nx + xs3[ex + 1]];
            });
            tp_raw<3, float>(h);
            const TPMacro<3, float> m = tp_macro_raw<3, float>(h, t.rho0);
            tp_raw_to_central<3, float>(h, m.u);
            float om[8] = {0.f, 0.f, t.omega2, 0.f, 0.f, 0.f, 0.f, 0.f};
            float zz[kNOut];
            {
                MlpTrace tr;
                closure_rates<true>(net, h, m.drho, t.rho0, m.u, xs, om, &tr, zz);
                // pre-activations from accumulator layout to node rows
                const int g = lane >> 4, r = lane & 15;
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            H1[16 * nt + r][16 * mt + 4 * g + j] = tr.a1[mt][nt][j];
                            H2[16 * nt + r][16 * mt + 4 * g + j] = tr.a2[mt][nt][j];
                        }
            }
            float neq[27];
            tp3_noneq(h, m.drho, t.rho0, m.u, neq);
            static_for<0, 27>([&](auto Pc) {
                constexpr int p = decltype(Pc)::value;
                constexpr int order = p % 3 + (p / 3) % 3 + p / 9;
                if constexpr (order >= 2) h[p] -= om[order] * neq[p];
            });
            tp_inverse<3, float>(h, m.u);
            if (t.mode == 0) {
                // residuals and the objective (h now holds f* - w rho0)
                static_for<0, 27>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const float e = h[i] - Tg[i * plane + node];
                    loss += e * e * inv_w27(i) * t.inv_count;
                    h[i] = 2.0f * e * inv_w27(i) * t.inv_count;
                });
            } else {
                // adjoint of f*_i: e_i . D at the node f*_i streams to, y + e_i
                const float* Dp = t.target + pair * 3 * plane;
                const float d0 = Dp[node], d1 = Dp[plane + node], d2 = Dp[2 * plane + node];
                loss += (d0 * d0 + d1 * d1 + d2 * d2) * (0.25f / t.inv_count);
                static_for<0, 27>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    constexpr int ex = TP<3>::ex(i), ey = TP<3>::ey(i), ez = TP<3>::ez(i);
                    // xs3[1 - e] is x + e
                    const uint64_t nb = ((uint64_t)zs3[1 - ez] * ny + ys3[1 - ey]) * nx + xs3[1 - ex];
                    float lam = 0.0f;
                    if constexpr (ex != 0) lam += float(ex) * Dp[nb];
                    if constexpr (ey != 0) lam += float(ey) * Dp[plane + nb];
                    if constexpr (ez != 0) lam += float(ez) * Dp[2 * plane + nb];
                    h[i] = lam;
                });
            }
            // d objective / d omega_n = -sum_{|p| = n} (K^-T r)_p neq_p
            tp3_inverse_adjoint(h, m.u);
            float dom[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            static_for<0, 27>([&](auto Pc) {
                constexpr int p = decltype(Pc)::value;
                constexpr int order = p % 3 + (p / 3) % 3 + p / 9;
                if constexpr (order >= 3) dom[order] -= h[p] * neq[p];
            });
            const bool tied = net->tie_even != 0;
#pragma unroll
            for (int j = 0; j < kNOut; ++j) {
                const float s = sigmoid_f(zz[j]);
                DZ[lane][j] = (tied && (j & 1)) ? 0.0f : dom[3 + j] * 1.45f * s * (1.0f - s);
            }
        }
        __syncthreads();
        // backward through the hidden layers, one node per lane.  The weight
        // gradients use the activations the forward pass fed to the next
        // layer: GELU of the same FP32 pre-activation, rounded to BF16.
        {
            float d2[kNH];
            const float dz0 = DZ[lane][0], dz1 = DZ[lane][1], dz2 = DZ[lane][2], dz3 = DZ[lane][3];
#pragma unroll 8
            for (int k = 0; k < kNH; ++k) {
                const float a2 = H2[lane][k];
                const float s = net->w3f[0][k] * dz0 + net->w3f[1][k] * dz1 + net->w3f[2][k] * dz2 + net->w3f[3][k] * dz3;
                d2[k] = s * gelu_grad_f(a2);
                H2[lane][k] = (float)(__bf16)gelu_f(a2);
                D2[lane][k] = d2[k];
            }
#pragma unroll 2
            for (int k = 0; k < kNH; ++k) {
                float s = 0.0f;
#pragma unroll
                for (int j = 0; j < kNH; ++j) s += net->w2f[j][k] * d2[j];
                const float a1 = H1[lane][k];
                D1[lane][k] = s * gelu_grad_f(a1);
                H1[lane][k] = (float)(__bf16)gelu_f(a1);
            }
        }
        __syncthreads();
        // weight gradients summed over the 64 nodes of the tile
        for (int q = 0; q < kGradPerLane; ++q) {
            int sec, j, mm;
            if (!grad_entry(q, lane, sec, j, mm)) continue;
            float s = 0.0f;
            if (sec == 0) {
                if (mm < kNIn)
                    for (int n = 0; n < 64; ++n) s += D1[n][j] * (float)xs[n * 40 + mm];
                else
                    for (int n = 0; n < 64; ++n) s += D1[n][j];
            } else if (sec == 1) {
                if (mm < kNH)
                    for (int n = 0; n < 64; ++n) s += D2[n][j] * H1[n][mm];
                else
                    for (int n = 0; n < 64; ++n) s += D2[n][j];
            } else {
                if (mm < kNH)
                    for (int n = 0; n < 64; ++n) s += DZ[n][j] * H2[n][mm];
                else
                    for (int n = 0; n < 64; ++n) s += DZ[n][j];
            }
            ACC[q][lane] += s;
        }
        __syncthreads();
    }
    // scatter the lane's entries into the packed parameter order
    float* out = partials + (uint64_t)blockIdx.x * kPartialStride;
    for (int q = 0; q < kGradPerLane; ++q) {
        int sec, j, mm;
        if (grad_entry(q, lane, sec, j, mm)) out[grad_index(sec, j, mm)] = ACC[q][lane];
    }
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
    if (lane == 0) out[kNParam] = loss;
}

// Momentum mismatch two steps ahead: for each pair and node x,
// j2(x) = sum_i e_i f1_i(x - e_i) (f1: the closure step of the state; the
// next collision conserves momentum), jbar(x) = sum_i e_i target_i(x), and
// D = 2 inv_count (j2 - jbar), written [pair][3][nodes].  Deviations carry
// the momenta of the populations (sum_i e_i w_i = 0).
__global__ __launch_bounds__(256) void k_closure_momentum(const float* __restrict__ f1,
                                                          const float* __restrict__ target, GridArgs g,
                                                          int64_t n_pairs, float inv_count, float* __restrict__ D) {
    const uint64_t plane = nodes_of(g);
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= plane * (uint64_t)n_pairs) return;
    const uint64_t pair = id / plane, node = id % plane;
    const uint32_t nx = g.nx, ny = g.ny, nz = g.nz;
    const uint32_t x = node % nx, y = (node / nx) % ny, z = node / ((uint64_t)nx * ny);
    const uint32_t xs3[3] = {x + 1 == nx ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const uint32_t ys3[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const uint32_t zs3[3] = {z + 1 == nz ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
    const float* F = f1 + pair * 27 * plane;
    const float* T = target + pair * 27 * plane;
    float j[3] = {0.0f, 0.0f, 0.0f};
    static_for<0, 27>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = TP<3>::ex(i), ey = TP<3>::ey(i), ez = TP<3>::ez(i);
        const float v = F[i * plane + ((uint64_t)zs3[ez + 1] * ny + ys3[ey + 1]) * nx + xs3[ex + 1]]
                        - T[i * plane + node];
        if constexpr (ex != 0) j[0] += float(ex) * v;
        if constexpr (ey != 0) j[1] += float(ey) * v;
        if constexpr (ez != 0) j[2] += float(ez) * v;
    });
    float* out = D + pair * 3 * plane;
    static_for<0, 3>([&](auto K) {
        constexpr int k = decltype(K)::value;
        out[k * plane + node] = 2.0f * inv_count * j[k];
    });
}

// Sum the per-block partial rows in block order (deterministic).
__global__ __launch_bounds__(256) void k_closure_reduce(const float* __restrict__ partials, int nblocks,
                                                        float* __restrict__ grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kPartialStride) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partials[(uint64_t)b * kPartialStride + e];
    grad[e] = (float)s;
}

// Adam on the FP32 master weights; c1, c2 undo the moments' start-up bias.
// Bit j of `frozen` keeps output j's weights (row j of W3 and b3[j]) and
// their moments unchanged.
__global__ __launch_bounds__(256) void k_closure_adam(float* __restrict__ P, float* __restrict__ m1,
                                                      float* __restrict__ m2, const float* __restrict__ grad,
                                                      float lr, float b1, float b2, float eps, float c1, float c2,
                                                      int frozen) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNParam) return;
    const int out = e >= kOb3 ? e - kOb3 : (e >= kOW3 ? (e - kOW3) / kNH : -1);
    if (out >= 0 && ((frozen >> out) & 1)) return;
    const float g = grad[e];
    const float a = b1 * m1[e] + (1.0f - b1) * g;
    const float b = b2 * m2[e] + (1.0f - b2) * g * g;
    m1[e] = a;
    m2[e] = b;
    P[e] -= lr * (a * c1) / (sqrtf(b * c2) + eps);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
size_t closure_net_bytes() { return sizeof(ClosureNet); }
int closure_partial_stride() { return kPartialStride; }

void launch_closure_pack(const float* P, const float* norm, int tie_even, void* net, hipStream_t s) {
    hipLaunchKernelGGL(k_closure_pack, dim3(1), dim3(256), 0, s, P, norm, tie_even, static_cast<ClosureNet*>(net));
}

void launch_step_closure(const StepArgs& a, const void* net, hipStream_t s) {
    const uint32_t bs = a.g.nx >= 256 ? 256u : ((a.g.nx + 63u) / 64u) * 64u;
    hipLaunchKernelGGL(k_step_closure, dim3(a.g.nchunks * a.g.ny * a.g.nz), dim3(bs), 0, s, a,
                       static_cast<const ClosureNet*>(net));
}

void launch_closure_momentum(const float* f1, const float* target, int64_t n_pairs, const GridArgs& g, float* D,
                             hipStream_t s) {
    const uint64_t n = nodes_of(g) * (uint64_t)n_pairs;
    const float inv_count = (float)(1.0 / (double)n);
    hipLaunchKernelGGL(k_closure_momentum, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, f1, target, g, n_pairs,
                       inv_count, D);
}

void launch_closure_train(const float* state, const float* target, int64_t n_pairs, const GridArgs& g, float rho0,
                          float omega2, const void* net, float* partials, int nblocks, float* grad, int mode,
                          hipStream_t s) {
    TrainArgs t;
    t.state = state;
    t.target = target;
    t.g = g;
    t.n_pairs = n_pairs;
    t.rho0 = rho0;
    t.omega2 = omega2;
    t.inv_count = (float)(1.0 / ((double)n_pairs * (double)nodes_of(g)));
    t.mode = mode;
    hipLaunchKernelGGL(k_closure_train, dim3(nblocks), dim3(64), 0, s, t, static_cast<const ClosureNet*>(net),
                       partials);
    hipLaunchKernelGGL(k_closure_reduce, dim3((kPartialStride + 255) / 256), dim3(256), 0, s, partials, nblocks,
                       grad);
}

void launch_closure_adam(float* P, float* m1, float* m2, const float* grad, float lr, float b1, float b2, float eps,
                         int frozen, int step, hipStream_t s) {
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, step)));
    hipLaunchKernelGGL(k_closure_adam, dim3((kNParam + 255) / 256), dim3(256), 0, s, P, m1, m2, grad, lr, b1, b2, eps,
                       c1, c2, frozen);
}

}  // namespace cmlb
