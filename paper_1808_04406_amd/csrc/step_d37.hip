// Fused pull-stream + collide for the thermal 2D Hermite rules (the
// 37-velocity rules with order-4 truncation, the 17-velocity rules with
// order-3 truncation; central-moment or raw-moment MRT), and its launchers.
// Same thread/block mapping as the tensor-product step: one thread per
// node, one x-segment of a row (up to 512 nodes) per block, block-uniform
// source rows.
#include "launch.hpp"

#include "collide_h2.hpp"

namespace cmlb {

// ---------------------------------------------------------------------------
// Hot path: stream + collide on a 2D Hermite rule
// ---------------------------------------------------------------------------
// PAD: x-rows padded to the pitch (otherwise the row stride is nx).
template <int LAT, int ST, int MODEL, bool PAD>
__device__ __forceinline__ void step_h2_body(const StepArgs& a) {
    using S = Store<ST>;
    using R = typename S::R;
    using T = typename S::T;
    using L = H2<LAT>;
    const uint32_t nx = a.g.nx, ny = a.g.ny;
    const uint32_t blk = xcd_block(a.g.nchunks);
    const uint32_t chunk = blk % a.g.nchunks;
    const uint32_t y = blk / a.g.nchunks;
    const uint32_t x = chunk * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const char* __restrict__ src = static_cast<const char*>(a.src);
    char* __restrict__ dst = static_cast<char*>(a.dst);
    const uint64_t plane_bytes = a.g.plane * sizeof(T);

    R h[L::Q];
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = L::tab.ex[i], ey = L::tab.ey[i];
        const uint32_t ys = wrap_sub(y, ey, ny);                       // block-uniform
        const uint32_t xo = wrap_sub(x, ex, nx) * (uint32_t)sizeof(T);  // lane byte offset
        const char* rowp = src + i * plane_bytes + (uint64_t)ys * (PAD ? a.pitch : nx) * sizeof(T);
        R v = S::load(reinterpret_cast<const T*>(rowp + xo));
        if constexpr (S::kScaled) v *= R(a.inv_s[i]);
        h[i] = v;
    });

    R om[8];
    static_for<0, 8>([&](auto N) { om[decltype(N)::value] = R(a.omega[decltype(N)::value]); });
    R wc[8];
    static_for<0, 8>([&](auto N) { wc[decltype(N)::value] = R(a.wcls[decltype(N)::value]); });
    h2_collide<LAT, MODEL, R>(h, R(a.rho0), om, R(a.r), wc, a.thermal != 0, R(a.theta0));

    char* outrow = dst + (uint64_t)y * (PAD ? a.pitch : nx) * sizeof(T);
    const uint32_t xo = x * (uint32_t)sizeof(T);
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        R v = h[i];
        if constexpr (S::kScaled) v *= R(a.s[i]);
        S::store(reinterpret_cast<T*>(outrow + i * plane_bytes + xo), v);
    });
}

template <int LAT, int ST, int MODEL, bool PAD>
__global__ __launch_bounds__(512) void k_step_h2(StepArgs a) {
    step_h2_body<LAT, ST, MODEL, PAD>(a);
}

// One step of each lattice of a batch (blockIdx.y = lattice); D2Q37.
template <int ST, int MODEL, bool PAD>
__global__ __launch_bounds__(512) void k_step_d37_batch(BatchArgs A) {
    step_h2_body<kD2Q37, ST, MODEL, PAD>(batch_member(A));
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int LAT, int ST, int MODEL>
static void launch_h2(StepArgs a, hipStream_t s) {
    dim3 grid, block;
    step_shape(a, grid, block, a.g.ny, 512);   // FP64 needs up to 142 VGPRs: at most 512 threads
    if (a.pitch != a.g.nx) hipLaunchKernelGGL((k_step_h2<LAT, ST, MODEL, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_step_h2<LAT, ST, MODEL, false>), grid, block, 0, s, a);
}

template <int ST, int MODEL>
static void launch_d37_batch(BatchArgs A, int count, hipStream_t s) {
    dim3 grid, block;
    step_shape(A.a, grid, block, A.a.g.ny, 512);
    grid.y = count;
    if (A.a.pitch != A.a.g.nx) hipLaunchKernelGGL((k_step_d37_batch<ST, MODEL, true>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_step_d37_batch<ST, MODEL, false>), grid, block, 0, s, A);
}

int launch_step_d37_batch(int storage, int model, const BatchArgs& A, int count, hipStream_t s) {
    const bool raw = (model == kRawMRT);
    switch (storage) {
        case kF64: raw ? launch_d37_batch<kF64, kRawMRT>(A, count, s) : launch_d37_batch<kF64, kCM>(A, count, s); return 0;
        case kF32: raw ? launch_d37_batch<kF32, kRawMRT>(A, count, s) : launch_d37_batch<kF32, kCM>(A, count, s); return 0;
        case kBF16: raw ? launch_d37_batch<kBF16, kRawMRT>(A, count, s) : launch_d37_batch<kBF16, kCM>(A, count, s); return 0;
        case kF16: raw ? launch_d37_batch<kF16, kRawMRT>(A, count, s) : launch_d37_batch<kF16, kCM>(A, count, s); return 0;
    }
    return -1;
}

// The other rules of Fig. 2 carry the central-moment model (and regularised
// BGK, which is that kernel with one rate) in FP64 and FP32 storage only, the
// convergence study's configurations.
template <int LAT>
static int launch_rule(int storage, int model, const StepArgs& a, hipStream_t s) {
    if (model == kRawMRT) return -1;
    if (storage == kF64) launch_h2<LAT, kF64, kCM>(a, s);
    else if (storage == kF32) launch_h2<LAT, kF32, kCM>(a, s);
    else return -1;
    return 0;
}

int launch_step_h2(int lattice, int storage, int model, const StepArgs& a, hipStream_t s) {
    if (lattice == kD2Q37) {
        const bool raw = (model == kRawMRT);
        switch (storage) {
            case kF64: raw ? launch_h2<kD2Q37, kF64, kRawMRT>(a, s) : launch_h2<kD2Q37, kF64, kCM>(a, s); return 0;
            case kF32: raw ? launch_h2<kD2Q37, kF32, kRawMRT>(a, s) : launch_h2<kD2Q37, kF32, kCM>(a, s); return 0;
            case kBF16: raw ? launch_h2<kD2Q37, kBF16, kRawMRT>(a, s) : launch_h2<kD2Q37, kBF16, kCM>(a, s); return 0;
            case kF16: raw ? launch_h2<kD2Q37, kF16, kRawMRT>(a, s) : launch_h2<kD2Q37, kF16, kCM>(a, s); return 0;
        }
        return -1;
    }
    switch (lattice) {
        case kE9B: return launch_rule<kE9B>(storage, model, a, s);
        case kE9C: return launch_rule<kE9C>(storage, model, a, s);
        case kE9D: return launch_rule<kE9D>(storage, model, a, s);
        case kE7A: return launch_rule<kE7A>(storage, model, a, s);
        case kE7B: return launch_rule<kE7B>(storage, model, a, s);
        case kE7C: return launch_rule<kE7C>(storage, model, a, s);
        case kE7D: return launch_rule<kE7D>(storage, model, a, s);
    }
    return -1;
}

}  // namespace cmlb
