// Fused pull-stream + collide for the thermal D2Q37 lattice (order-4
// Hermite truncation; central-moment or raw-moment MRT), and its launcher.
// Same thread/block mapping as the tensor-product step: one thread per
// node, one x-segment of a row (up to 512 nodes) per block, block-uniform
// source rows.
#include "launch.hpp"

#include "collide_d2q37.hpp"

namespace cmlb {

// ---------------------------------------------------------------------------
// Hot path: D2Q37 stream + collide (order-4 Hermite truncation)
// ---------------------------------------------------------------------------
// PAD: x-rows padded to the pitch (otherwise the row stride is nx).
template <int ST, int MODEL, bool PAD>
__device__ __forceinline__ void step_d37_body(const StepArgs& a) {
    using S = Store<ST>;
    using R = typename S::R;
    using T = typename S::T;
    const uint32_t nx = a.g.nx, ny = a.g.ny;
    const uint32_t blk = xcd_block(a.g.nchunks);
    const uint32_t chunk = blk % a.g.nchunks;
    const uint32_t y = blk / a.g.nchunks;
    const uint32_t x = chunk * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const char* __restrict__ src = static_cast<const char*>(a.src);
    char* __restrict__ dst = static_cast<char*>(a.dst);
    const uint64_t plane_bytes = a.g.plane * sizeof(T);

    R h[37];
    static_for<0, 37>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = kTab37.ex[i], ey = kTab37.ey[i];
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
    d37_collide<MODEL, R>(h, R(a.rho0), om, R(a.r), wc, a.thermal != 0, R(a.theta0));

    char* outrow = dst + (uint64_t)y * (PAD ? a.pitch : nx) * sizeof(T);
    const uint32_t xo = x * (uint32_t)sizeof(T);
    static_for<0, 37>([&](auto I) {
        constexpr int i = decltype(I)::value;
        R v = h[i];
        if constexpr (S::kScaled) v *= R(a.s[i]);
        S::store(reinterpret_cast<T*>(outrow + i * plane_bytes + xo), v);
    });
}

template <int ST, int MODEL, bool PAD>
__global__ __launch_bounds__(512) void k_step_d37(StepArgs a) {
    step_d37_body<ST, MODEL, PAD>(a);
}

// One step of each lattice of a batch (blockIdx.y = lattice).
template <int ST, int MODEL, bool PAD>
__global__ __launch_bounds__(512) void k_step_d37_batch(BatchArgs A) {
    step_d37_body<ST, MODEL, PAD>(batch_member(A));
}

// ---------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------
template <int ST, int MODEL>
static void launch_d37(StepArgs a, hipStream_t s) {
    dim3 grid, block;
    step_shape(a, grid, block, a.g.ny, 512);   // FP64 needs up to 142 VGPRs: at most 512 threads
    if (a.pitch != a.g.nx) hipLaunchKernelGGL((k_step_d37<ST, MODEL, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_step_d37<ST, MODEL, false>), grid, block, 0, s, a);
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

int launch_step_d37(int storage, int model, const StepArgs& a, hipStream_t s) {
    const bool raw = (model == kRawMRT);
    switch (storage) {
        case kF64: raw ? launch_d37<kF64, kRawMRT>(a, s) : launch_d37<kF64, kCM>(a, s); return 0;
        case kF32: raw ? launch_d37<kF32, kRawMRT>(a, s) : launch_d37<kF32, kCM>(a, s); return 0;
        case kBF16: raw ? launch_d37<kBF16, kRawMRT>(a, s) : launch_d37<kBF16, kCM>(a, s); return 0;
        case kF16: raw ? launch_d37<kF16, kRawMRT>(a, s) : launch_d37<kF16, kCM>(a, s); return 0;
    }
    return -1;
}

}  // namespace cmlb
