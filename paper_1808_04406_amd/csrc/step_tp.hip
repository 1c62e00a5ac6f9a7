// Fused pull-stream + collide for the tensor-product lattices D2Q9 and
// D3Q27 (the hot path), and its launcher.
//
// One thread per node; a block covers one contiguous x-segment of a row (the
// whole row up to 1024 nodes), so the y/z neighbour rows of every population
// are block-uniform addresses and each wavefront reads and writes 27 (9)
// contiguous runs of the structure-of-arrays field F[i][z][y][x].  Two buffers alternate (pull from
// one, write the other), so reads and writes never alias.
#include "launch.hpp"

#include "collide_tp.hpp"

namespace cmlb {

// ---------------------------------------------------------------------------
// Hot path: D2Q9 / D3Q27 stream + collide
// ---------------------------------------------------------------------------
// PAD: x-rows padded to the pitch (otherwise the row stride is nx, which
// keeps one scalar register free in the common, unpadded case).
template <int D, int ST, bool PAD>
__device__ __forceinline__ void step_tp_body(const StepArgs& a) {
    using S = Store<ST>;
    using R = typename S::R;
    using T = typename S::T;
    constexpr int Q = TP<D>::Q;
    const uint32_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const uint32_t pitch = PAD ? a.pitch : nx;
    const uint32_t blk = xcd_block(a.g.nchunks);
    const uint32_t chunk = blk % a.g.nchunks;
    const uint32_t row = blk / a.g.nchunks;
    const uint32_t x = chunk * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const uint32_t y = row % ny, z = row / ny;
    // Row bases are block-uniform (scalar registers); lanes add a 32-bit byte
    // offset, which maps onto the saddr + voffset form of global loads/stores.
    const char* __restrict__ src = static_cast<const char*>(a.src);
    char* __restrict__ dst = static_cast<char*>(a.dst);
    const uint64_t plane_bytes = a.g.plane * sizeof(T);
    const uint32_t xoff[3] = {wrap_inc(x, nx) * (uint32_t)sizeof(T), x * (uint32_t)sizeof(T),
                              wrap_dec(x, nx) * (uint32_t)sizeof(T)};  // x - e for e = -1, 0, +1
    const uint32_t ysrc[3] = {wrap_inc(y, ny), y, wrap_dec(y, ny)};
    const uint32_t zsrc[3] = {D == 3 ? wrap_inc(z, nz) : 0u, z, D == 3 ? wrap_dec(z, nz) : 0u};

    R h[Q];
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = TP<D>::ex(i), ey = TP<D>::ey(i), ez = TP<D>::ez(i);
        const char* rowp = src + i * plane_bytes + ((uint64_t)zsrc[ez + 1] * ny + ysrc[ey + 1]) * pitch * sizeof(T);
        R v = S::load(reinterpret_cast<const T*>(rowp + xoff[ex + 1]));
        if constexpr (S::kScaled) v *= R(a.inv_s[i]);
        h[i] = v;
    });

    R om[8];
    static_for<0, 8>([&](auto N) { om[decltype(N)::value] = R(a.omega[decltype(N)::value]); });
    tp_collide<D, R>(h, R(a.rho0), om);

    char* outrow = dst + ((uint64_t)z * ny + y) * pitch * sizeof(T);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        R v = h[i];
        if constexpr (S::kScaled) v *= R(a.s[i]);
        S::store(reinterpret_cast<T*>(outrow + i * plane_bytes + xoff[1]), v);
    });
}

template <int D, int ST, bool PAD>
__global__ __launch_bounds__(1024) void k_step_tp(StepArgs a) {
    step_tp_body<D, ST, PAD>(a);
}

// One step of each lattice of a batch (blockIdx.y = lattice).
template <int D, int ST, bool PAD>
__global__ __launch_bounds__(1024) void k_step_tp_batch(BatchArgs A) {
    step_tp_body<D, ST, PAD>(batch_member(A));
}

// ---------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------
template <int D, int ST>
static void launch_tp(StepArgs a, hipStream_t s) {
    dim3 grid, block;
    step_shape(a, grid, block, a.g.ny * a.g.nz, 1024);
    if (a.pitch != a.g.nx) hipLaunchKernelGGL((k_step_tp<D, ST, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_step_tp<D, ST, false>), grid, block, 0, s, a);
}

template <int D, int ST>
static void launch_tp_batch(BatchArgs A, int count, hipStream_t s) {
    dim3 grid, block;
    step_shape(A.a, grid, block, A.a.g.ny * A.a.g.nz, 1024);
    grid.y = count;
    if (A.a.pitch != A.a.g.nx) hipLaunchKernelGGL((k_step_tp_batch<D, ST, true>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_step_tp_batch<D, ST, false>), grid, block, 0, s, A);
}

int launch_step_tp_batch(int lattice, int storage, const BatchArgs& A, int count, hipStream_t s) {
    const int D = lattice == kD2Q9 ? 2 : 3;
#define CMLB_TPB(DD)                                                         \
    switch (storage) {                                                       \
        case kF64: launch_tp_batch<DD, kF64>(A, count, s); return 0;         \
        case kF32: launch_tp_batch<DD, kF32>(A, count, s); return 0;         \
        case kBF16: launch_tp_batch<DD, kBF16>(A, count, s); return 0;       \
        case kF16: launch_tp_batch<DD, kF16>(A, count, s); return 0;         \
    }                                                                        \
    return -1;
    if (D == 2) { CMLB_TPB(2) }
    CMLB_TPB(3)
#undef CMLB_TPB
}

int launch_step_tp(int lattice, int storage, const StepArgs& a, hipStream_t s) {
    const int D = lattice == kD2Q9 ? 2 : 3;
#define CMLB_TP(DD)                                                  \
    switch (storage) {                                               \
        case kF64: launch_tp<DD, kF64>(a, s); return 0;              \
        case kF32: launch_tp<DD, kF32>(a, s); return 0;              \
        case kBF16: launch_tp<DD, kBF16>(a, s); return 0;            \
        case kF16: launch_tp<DD, kF16>(a, s); return 0;              \
    }                                                                \
    return -1;
    if (D == 2) { CMLB_TP(2) }
    CMLB_TP(3)
#undef CMLB_TP
}

}  // namespace cmlb
