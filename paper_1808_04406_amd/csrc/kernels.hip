// HIP kernels of the cmlb library (gfx950) other than the step kernels
// (step_tp.hip, step_d37.hip, kernels_closure.hip), and their launchers.
//
//  k_init_*                 state <- discrete equilibrium of given fields
//  k_moments                rho, u, theta readout (FP64)
//  k_decode / k_encode      full FP64 populations <-> storage
//  k_reduce_*               deterministic FP64 global diagnostics
//
// Layout: populations are structure-of-arrays F[i][z][y][x], x fastest, in
// the storage type.
#include "launch.hpp"

#include "collide_h2.hpp"
#include "collide_tp.hpp"

namespace cmlb {

// ---------------------------------------------------------------------------
// Initialisation from fields (FP64 arithmetic, then encode)
// ---------------------------------------------------------------------------
template <int D, int ST>
__global__ __launch_bounds__(256) void k_init_tp(StepArgs a, FieldArgs fa) {
    using S = Store<ST>;
    using T = typename S::T;
    constexpr int Q = TP<D>::Q;
    T* dst = static_cast<T*>(a.dst);
    for (uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; n < nodes_of(a.g);
         n += (uint64_t)gridDim.x * blockDim.x) {
        double u[3] = {fa.u[n], fa.u[nodes_of(a.g) + n], D == 3 ? fa.u[2 * nodes_of(a.g) + n] : 0.0};
        double h[Q];
        tp_equilibrium<D, double>(h, fa.rho[n] - a.rho0, a.rho0, u);
        const uint64_t off = node_offset(a.g.nx, a.pitch, n);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            dst[(uint64_t)i * a.g.plane + off] = S::from_double(h[i] * (double)a.s[i]);
        });
    }
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_init_h2(StepArgs a, FieldArgs fa) {
    using S = Store<ST>;
    using T = typename S::T;
    constexpr int Q = H2<LAT>::Q;
    T* dst = static_cast<T*>(a.dst);
    double wc[8];
    for (int k = 0; k < 8; ++k) wc[k] = a.wcls[k];
    for (uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; n < nodes_of(a.g);
         n += (uint64_t)gridDim.x * blockDim.x) {
        const double th = fa.theta ? fa.theta[n] : a.theta0;
        double h[Q];
        const uint64_t off = node_offset(a.g.nx, a.pitch, n);
        h2_equilibrium<LAT, double>(h, fa.rho[n] - a.rho0, a.rho0, a.r * fa.u[n], a.r * fa.u[nodes_of(a.g) + n],
                                    th - 1.0, a.r, wc);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            dst[(uint64_t)i * a.g.plane + off] = S::from_double(h[i] * (double)a.s[i]);
        });
    }
}

// ---------------------------------------------------------------------------
// Readout, codecs
// ---------------------------------------------------------------------------
template <int LAT>
struct LatInfo {   // the 2D Hermite rules
    static constexpr int D = 2, Q = H2<LAT>::Q;
    static constexpr int ex(int i) { return H2<LAT>::tab.ex[i]; }
    static constexpr int ey(int i) { return H2<LAT>::tab.ey[i]; }
    static constexpr int ez(int) { return 0; }
};
template <>
struct LatInfo<kD2Q9> {
    static constexpr int D = 2, Q = 9;
    static constexpr int ex(int i) { return TP<2>::ex(i); }
    static constexpr int ey(int i) { return TP<2>::ey(i); }
    static constexpr int ez(int) { return 0; }
};
template <>
struct LatInfo<kD3Q27> {
    static constexpr int D = 3, Q = 27;
    static constexpr int ex(int i) { return TP<3>::ex(i); }
    static constexpr int ey(int i) { return TP<3>::ey(i); }
    static constexpr int ez(int i) { return TP<3>::ez(i); }
};

// Sums of one node's deviation populations (FP64): sum h, sum h e, sum h |e|^2.
template <int LAT, int ST>
__device__ __forceinline__ void node_sums(const typename Store<ST>::T* src, uint64_t plane, uint64_t n,
                                          const float* inv_s, double& s0, double (&j)[3], double& e2,
                                          int& nonfinite) {
    using S = Store<ST>;
    using L = LatInfo<LAT>;
    s0 = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    e2 = 0.0;
    nonfinite = 0;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        double v = S::to_double(src[(uint64_t)i * plane + n]);
        if constexpr (S::kScaled) v *= (double)inv_s[i];
        nonfinite += (v - v != 0.0) ? 1 : 0;
        s0 += v;
        j[0] += L::ex(i) * v;
        j[1] += L::ey(i) * v;
        j[2] += L::ez(i) * v;
        e2 += (L::ex(i) * L::ex(i) + L::ey(i) * L::ey(i) + L::ez(i) * L::ez(i)) * v;
    });
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_moments(StepArgs a, FieldArgs fa) {
    using L = LatInfo<LAT>;
    using T = typename Store<ST>::T;
    const T* src = static_cast<const T*>(a.src);
    const double r2 = a.r * a.r;
    // sum_i w_i |e_i|^2 = D / r^2 (second moment of the quadrature)
    const double w_e2 = L::D / r2;
    for (uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; n < nodes_of(a.g);
         n += (uint64_t)gridDim.x * blockDim.x) {
        double s0, j[3], e2;
        int nf;
        node_sums<LAT, ST>(src, a.g.plane, node_offset(a.g.nx, a.pitch, n), a.inv_s, s0, j, e2, nf);
        const double rho = a.rho0 + s0;
        const double ux = j[0] / rho, uy = j[1] / rho, uz = j[2] / rho;
        if (fa.out_rho) fa.out_rho[n] = rho;
        if (fa.out_u) {
            fa.out_u[n] = ux;
            fa.out_u[nodes_of(a.g) + n] = uy;
            if (L::D == 3) fa.out_u[2 * nodes_of(a.g) + n] = uz;
        }
        if (fa.out_theta) {
            // rho (|u|^2 + D theta) = sum f |xi|^2, xi = r e
            const double uu = ux * ux + uy * uy + uz * uz;
            fa.out_theta[n] = r2 * ((e2 + a.rho0 * w_e2) / rho - uu) / L::D;
        }
    }
}

struct CodecArgs {
    void* stor;         // the state: [Q][plane], rows padded to the pitch
    double* full;       // [Q][node], unpadded
    const float* dev;   // [Q][node], unpadded FP32 deviations f - w rho0 (k_encode_dev)
    GridArgs g;
    uint32_t pitch;
    uint64_t plane;     // nodes (the loop bound of the codecs)
    double rho0;
    double w[37];
    float s[37];
    float inv_s[37];
};

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_decode(CodecArgs c) {
    using S = Store<ST>;
    using T = typename S::T;
    const T* src = static_cast<const T*>(c.stor);
    for (uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; n < c.plane;
         n += (uint64_t)gridDim.x * blockDim.x) {
        static_for<0, LatInfo<LAT>::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            double v = S::to_double(src[(uint64_t)i * c.g.plane + node_offset(c.g.nx, c.pitch, n)]);
            if constexpr (S::kScaled) v *= (double)c.inv_s[i];
            c.full[(uint64_t)i * c.plane + n] = v + c.w[i] * c.rho0;
        });
    }
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_encode(CodecArgs c) {
    using S = Store<ST>;
    using T = typename S::T;
    T* dst = static_cast<T*>(c.stor);
    for (uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; n < c.plane;
         n += (uint64_t)gridDim.x * blockDim.x) {
        static_for<0, LatInfo<LAT>::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double v = (c.full[(uint64_t)i * c.plane + n] - c.w[i] * c.rho0) * (double)c.s[i];
            dst[(uint64_t)i * c.g.plane + node_offset(c.g.nx, c.pitch, n)] = S::from_double(v);
        });
    }
}

// Encode unpadded FP32 deviations (the box filter's output layout) into the
// state's storage type and layout.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_encode_dev(CodecArgs c) {
    using S = Store<ST>;
    using T = typename S::T;
    T* dst = static_cast<T*>(c.stor);
    for (uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; n < c.plane;
         n += (uint64_t)gridDim.x * blockDim.x) {
        static_for<0, LatInfo<LAT>::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double v = (double)c.dev[(uint64_t)i * c.plane + n] * (double)c.s[i];
            dst[(uint64_t)i * c.g.plane + node_offset(c.g.nx, c.pitch, n)] = S::from_double(v);
        });
    }
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions
// ---------------------------------------------------------------------------
// Values 0..7 are sums (drho, jx, jy, jz, e2, ke, enstrophy, nonfinite);
// values 8..10 are maxima (-drho, drho, |u|^2), so the smallest and largest
// density and the largest speed come out of the same passes.  fmax ignores
// NaN: non-finite nodes are counted by value 7 instead.
constexpr int kRedSums = 8;
static_assert(kRedVals == 11, "eight sums and three maxima");

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void reset_acc(double (&acc)[kRedVals]) {
    for (int k = 0; k < kRedVals; ++k) acc[k] = k < kRedSums ? 0.0 : -HUGE_VAL;
}

// Block reduction of kRedVals values; thread k < kRedVals writes value k of
// the block's partial row.
__device__ __forceinline__ void block_partials(double (&v)[kRedVals], double* partials) {
    __shared__ double lds[4][kRedVals];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < kRedVals; ++k) v[k] = k < kRedSums ? wave_sum(v[k]) : wave_max(v[k]);
    if (lane == 0)
        for (int k = 0; k < kRedVals; ++k) lds[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < kRedVals) {
        const int k = threadIdx.x;
        double s = k < kRedSums ? 0.0 : -HUGE_VAL;
        const int nw = blockDim.x >> 6;
        for (int w = 0; w < nw; ++w) s = k < kRedSums ? s + lds[w][k] : fmax(s, lds[w][k]);
        partials[(uint64_t)blockIdx.x * kRedVals + k] = s;
    }
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_reduce_nodes(StepArgs a, double* uf, double* partials) {
    using T = typename Store<ST>::T;
    const T* src = static_cast<const T*>(a.src);
    double acc[kRedVals];
    reset_acc(acc);
    for (uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; n < nodes_of(a.g);
         n += (uint64_t)gridDim.x * blockDim.x) {
        double s0, j[3], e2;
        int nf;
        node_sums<LAT, ST>(src, a.g.plane, node_offset(a.g.nx, a.pitch, n), a.inv_s, s0, j, e2, nf);
        const double rho = a.rho0 + s0;
        const double ux = j[0] / rho, uy = j[1] / rho, uz = j[2] / rho;
        acc[0] += s0;
        acc[1] += j[0];
        acc[2] += j[1];
        acc[3] += j[2];
        acc[4] += e2;
        const double uu = ux * ux + uy * uy + uz * uz;
        acc[5] += 0.5 * rho * uu;
        acc[7] += nf;
        acc[8] = fmax(acc[8], -s0);
        acc[9] = fmax(acc[9], s0);
        acc[10] = fmax(acc[10], uu);
        uf[n] = ux;
        uf[nodes_of(a.g) + n] = uy;
        uf[2 * nodes_of(a.g) + n] = uz;
    }
    block_partials(acc, partials);
}

// Enstrophy 1/2 |curl u|^2 with second-order central differences (periodic).
__global__ __launch_bounds__(256) void k_reduce_vort(GridArgs g, int D, const double* uf, double* partials) {
    double acc[kRedVals];
    reset_acc(acc);
    const uint64_t P = nodes_of(g);   // uf is unpadded
    for (uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; n < P;
         n += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = n % g.nx, y = (n / g.nx) % g.ny, z = n / ((uint64_t)g.nx * g.ny);
        auto at = [&](int c, uint32_t xx, uint32_t yy, uint32_t zz) {
            return uf[(uint64_t)c * P + ((uint64_t)zz * g.ny + yy) * g.nx + xx];
        };
        const uint32_t xp = x + 1 == g.nx ? 0 : x + 1, xm = x == 0 ? g.nx - 1 : x - 1;
        const uint32_t yp = y + 1 == g.ny ? 0 : y + 1, ym = y == 0 ? g.ny - 1 : y - 1;
        // d/dx of component c
        const double dvy_dx = 0.5 * (at(1, xp, y, z) - at(1, xm, y, z));
        const double dvx_dy = 0.5 * (at(0, x, yp, z) - at(0, x, ym, z));
        double w2 = (dvy_dx - dvx_dy) * (dvy_dx - dvx_dy);
        if (D == 3) {
            const uint32_t zp = z + 1 == g.nz ? 0 : z + 1, zm = z == 0 ? g.nz - 1 : z - 1;
            const double dvz_dy = 0.5 * (at(2, x, yp, z) - at(2, x, ym, z));
            const double dvy_dz = 0.5 * (at(1, x, y, zp) - at(1, x, y, zm));
            const double dvx_dz = 0.5 * (at(0, x, y, zp) - at(0, x, y, zm));
            const double dvz_dx = 0.5 * (at(2, xp, y, z) - at(2, xm, y, z));
            w2 += (dvz_dy - dvy_dz) * (dvz_dy - dvy_dz) + (dvx_dz - dvz_dx) * (dvx_dz - dvz_dx);
        }
        acc[6] += 0.5 * w2;
    }
    block_partials(acc, partials);
}

// Sum the partial rows of both passes in a fixed order: wave k sums value k,
// lane l takes rows l, l + 64, ... in order, then a fixed shuffle tree.
__global__ __launch_bounds__(64 * kRedVals) void k_reduce_final(const double* p1, const double* p2, int nblocks,
                                                                double* out) {
    const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double* p = (k == 6) ? p2 : p1;
    if (k < kRedSums) {
        double s = 0.0;
        for (int b = lane; b < nblocks; b += 64) s += p[(uint64_t)b * kRedVals + k];
        s = wave_sum(s);
        if (lane == 0) out[k] = s;
    } else {
        double m = -HUGE_VAL;
        for (int b = lane; b < nblocks; b += 64) m = fmax(m, p[(uint64_t)b * kRedVals + k]);
        m = wave_max(m);
        if (lane == 0) out[k] = m;
    }
}

// ---------------------------------------------------------------------------
// Box filter (coarse-graining) of a D3Q27 state: the mean of the deviations
// over factor^3 blocks, written as FP32 deviations on the coarse grid.
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(256) void k_box_filter(StepArgs a, int factor, float* __restrict__ dst) {
    using S = Store<ST>;
    using T = typename S::T;
    const T* src = static_cast<const T*>(a.src);
    const uint32_t cx = a.g.nx / factor, cy = a.g.ny / factor, cz = a.g.nz / factor;
    const uint64_t cplane = (uint64_t)cx * cy * cz;
    const double inv = 1.0 / ((double)factor * factor * factor);
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < cplane * 27;
         c += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = c / cplane;
        const uint64_t cn = c % cplane;
        const uint32_t X = cn % cx, Y = (cn / cx) % cy, Z = cn / ((uint64_t)cx * cy);
        double sum = 0.0;
        for (int dz = 0; dz < factor; ++dz)
            for (int dy = 0; dy < factor; ++dy) {
                const uint64_t rowb = (uint64_t)i * a.g.plane +
                                      (((uint64_t)(Z * factor + dz) * a.g.ny + (Y * factor + dy)) * a.pitch) +
                                      X * factor;
                for (int dx = 0; dx < factor; ++dx) sum += S::to_double(src[rowb + dx]);
            }
        double v = sum * inv;
        if constexpr (S::kScaled) v *= (double)a.inv_s[i];
        dst[c] = (float)v;
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
GridArgs make_grid(uint32_t nx, uint32_t ny, uint32_t nz, uint64_t plane) {
    GridArgs g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    uint32_t bs = nx >= 256 ? 256u : ((nx + 63u) / 64u) * 64u;
    g.nchunks = (nx + bs - 1) / bs;
    g.plane = plane;
    return g;
}

static dim3 flat_grid(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3((uint32_t)b);
}

int launch_step2(int lattice, int storage, int model, const StepArgs& a, int mode, hipStream_t s) {
    if (lattice == kD2Q37) return launch_step2_d37(storage, model, a, mode, s);
    if (lattice == kD2Q9 || lattice == kD3Q27) return launch_step2_tp(lattice, storage, a, mode != kFuseAuto, s);
    return -1;
}

int launch_step(int lattice, int storage, int model, const StepArgs& a, hipStream_t s) {
    if (lattice == kD2Q9 || lattice == kD3Q27) return launch_step_tp(lattice, storage, a, s);
    if (lattice >= kD2Q37 && lattice < kNumLattices) return launch_step_h2(lattice, storage, model, a, s);
    return -1;
}

int launch_step_batch(int lattice, int storage, int model, const BatchArgs& A, int count, hipStream_t s) {
    if (count < 1 || count > kMaxBatch) return -1;
    if (lattice == kD2Q9 || lattice == kD3Q27) return launch_step_tp_batch(lattice, storage, A, count, s);
    if (lattice == kD2Q37) return launch_step_d37_batch(storage, model, A, count, s);
    return -1;
}

// The other 2D rules: FP64 and FP32 storage.
template <int ST>
static int launch_init_rule(int lattice, const StepArgs& a, const FieldArgs& f, hipStream_t s) {
    if constexpr (ST != kF64 && ST != kF32) {
        return -1;
    } else {
        dim3 grid = flat_grid(nodes_of(a.g)), block(256);
        switch (lattice) {
            case kE9B: hipLaunchKernelGGL((k_init_h2<kE9B, ST>), grid, block, 0, s, a, f); return 0;
            case kE9C: hipLaunchKernelGGL((k_init_h2<kE9C, ST>), grid, block, 0, s, a, f); return 0;
            case kE9D: hipLaunchKernelGGL((k_init_h2<kE9D, ST>), grid, block, 0, s, a, f); return 0;
            case kE7A: hipLaunchKernelGGL((k_init_h2<kE7A, ST>), grid, block, 0, s, a, f); return 0;
            case kE7B: hipLaunchKernelGGL((k_init_h2<kE7B, ST>), grid, block, 0, s, a, f); return 0;
            case kE7C: hipLaunchKernelGGL((k_init_h2<kE7C, ST>), grid, block, 0, s, a, f); return 0;
            case kE7D: hipLaunchKernelGGL((k_init_h2<kE7D, ST>), grid, block, 0, s, a, f); return 0;
        }
        return -1;
    }
}

template <int ST>
static int launch_init_st(int lattice, const StepArgs& a, const FieldArgs& f, hipStream_t s) {
    dim3 grid = flat_grid(nodes_of(a.g)), block(256);
    if (lattice == kD2Q9) hipLaunchKernelGGL((k_init_tp<2, ST>), grid, block, 0, s, a, f);
    else if (lattice == kD3Q27) hipLaunchKernelGGL((k_init_tp<3, ST>), grid, block, 0, s, a, f);
    else if (lattice == kD2Q37) hipLaunchKernelGGL((k_init_h2<kD2Q37, ST>), grid, block, 0, s, a, f);
    else return launch_init_rule<ST>(lattice, a, f, s);
    return 0;
}

int launch_init(int lattice, int storage, const StepArgs& a, const FieldArgs& f, hipStream_t s) {
    switch (storage) {
        case kF64: return launch_init_st<kF64>(lattice, a, f, s);
        case kF32: return launch_init_st<kF32>(lattice, a, f, s);
        case kBF16: return launch_init_st<kBF16>(lattice, a, f, s);
        case kF16: return launch_init_st<kF16>(lattice, a, f, s);
    }
    return -1;
}

#define CMLB_DISPATCH(LAUNCH)                                                     \
    switch (lattice * 4 + storage) {                                              \
        case kD2Q9 * 4 + kF64: LAUNCH(kD2Q9, kF64); break;                        \
        case kD2Q9 * 4 + kF32: LAUNCH(kD2Q9, kF32); break;                        \
        case kD2Q9 * 4 + kBF16: LAUNCH(kD2Q9, kBF16); break;                      \
        case kD2Q9 * 4 + kF16: LAUNCH(kD2Q9, kF16); break;                        \
        case kD3Q27 * 4 + kF64: LAUNCH(kD3Q27, kF64); break;                      \
        case kD3Q27 * 4 + kF32: LAUNCH(kD3Q27, kF32); break;                      \
        case kD3Q27 * 4 + kBF16: LAUNCH(kD3Q27, kBF16); break;                    \
        case kD3Q27 * 4 + kF16: LAUNCH(kD3Q27, kF16); break;                      \
        case kD2Q37 * 4 + kF64: LAUNCH(kD2Q37, kF64); break;                      \
        case kD2Q37 * 4 + kF32: LAUNCH(kD2Q37, kF32); break;                      \
        case kD2Q37 * 4 + kBF16: LAUNCH(kD2Q37, kBF16); break;                    \
        case kD2Q37 * 4 + kF16: LAUNCH(kD2Q37, kF16); break;                      \
        case kE9B * 4 + kF64: LAUNCH(kE9B, kF64); break;                          \
        case kE9B * 4 + kF32: LAUNCH(kE9B, kF32); break;                          \
        case kE9C * 4 + kF64: LAUNCH(kE9C, kF64); break;                          \
        case kE9C * 4 + kF32: LAUNCH(kE9C, kF32); break;                          \
        case kE9D * 4 + kF64: LAUNCH(kE9D, kF64); break;                          \
        case kE9D * 4 + kF32: LAUNCH(kE9D, kF32); break;                          \
        case kE7A * 4 + kF64: LAUNCH(kE7A, kF64); break;                          \
        case kE7A * 4 + kF32: LAUNCH(kE7A, kF32); break;                          \
        case kE7B * 4 + kF64: LAUNCH(kE7B, kF64); break;                          \
        case kE7B * 4 + kF32: LAUNCH(kE7B, kF32); break;                          \
        case kE7C * 4 + kF64: LAUNCH(kE7C, kF64); break;                          \
        case kE7C * 4 + kF32: LAUNCH(kE7C, kF32); break;                          \
        case kE7D * 4 + kF64: LAUNCH(kE7D, kF64); break;                          \
        case kE7D * 4 + kF32: LAUNCH(kE7D, kF32); break;                          \
        default: return -1;                                                       \
    }

int launch_moments(int lattice, int storage, const StepArgs& a, const FieldArgs& f, hipStream_t s) {
    dim3 grid = flat_grid(nodes_of(a.g)), block(256);
#define L_MOM(L, S) hipLaunchKernelGGL((k_moments<L, S>), grid, block, 0, s, a, f)
    CMLB_DISPATCH(L_MOM)
#undef L_MOM
    return 0;
}

int launch_codec(int lattice, int storage, bool decode, void* stor, double* full, const StepArgs& a,
                 const double* w, hipStream_t s) {
    CodecArgs c;
    c.stor = stor;
    c.full = full;
    c.dev = nullptr;
    c.g = a.g;
    c.pitch = a.pitch;
    c.plane = nodes_of(a.g);
    c.rho0 = a.rho0;
    for (int i = 0; i < 37; ++i) {
        c.w[i] = w[i];
        c.s[i] = a.s[i];
        c.inv_s[i] = a.inv_s[i];
    }
    dim3 grid = flat_grid(nodes_of(a.g)), block(256);
#define L_DEC(L, S) hipLaunchKernelGGL((k_decode<L, S>), grid, block, 0, s, c)
#define L_ENC(L, S) hipLaunchKernelGGL((k_encode<L, S>), grid, block, 0, s, c)
    if (decode) {
        CMLB_DISPATCH(L_DEC)
    } else {
        CMLB_DISPATCH(L_ENC)
    }
#undef L_DEC
#undef L_ENC
    return 0;
}

int launch_encode_deviations(int lattice, int storage, void* stor, const float* dev, const StepArgs& a,
                             hipStream_t s) {
    CodecArgs c;
    c.stor = stor;
    c.full = nullptr;
    c.dev = dev;
    c.g = a.g;
    c.pitch = a.pitch;
    c.plane = nodes_of(a.g);
    c.rho0 = a.rho0;
    for (int i = 0; i < 37; ++i) {
        c.w[i] = 0.0;
        c.s[i] = a.s[i];
        c.inv_s[i] = a.inv_s[i];
    }
    dim3 grid = flat_grid(nodes_of(a.g)), block(256);
#define L_ENCD(L, S) hipLaunchKernelGGL((k_encode_dev<L, S>), grid, block, 0, s, c)
    CMLB_DISPATCH(L_ENCD)
#undef L_ENCD
    return 0;
}

int reduce_blocks(uint64_t plane) { return (int)flat_grid(plane).x; }

int launch_box_filter(int storage, const StepArgs& a, int factor, float* dst, hipStream_t s) {
    const uint64_t coarse = (uint64_t)(a.g.nx / factor) * (a.g.ny / factor) * (a.g.nz / factor) * 27;
    dim3 grid = flat_grid(coarse), block(256);
    switch (storage) {
        case kF64: hipLaunchKernelGGL((k_box_filter<kF64>), grid, block, 0, s, a, factor, dst); return 0;
        case kF32: hipLaunchKernelGGL((k_box_filter<kF32>), grid, block, 0, s, a, factor, dst); return 0;
        case kBF16: hipLaunchKernelGGL((k_box_filter<kBF16>), grid, block, 0, s, a, factor, dst); return 0;
        case kF16: hipLaunchKernelGGL((k_box_filter<kF16>), grid, block, 0, s, a, factor, dst); return 0;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Streaming copy, the achievable-bandwidth reference of the step kernels:
// P planes of `plane` FP32 values, one element of every plane per thread, as
// the step reads and writes its P = Q population planes.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_stream_copy(const float* __restrict__ src, float* __restrict__ dst,
                                                     uint64_t plane) {
    const uint64_t n = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (n >= plane) return;
    float v[P];   // all loads in flight before the first store, as in the step
    static_for<0, P>([&](auto I) { v[decltype(I)::value] = src[(uint64_t)decltype(I)::value * plane + n]; });
    static_for<0, P>([&](auto I) {
        constexpr int p = decltype(I)::value;
        __builtin_nontemporal_store(v[p], dst + (uint64_t)p * plane + n);
    });
}

// One plane: 16-byte accesses, four per thread (the best a plain copy does).
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy_wide(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                          uint64_t n4) {
    const uint64_t base = (blockIdx.x * (uint64_t)blockDim.x) * 4 + threadIdx.x;
    v4f v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t i = base + (uint64_t)k * blockDim.x;
        if (i < n4) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t i = base + (uint64_t)k * blockDim.x;
        if (i < n4) __builtin_nontemporal_store(v[k], dst + i);
    }
}

int launch_stream_copy(int planes, const float* src, float* dst, uint64_t plane, hipStream_t s) {
    if (planes == 1) {
        const uint64_t n4 = plane / 4;   // whole 16-byte groups
        const uint64_t blocks = (n4 + 1023) / 1024;
        if (blocks == 0 || blocks > 0x7fffffffull) return -1;
        hipLaunchKernelGGL(k_stream_copy_wide, dim3((uint32_t)blocks), dim3(256), 0, s,
                           reinterpret_cast<const v4f*>(src), reinterpret_cast<v4f*>(dst), n4);
        return 0;
    }
    const uint64_t blocks = (plane + 255) / 256;
    if (planes != 27 || blocks == 0 || blocks > 0x7fffffffull) return -1;
    hipLaunchKernelGGL((k_stream_copy<27>), dim3((uint32_t)blocks), dim3(256), 0, s, src, dst, plane);
    return 0;
}

int launch_reduce(int lattice, int storage, const StepArgs& a, double* uf, double* p1, double* p2, double* out,
                  hipStream_t s) {
    dim3 grid = flat_grid(nodes_of(a.g)), block(256);
#define L_RED(L, S) hipLaunchKernelGGL((k_reduce_nodes<L, S>), grid, block, 0, s, a, uf, p1)
    CMLB_DISPATCH(L_RED)
#undef L_RED
    const int D = (lattice == kD3Q27) ? 3 : 2;
    hipLaunchKernelGGL(k_reduce_vort, grid, block, 0, s, a.g, D, uf, p2);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64 * kRedVals), 0, s, p1, p2, (int)grid.x, out);
    return 0;
}

}  // namespace cmlb
