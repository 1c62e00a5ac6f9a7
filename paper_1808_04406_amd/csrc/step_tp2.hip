// Two D3Q27 stream + collide steps per launch (temporal blocking), and its
// launcher.
//
// The update of two consecutive steps at a node needs the once-updated
// populations of its 26 neighbours. Each workgroup owns a tile of TX x TY
// nodes in x-y and a chunk of planes in z, and marches up the chunk one
// plane at a time:
//   1. the first step is computed for the tile plus a one-node halo (the
//      "region", (TX+2) x (TY+2) nodes) of plane q, pulling from the stored
//      state in HBM; the results go to LDS, rounded exactly as a store and a
//      reload through the storage type would round them;
//   2. the second step is computed for the tile's own nodes of plane q - 1,
//      pulling from LDS, and written to HBM.
// A node's second step pulls population i from plane (q-1) - e_z,i: the nine
// populations with e_z = -1 from plane q (just computed), the nine with
// e_z = 0 from plane q - 1 and the nine with e_z = +1 from plane q - 2. LDS
// therefore holds one slot of the first group, two of the second and three
// of the third (54 populations per region node, 142,560 bytes for 64 x 8),
// so one workgroup fills a CU's LDS. The stored state read by the first step
// of plane q + 2 is fetched two iterations ahead into registers.
//
// Each population is read from HBM once per region node and written once per
// tile node: per two node updates about (TX+2)(TY+2)/(TX TY) x 108 B of
// reads and 108 B of writes, against 432 B for two single steps. The
// arithmetic is the single-step kernel's, node by node, so the result equals
// two single steps exactly.
//
// FP32 and FP64 storage take this path (FP64 with a 32 x 8 tile, whose 54
// doubles per region node fill the same LDS). With 16-bit storage one step
// per launch moves 108 B per update and is faster than this kernel, whose
// rate is set by its arithmetic and barriers rather than by HBM (measured at
// 256^3 and 512^3: about 46,000 MLUPS against 27,000-31,000).
#include "launch.hpp"

#include "collide_tp.hpp"

#include <algorithm>

namespace cmlb {

// Tile of one workgroup by storage: TX x TY nodes, a region of
// (TX + 2) x (TY + 2), 54 values per region node in LDS.  FP32: 64 x 8 in
// 142,560 B; FP64: 32 x 8 in 146,880 B.
template <int ST>
struct Tb2Geom;
template <>
struct Tb2Geom<kF32> {
    static constexpr int TX = 64, TY = 8, Threads = 704;
};
template <>
struct Tb2Geom<kF64> {
    static constexpr int TX = 32, TY = 8, Threads = 384;
};
template <int ST>
struct Tb2Tile : Tb2Geom<ST> {
    using G = Tb2Geom<ST>;
    static constexpr int RX = G::TX + 2, RY = G::TY + 2, RN = RX * RY;
    static constexpr int LdsBytes = 54 * RN * (int)sizeof(typename Store<ST>::R);
    static_assert(G::Threads >= RN && G::Threads >= G::TX * G::TY && G::Threads % 64 == 0, "tile threads");
    static_assert(LdsBytes <= 160 * 1024, "LDS of one CU");
};

struct Step2Args {
    StepArgs a;
    uint32_t ntx, nty;   // tiles in x and y
    uint32_t cz;         // planes per z chunk
};

// PAD: x-rows padded to the pitch (otherwise the row stride is nx).
// B32 (FP32 states below 4 GiB): the pulls go through one raw buffer
// resource, with a lane offset that is fixed for the whole z-march (the
// pulled row and column within a plane) and a scalar offset (population
// plane plus z-plane), so the loads need no per-population address
// arithmetic and no 64-bit per-population base addresses in scalar
// registers (which otherwise spill to vector-register lanes): 1.5 % faster
// at 256^3.  The stores stay global non-temporal stores; buffer stores
// with the same cache policy measured 3.5 % slower.
template <int ST, bool PAD, bool B32>
__global__ __launch_bounds__(Tb2Geom<ST>::Threads) void k_step2_tp(Step2Args A) {
    using S = Store<ST>;
    using T = typename S::T;
    using R = typename S::R;
    using Tile = Tb2Tile<ST>;
    static_assert(!S::kScaled && sizeof(R) == sizeof(T), "unscaled storage of the arithmetic type only");
    static_assert(!B32 || ST == kF32, "buffer addressing for FP32 states only");
    constexpr int TX = Tile::TX, TY = Tile::TY, RX = Tile::RX, RN = Tile::RN;
    __shared__ R lds[54 * RN];
    R* sD = lds;             // [9][RN]     e_z = -1 group, plane q
    R* sM = lds + 9 * RN;    // [2][9][RN]  e_z =  0 group, planes q, q - 1
    R* sU = lds + 27 * RN;   // [3][9][RN]  e_z = +1 group, planes q, q - 1, q - 2
    const StepArgs& a = A.a;
    const uint32_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;

    // Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous
    // range of tiles so that halo reads of neighbouring tiles share its L2.
    uint32_t b = blockIdx.x;
    if (gridDim.x % 8 == 0) b = (b % 8) * (gridDim.x / 8) + b / 8;
    const uint32_t bx = b % A.ntx, by = (b / A.ntx) % A.nty, bz = b / (A.ntx * A.nty);
    const uint32_t x0 = bx * TX, y0 = by * TY, z0 = bz * A.cz;
    const uint32_t zend = min(z0 + A.cz, nz);
    const int t = threadIdx.x;
    const char* __restrict__ src = static_cast<const char*>(a.src);
    char* __restrict__ dst = static_cast<char*>(a.dst);
    const uint64_t plane_bytes = a.g.plane * sizeof(T);
    const uint32_t rowb = (PAD ? a.pitch : nx) * (uint32_t)sizeof(T);
    const uint32_t plane_b = (uint32_t)plane_bytes;   // B32: 27 planes below 2^32 bytes
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(src), 0, (int)(27u * plane_b), kBufferWord3);

    // First step: region node r of this thread, its pulled x offsets and y rows.
    const bool act1 = t < RN;
    const int r = act1 ? t : 0;
    const int rx = r % RX, ry = r / RX;
    const uint32_t gx = (x0 + rx + nx - 1) % nx, gy = (y0 + ry + ny - 1) % ny;
    const uint32_t xoff[3] = {wrap_inc(gx, nx) * (uint32_t)sizeof(T), gx * (uint32_t)sizeof(T),
                              wrap_dec(gx, nx) * (uint32_t)sizeof(T)};   // x - e for e = -1, 0, +1
    const uint32_t ysrc[3] = {wrap_inc(gy, ny), gy, wrap_dec(gy, ny)};
    // In-plane byte offsets of the nine pulled (y, x) rows and columns: the
    // same for every plane of the z-march, so only the plane offset, uniform
    // across the workgroup, changes from one iteration to the next.
    uint32_t xyoff[3][3];
    static_for<0, 3>([&](auto Y) {
        constexpr int ey = decltype(Y)::value;
        static_for<0, 3>([&](auto X) {
            constexpr int ex = decltype(X)::value;
            xyoff[ey][ex] = ysrc[ey] * rowb + xoff[ex];
        });
    });
    const uint32_t zb = ny * rowb;   // bytes of one z-plane of a population
    // Second step: tile node of this thread.
    const bool in2 = t < TX * TY;
    const int ix = t % TX, iy = t / TX;
    const uint32_t gx2 = x0 + ix, gy2 = y0 + iy;
    const bool act2 = in2 && gx2 < nx && gy2 < ny;
    const int rc2 = (iy + 1) * RX + (ix + 1);

    R om[8];
    static_for<0, 8>([&](auto N) { om[decltype(N)::value] = R(a.omega[decltype(N)::value]); });
    const R rho0 = R(a.rho0);

    auto load_state = [&](R (&h)[27], uint32_t qz) {
        const uint32_t zo[3] = {wrap_inc(qz, nz) * zb, qz * zb, wrap_dec(qz, nz) * zb};
        static_for<0, 27>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int ex = TP<3>::ex(i), ey = TP<3>::ey(i), ez = TP<3>::ez(i);
            if constexpr (B32) {
                h[i] = __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(
                                                 rsrc, (int)xyoff[ey + 1][ex + 1], (int)((uint32_t)i * plane_b + zo[ez + 1]), 0));
            } else {
                const uint32_t off = zo[ez + 1] + xyoff[ey + 1][ex + 1];
                h[i] = S::load(reinterpret_cast<const T*>(src + i * plane_bytes + off));
            }
        });
    };
    const int J = (int)(zend - z0) + 1;   // iterations j = 0..J: first step at plane z0 - 1 + j
    // Iteration j: first step of plane z0 - 1 + j from h (then h <- the state
    // pulled for plane z0 + 1 + j), second step of plane z0 - 2 + j.
    auto iteration = [&](int j, R (&h)[27], uint32_t qz_ahead) {
        if (act1) {
            tp_collide<3, R>(h, rho0, om);
            R* pM = sM + (j & 1) * 9 * RN;
            R* pU = sU + (j % 3) * 9 * RN;
            static_for<0, 27>([&](auto I) {
                constexpr int i = decltype(I)::value;
                R v = h[i];
                v = S::round(v);
                R* slot = i < 9 ? sD : (i < 18 ? pM : pU);
                slot[(i % 9) * RN + r] = v;
            });
            if (j + 2 <= J) load_state(h, qz_ahead);
        }
        __syncthreads();
        if (j >= 2 && in2) {
            const R* pM = sM + ((j - 1) & 1) * 9 * RN;
            const R* pU = sU + ((j - 2) % 3) * 9 * RN;
            R g[27];
            static_for<0, 27>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int ex = TP<3>::ex(i), ey = TP<3>::ey(i), ez = TP<3>::ez(i);
                const R* slot = ez == -1 ? sD : (ez == 0 ? pM : pU);
                g[i] = slot[(i % 9) * RN + rc2 - ey * RX - ex];
            });
            tp_collide<3, R>(g, rho0, om);
            if (act2) {
                const uint32_t p = z0 + (uint32_t)j - 2;
                const uint32_t off = (p * ny + gy2) * rowb + gx2 * (uint32_t)sizeof(T);
                static_for<0, 27>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    S::store(reinterpret_cast<T*>(dst + i * plane_bytes + off), g[i]);
                });
            }
        }
        __syncthreads();
    };

    // Two register sets alternate so that the state for iteration j + 2 is in
    // flight during iteration j + 1.
    R ha[27], hb[27];
    const uint32_t q0 = (z0 + nz - 1) % nz, q1 = wrap_inc(q0, nz);
    if (act1) {
        load_state(ha, q0);
        load_state(hb, q1);
    }
    uint32_t qa = wrap_inc(q1, nz);   // plane of iteration j + 2
    for (int j = 0; j <= J; j += 2) {
        iteration(j, ha, qa);
        qa = wrap_inc(qa, nz);
        if (j + 1 <= J) iteration(j + 1, hb, qa);
        qa = wrap_inc(qa, nz);
    }
}

// ---------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------
// One workgroup (704 threads for FP32, 384 for FP64) fills a CU's LDS, so a
// launch of B workgroups runs in ceil(B / 256) rounds.  A workgroup whose chunk has cz planes makes
// cz + 2 first-step iterations (its first step starts one plane below the
// chunk and ends one plane above it) and cz second-step iterations.
//
// Cost model of a launch (fitted to MI355X measurements of grids from 32^3
// to 384^3, within about 6 %): a first-step iteration of a full round takes
// 3.55 us and a second-step one 2.75 us; half of that time scales with the
// fraction of tile nodes inside the grid (ragged tiles move less data); a
// launch costs 3 us.  The z chunking is the one with the lowest modelled
// time among chunks of at most 128 planes: at 512^3 longer chunks ran
// slower than the model predicts (one chunk of 512 planes: 36,600 MLUPS;
// four of 128: 39,100; eight of 64: 39,800), while at 256^3 the model's
// two chunks of 128 planes are the fastest.  A single step costs 3 us plus
// 38 ps per node (its HBM rate), which decides, in automatic mode, between
// this kernel and two single steps.  FP64 (32 x 8 tiles): 4.6 and 2.8 us per
// iteration, 84 ps per node for a single step.
struct Tb2Cost {
    double it1_us, it2_us;     // first- and second-step iteration of a full round
    double step_ps_per_node;   // one single-step launch, per node
};
constexpr Tb2Cost kTbCostF32 = {3.55, 2.75, 38.0};
constexpr Tb2Cost kTbCostF64 = {4.6, 2.8, 84.0};   // fitted at 256^3 and 512^3
constexpr double kLaunchUs = 3.0;
constexpr uint32_t kTbMaxChunk = 128;

namespace {
struct Step2Plan {
    Step2Args A;
    uint32_t blocks;
    double cost_us;   // model time of the launch
};

template <int ST>
Step2Plan step2_plan(const StepArgs& a, const Tb2Cost& cost) {
    using Tile = Tb2Tile<ST>;
    // the plan depends on the grid only; callers step one grid many times
    thread_local uint32_t key[3] = {0, 0, 0};
    thread_local Step2Plan last;
    if (key[0] == a.g.nx && key[1] == a.g.ny && key[2] == a.g.nz) {
        Step2Plan P = last;
        P.A.a = a;
        return P;
    }
    Step2Plan P;
    P.A.a = a;
    P.A.ntx = (a.g.nx + Tile::TX - 1) / Tile::TX;
    P.A.nty = (a.g.ny + Tile::TY - 1) / Tile::TY;
    const uint64_t tiles = (uint64_t)P.A.ntx * P.A.nty;
    const double fill = (double)a.g.nx * a.g.ny / ((double)tiles * Tile::TX * Tile::TY);
    const double scale = 0.5 + 0.5 * fill;
    auto model_us = [&](uint32_t cz) {
        const uint64_t nzc = (a.g.nz + cz - 1) / cz;
        const double rounds = (double)((tiles * nzc + 255) / 256);
        return rounds * ((cz + 2) * cost.it1_us + cz * cost.it2_us) * scale;
    };
    // counts from the fewest chunks of at most kTbMaxChunk planes; beyond
    // 4096 chunks every count needs more rounds than it saves planes
    const uint32_t nzc0 = std::min(std::min((a.g.nz + kTbMaxChunk - 1) / kTbMaxChunk, a.g.nz), 4096u);
    uint32_t best_cz = (a.g.nz + nzc0 - 1) / nzc0;
    double best = model_us(best_cz);
    for (uint32_t nzc = nzc0 + 1; nzc <= a.g.nz && nzc <= 4096; ++nzc) {
        const uint32_t cz = (a.g.nz + nzc - 1) / nzc;
        if ((a.g.nz + cz - 1) / cz != nzc) continue;   // the same chunking as a smaller count
        const double t = model_us(cz);
        if (t < best) { best = t; best_cz = cz; }
    }
    P.A.cz = best_cz;
    P.blocks = (uint32_t)(tiles * ((a.g.nz + best_cz - 1) / best_cz));
    P.cost_us = kLaunchUs + best;
    key[0] = a.g.nx; key[1] = a.g.ny; key[2] = a.g.nz;
    last = P;
    return P;
}

template <int ST>
int launch2(const StepArgs& a, const Tb2Cost& cost, bool force, hipStream_t s) {
    // lane byte offsets within a population plane are 32-bit
    if (a.g.plane * sizeof(typename Store<ST>::T) >= (1ull << 31)) return -1;
    const Step2Plan P = step2_plan<ST>(a, cost);
    if (!force) {
        const double single_us = kLaunchUs + (double)nodes_of(a.g) * cost.step_ps_per_node * 1e-6;
        if (P.cost_us >= 2.0 * single_us) return -1;
    }
    constexpr int threads = Tb2Geom<ST>::Threads;
    const bool pad = a.pitch != a.g.nx;
    if constexpr (ST == kF32) {
        // buffer addressing when the 27 planes span less than 4 GiB
        if (27ull * a.g.plane * sizeof(float) < (1ull << 32)) {
            if (pad) hipLaunchKernelGGL((k_step2_tp<ST, true, true>), dim3(P.blocks), dim3(threads), 0, s, P.A);
            else hipLaunchKernelGGL((k_step2_tp<ST, false, true>), dim3(P.blocks), dim3(threads), 0, s, P.A);
            return 0;
        }
    }
    if (pad) hipLaunchKernelGGL((k_step2_tp<ST, true, false>), dim3(P.blocks), dim3(threads), 0, s, P.A);
    else hipLaunchKernelGGL((k_step2_tp<ST, false, false>), dim3(P.blocks), dim3(threads), 0, s, P.A);
    return 0;
}
}  // namespace

int launch_step2_tp(int lattice, int storage, const StepArgs& a, bool force, hipStream_t s) {
    if (lattice != kD3Q27) return -1;
    if (storage == kF32) return launch2<kF32>(a, kTbCostF32, force, s);
    if (storage == kF64) return launch2<kF64>(a, kTbCostF64, force, s);
    return -1;
}

}  // namespace cmlb
