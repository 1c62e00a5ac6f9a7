// Two thermal D2Q37 stream + collide steps per launch (temporal blocking),
// and its launcher.
//
// Each workgroup owns a segment of tx columns (tx <= 122) and a chunk of cy
// rows, and marches up the chunk one row at a time.  Iteration j:
//   1. the first step of row y0 - 3 + j is computed for the segment plus
//      three halo columns on each side (the "region", tx + 6 <= 128 nodes,
//      one thread each), pulling from the stored state in HBM; the results go
//      to LDS;
//   2. the second step of row y0 - 6 + j is computed for the segment's own
//      nodes, pulling from LDS, and written to HBM.
// The second step of row R pulls population i from first-step row R - e_y,i,
// which was computed 3 + e_y,i iterations earlier.  LDS therefore keeps
// population i of each first-step row in a ring of 4 + e_y,i row slots.
// With 3, 5, 7, 7, 7, 5, 3 populations at e_y = -3..3 that is
// sum (4 + e_y,i) = 148 population rows of 128 columns: 75,776 bytes, so two
// workgroups share a CU.  The stored state for the first step of iteration
// j + 2 is fetched into registers during iteration j, right after the first
// step of iteration j has consumed its own.
//
// Each population is read from HBM about (tx + 6) / tx times per two node
// updates (plus the chunk's six lead-in rows) and written once, against
// twice each for two single steps.  The arithmetic is the single-step
// kernel's, node by node, and FP32 storage rounds nothing, so the result
// equals two single steps exactly.  FP32 storage only.
#include "launch.hpp"

#include "collide_h2.hpp"

namespace cmlb {

constexpr int kD2Threads = 128;                 // region columns
constexpr int kD2MaxTX = kD2Threads - 6;        // segment columns
constexpr int kD2Rows = 148;                    // population rows in LDS

// Ring placement of population i: slots of 4 + e_y,i rows, nk populations
// share each slot (those with the same e_y), k is i's place among them.
struct D37Ring {
    int base[37], len[37], nk[37], k[37];
    int total;
};

constexpr D37Ring make_d37_ring() {
    D37Ring R{};
    int count[7] = {};
    for (int i = 0; i < 37; ++i) ++count[kTab37.ey[i] + 3];
    int gbase[7] = {};
    int acc = 0;
    for (int g = 0; g < 7; ++g) {
        gbase[g] = acc;
        acc += (g + 1) * count[g];   // 4 + e_y slots for e_y = g - 3
    }
    int seen[7] = {};
    for (int i = 0; i < 37; ++i) {
        const int g = kTab37.ey[i] + 3;
        R.base[i] = gbase[g];
        R.len[i] = g + 1;
        R.nk[i] = count[g];
        R.k[i] = seen[g]++;
    }
    R.total = acc;
    return R;
}
inline constexpr D37Ring kRing37 = make_d37_ring();
static_assert(kRing37.total == kD2Rows, "D2Q37 ring rows");
// Workgroups that share a CU's 160 KB of LDS, and the workgroups of one full round.
constexpr int kD2PerCU = (160 * 1024) / (kD2Rows * kD2Threads * 4);
constexpr uint32_t kD2Slots = 256u * kD2PerCU;
static_assert(kD2PerCU >= 1, "one workgroup fits a CU's LDS");

struct Step2D37Args {
    StepArgs a;
    uint32_t ntx;   // segments per row
    uint32_t tx;    // columns per segment (<= kD2MaxTX)
    uint32_t cy;    // rows per chunk
};

// Ring groups by e_y (g = e_y + 3): first row and population count.
struct D37Groups {
    int base[7], nk[7];
};
constexpr D37Groups make_d37_groups() {
    D37Groups G{};
    for (int i = 0; i < 37; ++i) {
        const int g = kTab37.ey[i] + 3;
        G.base[g] = kRing37.base[i];
        G.nk[g] = kRing37.nk[i];
    }
    return G;
}
inline constexpr D37Groups kGroups37 = make_d37_groups();

// PAD: x-rows padded to the pitch (otherwise the row stride is nx).
// Addressing: the state (37 planes) is below 4 GiB, so each population is
// reached through a raw buffer resource on its base with a 32-bit lane
// offset (column and plane, fixed for the whole launch) plus a scalar row
// offset; the loop issues no per-population address arithmetic.
template <int MODEL, bool PAD>
__global__ __launch_bounds__(kD2Threads) void k_step2_d37(Step2D37Args A) {
    __shared__ float lds[kD2Rows * kD2Threads];
    const StepArgs& a = A.a;
    const uint32_t nx = a.g.nx, ny = a.g.ny;

    // Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous
    // range so that the halo columns of neighbouring segments share its L2.
    uint32_t b = blockIdx.x;
    if (gridDim.x % 8 == 0) b = (b % 8) * (gridDim.x / 8) + b / 8;
    const uint32_t bx = b % A.ntx, by = b / A.ntx;
    const uint32_t tx = A.tx;
    const uint32_t x0 = bx * tx, y0 = by * A.cy;
    const uint32_t yend = min(y0 + A.cy, ny);
    const int t = threadIdx.x;
    const uint32_t plane_b = (uint32_t)a.g.plane * (uint32_t)sizeof(float);
    const uint32_t rowb = (PAD ? a.pitch : nx) * (uint32_t)sizeof(float);
    const int nbytes = (int)(37u * plane_b);   // the descriptor's 32-bit record count
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.src), 0, nbytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rdst = __builtin_amdgcn_make_buffer_rsrc(a.dst, 0, nbytes, kBufferWord3);

    // First step: region column t, global x = x0 + t - 3 (periodic); lane
    // offset of population i: column x - e_x,i in plane i.
    const bool act1 = (uint32_t)t < tx + 6;
    const uint32_t gx = (x0 + (uint32_t)t + nx - 3) % nx;
    uint32_t voff[37];
    static_for<0, 37>([&](auto I) {
        constexpr int i = decltype(I)::value;
        voff[i] = wrap_sub(gx, kTab37.ex[i], nx) * (uint32_t)sizeof(float) + (uint32_t)i * plane_b;
    });
    // Second step: segment column t.
    const bool in2 = (uint32_t)t < tx;
    const uint32_t gx2 = x0 + (uint32_t)t;
    const bool act2 = in2 && gx2 < nx;
    uint32_t vst[37];   // lane offset of the output node in plane i
    static_for<0, 37>([&](auto I) {
        constexpr int i = decltype(I)::value;
        vst[i] = gx2 * (uint32_t)sizeof(float) + (uint32_t)i * plane_b;
    });

    float om[8], wc[8];
    static_for<0, 8>([&](auto N) {
        om[decltype(N)::value] = (float)a.omega[decltype(N)::value];
        wc[decltype(N)::value] = (float)a.wcls[decltype(N)::value];
    });
    const float rho0 = (float)a.rho0, r = (float)a.r, theta0 = (float)a.theta0;
    const bool thermal = a.thermal != 0;

    // Populations pulled by the first step at a row f of the region column;
    // srow[e_y + 3] is the byte offset of row f - e_y.
    auto load_state = [&](float (&h)[37], const uint32_t (&srow)[7]) {
        static_for<0, 37>([&](auto I) {
            constexpr int i = decltype(I)::value;
            h[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)voff[i],
                                                                                 (int)srow[kTab37.ey[i] + 3], 0));
        });
    };
    // Ring slot written this iteration per group, j mod (g + 1), kept as its
    // element offset slot * nk * 128; the slot read by the second step is
    // the one written next, (j + 1) mod (g + 1).
    int wslot[7] = {0, 0, 0, 0, 0, 0, 0};
    const int J = (int)(yend - y0) + 5;   // iterations j = 0..J
    const uint32_t wrapb = ny * rowb;
    auto next_row = [&](uint32_t (&srow)[7]) {
        static_for<0, 7>([&](auto E) {
            constexpr int e = decltype(E)::value;
            const uint32_t v = srow[e] + rowb;
            srow[e] = v == wrapb ? 0u : v;
        });
    };
    auto iteration = [&](int j, float (&h)[37], const uint32_t (&srow_ahead)[7]) {
        int rslot[7];
        static_for<0, 7>([&](auto G) {
            constexpr int g = decltype(G)::value;
            constexpr int step = kGroups37.nk[g] * kD2Threads;
            rslot[g] = (wslot[g] == g * step) ? 0 : wslot[g] + step;
        });
        if (act1) {
            h2_collide<kD2Q37, MODEL, float>(h, rho0, om, r, wc, thermal, theta0);
            static_for<0, 37>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int g = kTab37.ey[i] + 3;
                float* row = lds + kGroups37.base[g] * kD2Threads + wslot[g] + t;
                row[kRing37.k[i] * kD2Threads] = h[i];
            });
            if (j + 2 <= J) load_state(h, srow_ahead);
        }
        __syncthreads();
        if (j >= 6 && in2) {
            float g2[37];
            static_for<0, 37>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int g = kTab37.ey[i] + 3;
                const float* row = lds + kGroups37.base[g] * kD2Threads + rslot[g] + t + 3;
                g2[i] = row[kRing37.k[i] * kD2Threads - kTab37.ex[i]];
            });
            h2_collide<kD2Q37, MODEL, float>(g2, rho0, om, r, wc, thermal, theta0);
            if (act2) {
                const uint32_t so = (y0 + (uint32_t)j - 6) * rowb;
                static_for<0, 37>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, g2[i]), rdst, (int)vst[i],
                                                          (int)so, 0);
                });
            }
        }
        __syncthreads();
        static_for<0, 7>([&](auto G) { wslot[decltype(G)::value] = rslot[decltype(G)::value]; });
    };

    // Two register sets alternate so that the state for iteration j + 2 is in
    // flight during iteration j + 1.
    float ha[37], hb[37];
    uint32_t srow[7];   // rows pulled by the first step of iteration 0
    const uint32_t f0 = (y0 + ny - 3) % ny;
    static_for<0, 7>([&](auto E) {
        constexpr int e = decltype(E)::value - 3;
        srow[e + 3] = wrap_sub(f0, e, ny) * rowb;
    });
    if (act1) load_state(ha, srow);
    next_row(srow);
    if (act1) load_state(hb, srow);
    next_row(srow);   // now the rows of iteration j + 2
    for (int j = 0; j <= J; j += 2) {
        iteration(j, ha, srow);
        next_row(srow);
        if (j + 1 <= J) iteration(j + 1, hb, srow);
        next_row(srow);
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch, the second step's moments accumulated row by row
// ---------------------------------------------------------------------------
// The collision depends on the pulled populations only through their 15
// lattice moments M_kl (k + l <= 4).  Population i of first-step row f is
// pulled by second-step row f + e_y,i, so each first-step row, once in LDS,
// is folded into the moments of the seven second-step rows f - 3..f + 3
// that it feeds; a thread keeps those seven partial moment sets in
// registers, and row f - 3 is complete after row f has been folded in.  LDS
// then holds one first-step row (double-buffered: 37,888 bytes) instead of
// the 148-row ring, four workgroups share a CU, and each SIMD runs two waves.
// The moments are summed in another order than in the single-step kernel,
// so the result agrees with two single steps to FP32 rounding, not bitwise.
// Measured on one MI355X it is no faster than the ring kernel: the second
// wave per SIMD raises VALU use, but twice the workgroups means chunks of
// half the height, whose six lead-in rows add as much work.  It is selected
// explicitly (steps-per-launch mode 3), never automatically.
constexpr int kD2AccLds = 2 * 37 * kD2Threads;   // floats
constexpr int kD2AccPerCU = (160 * 1024) / (kD2AccLds * 4);
constexpr uint32_t kD2AccSlots = 256u * kD2AccPerCU;
static_assert(kD2AccPerCU == 4, "four workgroups of two waves per CU");

template <int MODEL, bool PAD>
__global__ __launch_bounds__(kD2Threads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_step2_d37_acc(Step2D37Args A) {
    __shared__ float lds[kD2AccLds];
    const StepArgs& a = A.a;
    const uint32_t nx = a.g.nx, ny = a.g.ny;
    uint32_t b = blockIdx.x;
    if (gridDim.x % 8 == 0) b = (b % 8) * (gridDim.x / 8) + b / 8;
    const uint32_t bx = b % A.ntx, by = b / A.ntx;
    const uint32_t tx = A.tx;
    const uint32_t x0 = bx * tx, y0 = by * A.cy;
    const uint32_t yend = min(y0 + A.cy, ny);
    const int t = threadIdx.x;
    const uint32_t plane_b = (uint32_t)a.g.plane * (uint32_t)sizeof(float);
    const uint32_t rowb = (PAD ? a.pitch : nx) * (uint32_t)sizeof(float);
    const int nbytes = (int)(37u * plane_b);
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.src), 0, nbytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rdst = __builtin_amdgcn_make_buffer_rsrc(a.dst, 0, nbytes, kBufferWord3);

    // First step: region column t, global x = x0 + t - 3 (periodic); xo[e + 3]
    // is the byte offset of column x - e.
    const bool act1 = (uint32_t)t < tx + 6;
    const uint32_t gx = (x0 + (uint32_t)t + nx - 3) % nx;
    uint32_t xo[7];
    static_for<0, 7>([&](auto E) {
        constexpr int e = decltype(E)::value - 3;
        xo[e + 3] = wrap_sub(gx, e, nx) * (uint32_t)sizeof(float);
    });
    // Second step: segment column t.
    const bool in2 = (uint32_t)t < tx;
    const uint32_t gx2 = x0 + (uint32_t)t;
    const bool act2 = in2 && gx2 < nx;
    const uint32_t xst = gx2 * (uint32_t)sizeof(float);

    float om[8], wc[8];
    static_for<0, 8>([&](auto N) {
        om[decltype(N)::value] = (float)a.omega[decltype(N)::value];
        wc[decltype(N)::value] = (float)a.wcls[decltype(N)::value];
    });
    const float rho0 = (float)a.rho0, r = (float)a.r, theta0 = (float)a.theta0;
    const bool thermal = a.thermal != 0;

    auto load_state = [&](float (&h)[37], const uint32_t (&srow)[7]) {
        static_for<0, 37>([&](auto I) {
            constexpr int i = decltype(I)::value;
            h[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                rsrc, (int)xo[kTab37.ex[i] + 3], (int)(srow[kTab37.ey[i] + 3] + (uint32_t)i * plane_b), 0));
        });
    };
    const uint32_t wrapb = ny * rowb;
    auto next_row = [&](uint32_t (&srow)[7]) {
        static_for<0, 7>([&](auto E) {
            constexpr int e = decltype(E)::value;
            const uint32_t v = srow[e] + rowb;
            srow[e] = v == wrapb ? 0u : v;
        });
    };

    // acc[s]: partial moments of second-step row f - 3 + s, f the first-step
    // row of the current iteration.
    Tri<float> acc[7];
    static_for<0, 7>([&](auto S) {
        static_for<0, 5>([&](auto K) {
            static_for<0, 5 - decltype(K)::value>([&](auto L) {
                acc[decltype(S)::value].v[decltype(K)::value][decltype(L)::value] = 0.0f;
            });
        });
    });

    float h[37];
    uint32_t srow[7];
    const uint32_t f0 = (y0 + ny - 3) % ny;
    static_for<0, 7>([&](auto E) {
        constexpr int e = decltype(E)::value - 3;
        srow[e + 3] = wrap_sub(f0, e, ny) * rowb;
    });
    if (act1) load_state(h, srow);
    const int J = (int)(yend - y0) + 5;   // iterations j = 0..J: first step of row y0 - 3 + j
    for (int j = 0; j <= J; ++j) {
        float* buf = lds + (j & 1) * (37 * kD2Threads);
        if (act1) {
            h2_collide<kD2Q37, MODEL, float>(h, rho0, om, r, wc, thermal, theta0);
            static_for<0, 37>([&](auto I) {
                constexpr int i = decltype(I)::value;
                buf[i * kD2Threads + t] = h[i];
            });
        }
        if (j < J) {   // the rows stay workgroup-uniform (scalar) outside the branch
            next_row(srow);
            if (act1) load_state(h, srow);
        }
        __syncthreads();
        if (in2) {
            // fold this row into the seven rows it feeds: population i goes to
            // slot e_y,i + 3 with weights e_x^k e_y^l
            static_for<0, 7>([&](auto G) {
                constexpr int e = decltype(G)::value - 3;
                float P[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};   // sum over the group of v e_x^k
                static_for<0, 37>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    if constexpr (kTab37.ey[i] == e) {
                        constexpr int ex = kTab37.ex[i];
                        const float v = buf[i * kD2Threads + t + 3 - ex];
                        static_for<0, 5>([&](auto K) {
                            constexpr int k = decltype(K)::value;
                            constexpr int c = ipow_c(ex, k);
                            if constexpr (c == 1) P[k] += v;
                            else if constexpr (c == -1) P[k] -= v;
                            else if constexpr (c != 0) P[k] += float(c) * v;
                        });
                    }
                });
                static_for<0, 5>([&](auto K) {
                    static_for<0, 5 - decltype(K)::value>([&](auto L) {
                        constexpr int k = decltype(K)::value, l = decltype(L)::value;
                        constexpr int c = ipow_c(e, l);
                        if constexpr (c == 1) acc[e + 3].v[k][l] += P[k];
                        else if constexpr (c == -1) acc[e + 3].v[k][l] -= P[k];
                        else if constexpr (c != 0) acc[e + 3].v[k][l] += float(c) * P[k];
                    });
                });
            });
            if (j >= 6) {
                float g2[37];
                h2_collide_moments<kD2Q37, MODEL, float>(acc[0], g2, rho0, om, r, wc, thermal, theta0);
                if (act2) {
                    const uint32_t so = (y0 + (uint32_t)j - 6) * rowb;
                    static_for<0, 37>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, g2[i]), rdst, (int)xst,
                                                              (int)(so + (uint32_t)i * plane_b), 0);
                    });
                }
            }
            static_for<0, 6>([&](auto S) { acc[decltype(S)::value] = acc[decltype(S)::value + 1]; });
            static_for<0, 5>([&](auto K) {
                static_for<0, 5 - decltype(K)::value>([&](auto L) {
                    acc[6].v[decltype(K)::value][decltype(L)::value] = 0.0f;
                });
            });
        }
    }
}

// ---------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------
// kD2PerCU workgroups share a CU's LDS, so a launch of B workgroups runs in
// ceil(B / kD2Slots) rounds of cy + 6 iterations, the first six of which
// (the lead-in rows) compute only first steps and cost about half.  The row
// chunking is the one with the lowest modelled time; the model also
// decides, in automatic mode, between this kernel and two single steps.
// Constants from MI355X measurements from 384^2 to 2048^2: a full iteration
// of a round takes 3.9-4.7 us (4.3 here), a single step 3 us plus 54-86 ps
// per node (58 here).  The model then picks the faster path at every size
// measured: single steps up to 512^2, two steps per launch from 640^2 on.
constexpr double kD2ItUs = 4.3, kD2LaunchUs = 3.0, kD2StepPsPerNode = 58.0;

// The row-accumulating kernel runs four workgroups per CU (kD2AccSlots per
// round); an iteration of a full round takes kD2AccItUs.
constexpr double kD2AccItUs = 6.0;

namespace {
struct Step2D37Plan {
    Step2D37Args A;
    uint32_t blocks;
    double cost_us;
};

// Segments of at most kD2MaxTX columns, and the row chunking with the lowest
// modelled time for `slots` workgroups per round.
template <uint32_t kSlots, int kTag>
Step2D37Plan step2_d37_plan(const StepArgs& a, double it_us) {
    thread_local uint32_t key[2] = {0, 0};
    thread_local Step2D37Plan last;
    if (key[0] == a.g.nx && key[1] == a.g.ny) {
        Step2D37Plan P = last;
        P.A.a = a;
        return P;
    }
    Step2D37Plan P;
    P.A.a = a;
    P.A.ntx = (a.g.nx + kD2MaxTX - 1) / kD2MaxTX;
    P.A.tx = (a.g.nx + P.A.ntx - 1) / P.A.ntx;
    double best = 0.0;
    uint32_t best_cy = a.g.ny;
    for (uint32_t nc = 1; nc <= a.g.ny && nc <= 8192; ++nc) {
        const uint32_t cy = (a.g.ny + nc - 1) / nc;
        if ((a.g.ny + cy - 1) / cy != nc) continue;   // the same chunking as a smaller count
        const double rounds = (double)(((uint64_t)P.A.ntx * nc + kSlots - 1) / kSlots);
        const double tm = rounds * (cy + 3) * it_us;   // six half-cost lead-in iterations
        if (nc == 1 || tm < best) { best = tm; best_cy = cy; }
    }
    P.A.cy = best_cy;
    P.blocks = P.A.ntx * ((a.g.ny + best_cy - 1) / best_cy);
    P.cost_us = kD2LaunchUs + best;
    key[0] = a.g.nx; key[1] = a.g.ny;
    last = P;
    return P;
}
}  // namespace

static int launch_step2_d37_acc(int model, const StepArgs& a, hipStream_t s) {
    const Step2D37Plan P = step2_d37_plan<kD2AccSlots, 1>(a, kD2AccItUs);
    const bool raw = (model == kRawMRT), pad = (a.pitch != a.g.nx);
    if (raw) {
        if (pad) hipLaunchKernelGGL((k_step2_d37_acc<kRawMRT, true>), dim3(P.blocks), dim3(kD2Threads), 0, s, P.A);
        else hipLaunchKernelGGL((k_step2_d37_acc<kRawMRT, false>), dim3(P.blocks), dim3(kD2Threads), 0, s, P.A);
    } else {
        if (pad) hipLaunchKernelGGL((k_step2_d37_acc<kCM, true>), dim3(P.blocks), dim3(kD2Threads), 0, s, P.A);
        else hipLaunchKernelGGL((k_step2_d37_acc<kCM, false>), dim3(P.blocks), dim3(kD2Threads), 0, s, P.A);
    }
    return 0;
}

int launch_step2_d37(int storage, int model, const StepArgs& a, int mode, hipStream_t s) {
    if (storage != kF32) return -1;
    // the kernels address the whole state (37 planes) with 32-bit offsets
    if (37ull * a.g.plane * 4 >= (1ull << 32)) return -1;
    if (mode == kFuseTwoAcc) return launch_step2_d37_acc(model, a, s);
    const bool force = (mode == kFuseTwo);
    const Step2D37Plan P = step2_d37_plan<kD2Slots, 0>(a, kD2ItUs);
    if (!force) {
        const double single_us = kD2LaunchUs + (double)nodes_of(a.g) * kD2StepPsPerNode * 1e-6;
        if (P.cost_us >= 2.0 * single_us) return -1;
    }
    const bool raw = (model == kRawMRT), pad = (a.pitch != a.g.nx);
    if (raw) {
        if (pad) hipLaunchKernelGGL((k_step2_d37<kRawMRT, true>), dim3(P.blocks), dim3(kD2Threads), 0, s, P.A);
        else hipLaunchKernelGGL((k_step2_d37<kRawMRT, false>), dim3(P.blocks), dim3(kD2Threads), 0, s, P.A);
    } else {
        if (pad) hipLaunchKernelGGL((k_step2_d37<kCM, true>), dim3(P.blocks), dim3(kD2Threads), 0, s, P.A);
        else hipLaunchKernelGGL((k_step2_d37<kCM, false>), dim3(P.blocks), dim3(kD2Threads), 0, s, P.A);
    }
    return 0;
}

}  // namespace cmlb
