// Shared device-side definitions of the cmlb HIP library: storage codecs,
// compile-time lattice tables, kernel argument blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace cmlb {

// D2Q37 is the ninth-degree 37-velocity rule on |e|^2 <= 10; E9B-E9D and
// E7A-E7D are the other minimal 2D rules of degree 9 (37 velocities) and 7
// (17 velocities) whose velocity components are at most 3.
enum Lattice { kD2Q9 = 0, kD3Q27 = 1, kD2Q37 = 2, kE9B = 3, kE9C = 4, kE9D = 5, kE7A = 6, kE7B = 7, kE7C = 8,
               kE7D = 9 };
constexpr int kNumLattices = 10;
enum Storage { kF64 = 0, kF32 = 1, kBF16 = 2, kF16 = 3 };
enum Model { kCM = 0, kRawMRT = 1, kRegBGK = 2 };

// ---------------------------------------------------------------------------
// Compile-time loops: the body receives std::integral_constant<int, I>, so
// every lattice index used inside is a constant expression and the population
// arrays stay in registers.
// ---------------------------------------------------------------------------
template <int I, int N, class F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Reciprocal: the hardware approximation (1 ulp) in FP32, exact division in FP64.
template <class R>
__device__ __forceinline__ R recip(R x) {
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(x);
    else return R(1) / x;
}

// Periodic neighbour indices.
__device__ __forceinline__ uint32_t wrap_dec(uint32_t v, uint32_t n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ uint32_t wrap_inc(uint32_t v, uint32_t n) { return v + 1 == n ? 0 : v + 1; }

// source coordinate v - e (periodic), |e| <= 3, for the D2Q37 gather
__device__ __forceinline__ uint32_t wrap_sub(uint32_t v, int e, uint32_t n) {
    int s = (int)v - e;
    s += (s < 0) ? (int)n : 0;
    s -= (s >= (int)n) ? (int)n : 0;
    return (uint32_t)s;
}

// ---------------------------------------------------------------------------
// Lattice velocity tables.
// D2Q9 / D3Q27: e in {-1,0,1}^D, index i = (ex+1) + 3(ey+1) + 9(ez+1).
// 2D Hermite rules: the velocities of their shells, ordered lexicographically
// in (ey, ex); the ordering is centrally symmetric, so -e_i is population
// Q - 1 - i and the rest population is (Q - 1) / 2.  cls(i) is the index of
// the velocity's shell, which numbers the weight classes.
// ---------------------------------------------------------------------------
struct Shells2 {
    int n;           // number of shells (8 on 37 velocities, 5 on 17)
    int ab[8][2];    // |e| component pairs, smaller first
};

constexpr Shells2 rule_shells(int lat) {
    switch (lat) {
        case kD2Q37: return {8, {{0, 0}, {0, 1}, {1, 1}, {0, 2}, {1, 2}, {2, 2}, {0, 3}, {1, 3}}};
        case kE9B: return {8, {{0, 0}, {0, 1}, {1, 1}, {0, 2}, {1, 2}, {2, 2}, {0, 3}, {2, 3}}};
        case kE9C: return {8, {{0, 0}, {0, 1}, {1, 1}, {0, 2}, {1, 2}, {3, 3}, {0, 3}, {1, 3}}};
        case kE9D: return {8, {{0, 0}, {0, 1}, {1, 1}, {0, 2}, {1, 2}, {3, 3}, {0, 3}, {2, 3}}};
        case kE7A: return {5, {{0, 0}, {0, 1}, {1, 1}, {2, 2}, {0, 3}}};
        case kE7B: return {5, {{0, 0}, {0, 1}, {1, 1}, {3, 3}, {0, 3}}};
        case kE7C: return {5, {{0, 0}, {0, 2}, {1, 1}, {3, 3}, {0, 3}}};
        case kE7D: return {5, {{0, 0}, {1, 1}, {2, 2}, {3, 3}, {0, 3}}};
    }
    return {0, {}};
}

struct TabH2 {
    int q;       // velocities
    int n;       // Hermite truncation N = M: 4 for degree 9, 3 for degree 7
    int ex[37], ey[37], cls[37];
};

constexpr TabH2 make_tab_h2(int lat) {
    TabH2 t{};
    const Shells2 sh = rule_shells(lat);
    t.n = sh.n == 8 ? 4 : 3;
    int k = 0;
    for (int ey = -3; ey <= 3; ++ey)
        for (int ex = -3; ex <= 3; ++ex) {
            const int ax = ex < 0 ? -ex : ex, ay = ey < 0 ? -ey : ey;
            const int a = ax < ay ? ax : ay, b = ax < ay ? ay : ax;
            for (int c = 0; c < sh.n; ++c)
                if (sh.ab[c][0] == a && sh.ab[c][1] == b) {
                    t.ex[k] = ex;
                    t.ey[k] = ey;
                    t.cls[k] = c;
                    ++k;
                }
        }
    t.q = k;
    return t;
}

// Compile-time description of a 2D Hermite rule.
template <int LAT>
struct H2 {
    static constexpr TabH2 tab = make_tab_h2(LAT);
    static constexpr int Q = tab.q, N = tab.n, rest = (tab.q - 1) / 2;
};

inline constexpr TabH2 kTab37 = make_tab_h2(kD2Q37);
static_assert(kTab37.q == 37 && kTab37.ex[36] == 1 && kTab37.ey[36] == 3, "D2Q37 table");
static_assert(kTab37.ex[18] == 0 && kTab37.ey[18] == 0, "D2Q37 rest population");
static_assert(H2<kE7A>::Q == 17 && H2<kE7D>::Q == 17 && H2<kE9D>::Q == 37, "rule sizes");
static_assert(H2<kE7C>::tab.ex[8] == 0 && H2<kE7C>::tab.ey[8] == 0, "17-velocity rest population");

template <int D>
struct TP {
    static constexpr int Q = (D == 2) ? 9 : 27;
    static constexpr int ex(int i) { return i % 3 - 1; }
    static constexpr int ey(int i) { return (i / 3) % 3 - 1; }
    static constexpr int ez(int i) { return D == 3 ? i / 9 - 1 : 0; }
};

// ---------------------------------------------------------------------------
// Storage codecs.  The stored value is g = s (f - w rho0); decode returns the
// deviation in the arithmetic type R.  16-bit encodes round to nearest even.
// Stores are non-temporal: the output is not read again within a step.
// ---------------------------------------------------------------------------
template <int ST>
struct Store;

template <>
struct Store<kF64> {
    using T = double;
    using R = double;
    static constexpr bool kScaled = false;
    __device__ static R load(const T* p) { return *p; }
    __device__ static void store(T* p, R v) { __builtin_nontemporal_store(v, p); }
    __device__ static R round(R v) { return v; }   // value after a store and a load
    __host__ __device__ static double to_double(T v) { return v; }
    __host__ __device__ static T from_double(double v) { return v; }
};

template <>
struct Store<kF32> {
    using T = float;
    using R = float;
    static constexpr bool kScaled = false;
    __device__ static R load(const T* p) { return *p; }
    __device__ static void store(T* p, R v) { __builtin_nontemporal_store(v, p); }
    __device__ static R round(R v) { return v; }
    __host__ __device__ static double to_double(T v) { return v; }
    __host__ __device__ static T from_double(double v) { return (float)v; }
};

__host__ __device__ inline uint16_t f32_to_bf16_rne(float v) {
    uint32_t b = __builtin_bit_cast(uint32_t, v);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);  // quiet NaN
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

template <>
struct Store<kBF16> {
    using T = uint16_t;
    using R = float;
    static constexpr bool kScaled = true;
    __device__ static R load(const T* p) { return bf16_to_f32(*p); }
    // the hardware conversion rounds to nearest even, as f32_to_bf16_rne does
    __device__ static T encode(R v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    __device__ static void store(T* p, R v) { __builtin_nontemporal_store(encode(v), p); }
    __device__ static R round(R v) { return bf16_to_f32(encode(v)); }
    __host__ __device__ static double to_double(T v) { return bf16_to_f32(v); }
    __host__ __device__ static T from_double(double v) { return f32_to_bf16_rne((float)v); }
};

template <>
struct Store<kF16> {
    using T = uint16_t;
    using R = float;
    static constexpr bool kScaled = true;
    __device__ static R load(const T* p) { return (float)__builtin_bit_cast(_Float16, *p); }
    __device__ static void store(T* p, R v) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, (_Float16)v), p);
    }
    __device__ static R round(R v) { return (float)(_Float16)v; }
    __device__ static double to_double(T v) { return (double)__builtin_bit_cast(_Float16, v); }
    __device__ static T from_double(double v) { return __builtin_bit_cast(uint16_t, (_Float16)(float)v); }
};

// ---------------------------------------------------------------------------
// Kernel argument blocks (passed by value).
// ---------------------------------------------------------------------------
// The state is structure of arrays: population i of node (x, y, z) sits at
// i * plane + (z * ny + y) * pitch + x.  Rows are padded from nx to pitch
// (StepArgs::pitch) so that every row starts on a 128-byte line (see
// row_pitch); x >= nx is never read or written by the steps.
struct GridArgs {
    uint32_t nx, ny, nz;
    uint32_t nchunks;   // x chunks of blockDim.x per row
    uint64_t plane;     // population-plane stride in elements: pitch * ny * nz
};

__host__ __device__ inline uint64_t nodes_of(const GridArgs& g) { return (uint64_t)g.nx * g.ny * g.nz; }

// Row stride for nx elements of `elem` bytes: nx rounded up to a multiple of
// 128 bytes, unless that adds more than one eighth (short rows stay unpadded).
__host__ __device__ inline uint32_t row_pitch(uint32_t nx, uint32_t elem) {
    const uint32_t unit = 128u / elem;
    const uint32_t padded = (nx + unit - 1) / unit * unit;
    return (uint64_t)(padded - nx) * 8u <= nx ? padded : nx;
}

// Population-plane stride in elements for planes of `elems` elements of
// `elem` bytes: a plane of at least 1 MiB starts 4 KiB past a multiple of
// 8 KiB after the previous one (its bytes rounded up to 8 KiB, plus 4 KiB).
// 27 concurrent streams whose starts lie a multiple of 8 KiB apart copy up
// to 10 % slower on MI355X's HBM3E than with this offset.
__host__ __device__ inline uint64_t plane_stride(uint64_t elems, uint32_t elem) {
    const uint64_t bytes = elems * elem;
    if (bytes < (1ull << 20)) return elems;
    return ((bytes + 8191u) / 8192u * 8192u + 4096u) / elem;
}

// Plane stride of a state of `elems` = pitch * ny * nz elements.  Only D3Q27
// states in 16-bit storage take the offset: their one-step kernel runs 3 %
// faster with it at 512^3, while the two-step FP32 and FP64 kernels and the
// D2Q37 row sweep measured the same or slower (FP64 at 512^3 -4 %, D2Q37 at
// 2048^2 -7 %), so their planes stay unpadded.
__host__ __device__ inline uint64_t state_plane(int lattice, int storage, uint64_t elems) {
    return (lattice == kD3Q27 && (storage == kBF16 || storage == kF16)) ? plane_stride(elems, 2u) : elems;
}

// Raw buffer resource word 3 for gfx9-family devices (32-bit data, no swizzle).
constexpr int kBufferWord3 = 0x00020000;

// Row stride of a state.  D3Q27 FP32 states are stepped two steps per launch
// by default, and that kernel, which moves 64-node tile rows, streams rows
// aligned to 32 bytes as fast as padded ones (padding them measured slower),
// so such rows stay unpadded; every other state takes row_pitch.
__host__ __device__ inline uint32_t state_pitch(int lattice, int storage, uint32_t nx) {
    const uint32_t elem = storage == kF64 ? 8u : (storage == kF32 ? 4u : 2u);
    if (lattice == kD3Q27 && storage == kF32 && nx % 8u == 0) return nx;
    return row_pitch(nx, elem);
}

// Padded offset of node n (flat index over nx * ny * nz, below 2^32).
__host__ __device__ inline uint64_t node_offset(uint32_t nx, uint32_t pitch, uint64_t n) {
    const uint32_t m = (uint32_t)n;
    return (uint64_t)(m / nx) * pitch + m % nx;
}

struct StepArgs {
    const void* src;
    void* dst;
    GridArgs g;
    double rho0;
    double theta0;      // frozen temperature (isothermal)
    double omega[8];    // omega[n] = 1 / tau_n
    float s[37];        // storage scale per population
    float inv_s[37];
    double r;           // D2Q37 abscissa scale
    double wcls[8];     // D2Q37 weight per |e|^2 class
    int thermal;
    uint32_t pitch;     // row stride of the state in elements (>= g.nx); fills the
                        // struct's tail padding, so the argument block keeps its size
};

// Several lattices of one configuration stepped by one launch: blockIdx.y
// selects the lattice; its buffers and relaxation rates replace those of a.
constexpr int kMaxBatch = 16;

struct BatchLattice {
    const void* src;
    void* dst;
    double omega[8];
};

struct BatchArgs {
    StepArgs a;
    BatchLattice l[kMaxBatch];
};

// The step arguments of lattice blockIdx.y of a batch.
__device__ __forceinline__ StepArgs batch_member(const BatchArgs& A) {
    StepArgs a = A.a;
    const BatchLattice& L = A.l[blockIdx.y];
    a.src = L.src;
    a.dst = L.dst;
    for (int n = 0; n < 8; ++n) a.omega[n] = L.omega[n];
    return a;
}

struct FieldArgs {
    const double* rho;
    const double* u;      // [D][node], lattice units
    const double* theta;  // may be null
    double* out_rho;
    double* out_u;
    double* out_theta;
};

}  // namespace cmlb
