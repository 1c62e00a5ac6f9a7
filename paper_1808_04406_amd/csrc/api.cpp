// C ABI of the cmlb library: context management, validation, lattice tables,
// and the host side of every entry point declared in include/cmlb.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/cmlb.h"
#include "launch.hpp"

using namespace cmlb;

namespace {

thread_local std::string g_create_error;

struct HostLattice {
    int D = 0, Q = 0;
    int e[37][3] = {};
    double w[37] = {};
    double r = 0.0;
    double wcls[8] = {};
};

// Weights per shell and the scale r of a 2D Hermite rule.  The
// even-moment conditions of its degree (nine for degree 9, six for degree
// 7), sum_i w_i xi_x^p xi_y^q = E[X^p] E[Y^q] with xi = r e, are solved for
// the shell weights and x = 1/r^2 by Newton's method (the conditions are
// linear in w and polynomial in x).  Newton starts from equal weights and
// x = 0.5, then from other x until it reaches the rule's one solution with
// positive weights.
bool solve_rule(int kind, double (&wcls)[8], double& r) {
    const TabH2 t = make_tab_h2(kind);
    const int nc = (t.q == 37) ? 8 : 5, nm = nc + 1;
    static const int mons9[9][2] = {{0, 0}, {2, 0}, {4, 0}, {2, 2}, {6, 0}, {4, 2}, {8, 0}, {6, 2}, {4, 4}};
    static const int mons7[6][2] = {{0, 0}, {2, 0}, {4, 0}, {2, 2}, {6, 0}, {4, 2}};
    const int (*mons)[2] = (t.q == 37) ? mons9 : mons7;
    auto gm = [](int p) { double m = 1.0; if (p % 2) return 0.0; for (int k = p - 1; k > 0; k -= 2) m *= k; return m; };
    double S[9][8] = {};
    for (int i = 0; i < t.q; ++i) {
        const int ex = t.ex[i], ey = t.ey[i], c = t.cls[i];
        for (int k = 0; k < nm; ++k) S[k][c] += std::pow((double)ex, mons[k][0]) * std::pow((double)ey, mons[k][1]);
    }
    static const double x0s[6] = {0.5, 0.3, 0.7, 1.0, 1.5, 2.0};
    for (double x0 : x0s) {
        double v[9];
        for (int c = 0; c < nc; ++c) v[c] = 1.0 / t.q;
        v[nc] = x0;
        bool ok = true;
        for (int it = 0; it < 100 && ok; ++it) {
            double J[9][10];
            double norm = 0.0;
            for (int k = 0; k < nm; ++k) {
                const int h = (mons[k][0] + mons[k][1]) / 2;
                const double g = gm(mons[k][0]) * gm(mons[k][1]);
                double F = -g * std::pow(v[nc], h);
                for (int c = 0; c < nc; ++c) { F += S[k][c] * v[c]; J[k][c] = S[k][c]; }
                J[k][nc] = h ? -g * h * std::pow(v[nc], h - 1) : 0.0;
                J[k][nm] = -F;
                norm += F * F;
            }
            // Gaussian elimination with partial pivoting on the augmented system
            for (int col = 0; col < nm && ok; ++col) {
                int piv = col;
                for (int row = col + 1; row < nm; ++row)
                    if (std::fabs(J[row][col]) > std::fabs(J[piv][col])) piv = row;
                if (J[piv][col] == 0.0) { ok = false; break; }
                for (int k = 0; k <= nm; ++k) std::swap(J[col][k], J[piv][k]);
                for (int row = col + 1; row < nm; ++row) {
                    const double m = J[row][col] / J[col][col];
                    for (int k = col; k <= nm; ++k) J[row][k] -= m * J[col][k];
                }
            }
            if (!ok) break;
            double dv[9];
            for (int row = nm - 1; row >= 0; --row) {
                double sum = J[row][nm];
                for (int k = row + 1; k < nm; ++k) sum -= J[row][k] * dv[k];
                dv[row] = sum / J[row][row];
            }
            for (int k = 0; k < nm; ++k) v[k] += dv[k];
            if (norm < 1e-30 && it > 3) break;
        }
        bool pos = ok && v[nc] > 0.0 && std::isfinite(v[nc]);
        for (int c = 0; c < nc && pos; ++c) pos = v[c] > 0.0;
        if (!pos) continue;
        // converged: every condition holds
        double worst = 0.0;
        for (int k = 0; k < nm; ++k) {
            double F = -gm(mons[k][0]) * gm(mons[k][1]) * std::pow(v[nc], (mons[k][0] + mons[k][1]) / 2);
            for (int c = 0; c < nc; ++c) F += S[k][c] * v[c];
            worst = std::fmax(worst, std::fabs(F));
        }
        if (!(worst < 1e-12)) continue;
        for (int c = 0; c < 8; ++c) wcls[c] = c < nc ? v[c] : 0.0;
        r = 1.0 / std::sqrt(v[nc]);
        return true;
    }
    return false;
}

bool host_lattice(int kind, HostLattice& L) {
    if (kind == CMLB_D2Q9 || kind == CMLB_D3Q27) {
        const int D = (kind == CMLB_D2Q9) ? 2 : 3;
        static const double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
        L.D = D;
        L.Q = (D == 2) ? 9 : 27;
        L.r = std::sqrt(3.0);
        for (int i = 0; i < L.Q; ++i) {
            const int ix = i % 3, iy = (i / 3) % 3, iz = (D == 3) ? i / 9 : 1;
            L.e[i][0] = ix - 1;
            L.e[i][1] = iy - 1;
            L.e[i][2] = (D == 3) ? iz - 1 : 0;
            L.w[i] = w1[ix] * w1[iy] * (D == 3 ? w1[iz] : 1.0);
        }
        return true;
    }
    if (kind >= CMLB_D2Q37 && kind < kNumLattices) {
        static std::mutex m;
        static bool done[kNumLattices] = {};
        static double wc_all[kNumLattices][8], r_all[kNumLattices];
        {
            std::lock_guard<std::mutex> lock(m);
            if (!done[kind]) {
                if (!solve_rule(kind, wc_all[kind], r_all[kind])) return false;
                done[kind] = true;
            }
        }
        const TabH2 t = make_tab_h2(kind);
        L.D = 2;
        L.Q = t.q;
        L.r = r_all[kind];
        for (int c = 0; c < 8; ++c) L.wcls[c] = wc_all[kind][c];
        for (int i = 0; i < t.q; ++i) {
            L.e[i][0] = t.ex[i];
            L.e[i][1] = t.ey[i];
            L.e[i][2] = 0;
            L.w[i] = wc_all[kind][t.cls[i]];
        }
        return true;
    }
    return false;
}

size_t storage_bytes(int st) { return st == CMLB_F64 ? 8 : st == CMLB_F32 ? 4 : 2; }

int lattice_q(int lattice) {
    return lattice == CMLB_D2Q9 ? 9 : (lattice == CMLB_D3Q27 ? 27 : make_tab_h2(lattice).q);
}

// Population-plane stride in elements (pitch * ny * nz, padded by state_plane).
uint64_t state_plane_of(const cmlb_params* p) {
    const uint64_t pitch = cmlb::state_pitch(p->lattice, p->storage, (uint32_t)p->nx);
    return cmlb::state_plane(p->lattice, p->storage, pitch * (uint64_t)p->ny * (uint64_t)p->nz);
}

// Bytes of one population buffer: Q planes.
size_t state_bytes_of(const cmlb_params* p) {
    return (size_t)lattice_q(p->lattice) * state_plane_of(p) * storage_bytes(p->storage);
}

}  // namespace

static_assert(CMLB_D2Q37 == cmlb::kD2Q37 && CMLB_E9B == cmlb::kE9B && CMLB_E7A == cmlb::kE7A &&
              CMLB_E7D == cmlb::kE7D && CMLB_E7D + 1 == cmlb::kNumLattices, "lattice numbering");
static_assert(CMLB_MAX_BATCH == cmlb::kMaxBatch, "batch size limit");
static_assert(sizeof(cmlb::BatchArgs) <= 4096, "batch arguments fit the kernel argument segment");

struct cmlb_ctx {
    cmlb_params p{};
    HostLattice L;
    uint64_t nodes = 0;
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    bool owns = true;
    bool own_stream = false;
    bool initialised = false;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;      // orders batched launches across streams (created on first use)
    double omega[8] = {};
    float s[37] = {}, inv_s[37] = {};
    int64_t steps = 0;
    int fuse = 0;                 // 0 automatic, 1 one step per launch, 2 two where supported, 3 two, D2Q37 rows accumulated
    // HIP graph of graph_steps steps (0: launch eagerly), captured from the
    // buffer parity graph_cur; replays leave the parity unchanged
    int graph_steps = 0;
    hipGraphExec_t gexec = nullptr;
    int graph_cur = -1;
    std::string err;
    // reduction scratch (allocated on first use)
    double* red_u = nullptr;
    double* red_p = nullptr;
    double* red_out = nullptr;
    // learned closure
    bool closure_loaded = false;
    bool closure_on = false;
    float* cl_params = nullptr;   // FP32 master weights, Adam moments m1, m2 (3 x 2084), sigma (27)
    void* cl_net = nullptr;       // packed network
    float* cl_partials = nullptr; // per-block partial gradients
    float* cl_grad = nullptr;     // reduced gradient + objective
    int cl_blocks = 0;
    int cl_step = 0;
    int cl_tie_even = 0;
    int cl_objective = 0;         // CMLB_CLOSURE_OBJ_POPULATIONS or CMLB_CLOSURE_OBJ_MOMENTUM
    float cl_beta1 = 0.9f, cl_beta2 = 0.999f, cl_eps = 1e-8f;   // Adam
    int cl_frozen = 0;            // bit j: Adam leaves output j's weights unchanged
    float* cl_f1 = nullptr;       // momentum objective: closure step of each pair [pair][27][nodes]
    float* cl_D = nullptr;        //   and the mismatch field [pair][3][nodes]
    int64_t cl_pairs_cap = 0;     //   pairs the two buffers hold
};

namespace {

int fail(cmlb_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(cmlb_ctx* c, hipError_t e, const char* where) {
    return fail(c, CMLB_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Forget the captured step graph (its kernel arguments are out of date).
void graph_drop(cmlb_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->graph_cur = -1;
}

StepArgs base_args(const cmlb_ctx* c) {
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.pitch = state_pitch(c->p.lattice, c->p.storage, (uint32_t)c->p.nx);
    a.g = make_grid((uint32_t)c->p.nx, (uint32_t)c->p.ny, (uint32_t)c->p.nz, state_plane_of(&c->p));
    a.rho0 = c->p.rho0;
    a.theta0 = c->p.theta0;
    for (int n = 0; n < 8; ++n) a.omega[n] = c->omega[n];
    for (int i = 0; i < 37; ++i) {
        a.s[i] = c->s[i];
        a.inv_s[i] = c->inv_s[i];
    }
    a.r = c->L.r;
    for (int k = 0; k < 8; ++k) a.wcls[k] = c->L.wcls[k];
    a.thermal = c->p.thermal;
    return a;
}

void set_omegas(cmlb_ctx* c) {
    for (int n = 0; n < 8; ++n) {
        const double t = (n < 2) ? 1.0 : (c->p.tau[n] == 0.0 ? 1.0 : c->p.tau[n]);
        c->omega[n] = (n < 2) ? 0.0 : 1.0 / t;
    }
    if (c->p.model == CMLB_MODEL_REG_BGK)
        for (int n = 3; n < 8; ++n) c->omega[n] = c->omega[2];
}

std::string validate(const cmlb_params* p) {
    if (!p) return "params is NULL";
    if (p->lattice < CMLB_D2Q9 || p->lattice > CMLB_E7D) return "unknown lattice";
    if (p->storage < CMLB_F64 || p->storage > CMLB_F16) return "unknown storage";
    if (p->model < CMLB_MODEL_CM || p->model > CMLB_MODEL_REG_BGK) return "unknown collision model";
    const bool rule2d = p->lattice >= CMLB_D2Q37;   // a 2D Hermite rule
    if (p->model == CMLB_MODEL_RAW_MRT && p->lattice != CMLB_D2Q37)
        return "raw-moment MRT is implemented for D2Q37 only";
    if (p->model == CMLB_MODEL_REG_BGK && !rule2d)
        return "regularised BGK is implemented for the 2D Hermite rules only";
    if (rule2d && p->lattice != CMLB_D2Q37 && p->storage != CMLB_F64 && p->storage != CMLB_F32)
        return "the 2D rules other than D2Q37 take FP64 or FP32 storage";
    if (p->thermal && !rule2d) return "thermal mode needs a 2D Hermite rule (D2Q37, E9*, E7*)";
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "grid sizes must be >= 1";
    if (p->lattice != CMLB_D3Q27 && p->nz != 1) return "2D lattices need nz == 1";
    // the gather of the 2D rules wraps shifts of up to 3 cells with a single correction
    if (rule2d && (p->nx < 3 || p->ny < 3)) return "the 2D Hermite rules need nx, ny >= 3";
    if (p->nx > (1 << 20) || p->ny > (1 << 20) || p->nz > (1 << 20)) return "grid size too large";
    const int Q = lattice_q(p->lattice);
    const double nodes = (double)p->nx * (double)p->ny * (double)p->nz;
    if (nodes * Q >= 4294967296.0 * 8) return "grid too large";
    if ((uint64_t)p->nx * (uint64_t)p->ny * (uint64_t)p->nz >= (1ull << 32)) return "more than 2^32 nodes";
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return "rho0 must be positive";
    if (!(p->theta0 > 0.0) || !std::isfinite(p->theta0)) return "theta0 must be positive";
    for (int n = 2; n < 8; ++n) {
        const double t = p->tau[n];
        if (t != 0.0 && !(t > 0.0 && std::isfinite(t))) return "tau must be positive (0 = default 1.0)";
    }
    for (int i = 0; i < Q; ++i) {
        const double s = p->scale[i];
        if (s != 0.0 && !(s > 0.0 && std::isfinite(s))) return "scale must be positive (0 = automatic)";
    }
    if (p->reserved != 0) return "reserved must be 0";
    return "";
}

int create_impl(const cmlb_params* p, void* fa, void* fb, cmlb_ctx** out) {
    if (!out) { g_create_error = "out is NULL"; return CMLB_EINVAL; }
    *out = nullptr;
    std::string why = validate(p);
    if (!why.empty()) { g_create_error = why; return CMLB_EINVAL; }
    cmlb_ctx* c = new (std::nothrow) cmlb_ctx();
    if (!c) { g_create_error = "host allocation failed"; return CMLB_ENOMEM; }
    c->p = *p;
    if (!host_lattice(p->lattice, c->L)) {
        delete c;
        g_create_error = "lattice table generation failed";
        return CMLB_EINVAL;
    }
    c->nodes = (uint64_t)p->nx * p->ny * p->nz;
    set_omegas(c);
    for (int i = 0; i < c->L.Q; ++i) {
        double s = p->scale[i];
        if (s == 0.0) {
            s = 1.0;
            if (p->storage == CMLB_F16) {
                // largest power of two with 16 w_i rho0 s_i <= 65504 / 2
                s = std::exp2(std::floor(std::log2(32752.0 / (16.0 * c->L.w[i] * p->rho0))));
            }
        }
        c->s[i] = (float)s;
        c->inv_s[i] = (float)(1.0 / s);
    }
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) { g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e); delete c; return CMLB_EDEVICE; }
    if (p->hip_stream) {
        c->stream = (hipStream_t)p->hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { g_create_error = std::string("hipStreamCreate: ") + hipGetErrorString(e); delete c; return CMLB_EDEVICE; }
        c->own_stream = true;
    }
    const size_t bytes = state_bytes_of(p);
    if (fa || fb) {
        const uintptr_t a0 = (uintptr_t)fa, b0 = (uintptr_t)fb;
        const bool overlap = a0 < b0 + bytes && b0 < a0 + bytes;   // the step reads one and writes the other
        if (!fa || !fb || overlap || (a0 % 256) || (b0 % 256)) {
            g_create_error = "external buffers must be two non-overlapping non-NULL 256-byte aligned pointers";
            cmlb_destroy(c);
            return CMLB_EINVAL;
        }
        c->f[0] = fa;
        c->f[1] = fb;
        c->owns = false;
    } else {
        for (int k = 0; k < 2; ++k) {
            e = hipMalloc(&c->f[k], bytes);
            if (e != hipSuccess) {
                g_create_error = std::string("hipMalloc population buffer: ") + hipGetErrorString(e);
                (void)hipGetLastError();
                cmlb_destroy(c);
                return CMLB_ENOMEM;
            }
            // row and plane padding is never written by the kernels: zero it once
            if ((e = hipMemsetAsync(c->f[k], 0, bytes, c->stream)) != hipSuccess) {
                g_create_error = std::string("hipMemsetAsync population buffer: ") + hipGetErrorString(e);
                cmlb_destroy(c);
                return CMLB_EDEVICE;
            }
        }
    }
    *out = c;
    return CMLB_OK;
}

// Device staging for host FP64 arrays.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

extern "C" {

int cmlb_lattice_info(int lattice, int* D, int* Q, int* e, double* w, double* r) {
    HostLattice L;
    if (!host_lattice(lattice, L)) return CMLB_EINVAL;
    if (D) *D = L.D;
    if (Q) *Q = L.Q;
    if (r) *r = L.r;
    for (int i = 0; i < L.Q; ++i) {
        if (w) w[i] = L.w[i];
        if (e)
            for (int d = 0; d < 3; ++d) e[3 * i + d] = L.e[i][d];
    }
    return CMLB_OK;
}

int cmlb_copy_bandwidth(int device, uint64_t bytes, int planes, int reps, double* gbps) {
    if (!gbps || reps < 1 || (planes != 1 && planes != 27)) return CMLB_EINVAL;
    uint64_t plane = bytes / (4ull * (uint64_t)planes);
    if (planes == 1) plane -= plane % 4;   // whole 16-byte groups
    if (plane == 0) return CMLB_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return CMLB_EDEVICE;
    const size_t n = (size_t)plane * planes * sizeof(float);
    float *src = nullptr, *dst = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = CMLB_OK;
    float ms = 0.0f;
    if (hipMalloc(&src, n) != hipSuccess || hipMalloc(&dst, n) != hipSuccess) {
        (void)hipGetLastError();
        rc = CMLB_ENOMEM;
    } else if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = CMLB_EDEVICE;
    } else {
        bool ok = hipMemsetAsync(src, 0, n, s) == hipSuccess &&
                  launch_stream_copy(planes, src, dst, plane, s) == 0;       // warm-up
        ok = ok && hipEventRecord(e0, s) == hipSuccess;
        for (int r = 0; ok && r < reps; ++r) ok = launch_stream_copy(planes, src, dst, plane, s) == 0;
        ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!ok || !(ms > 0.0f)) rc = CMLB_EDEVICE;
        else *gbps = 2.0 * (double)n * reps / (ms * 1e-3) / 1e9;
    }
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    return rc;
}

int cmlb_state_bytes(const cmlb_params* p, size_t* bytes) {
    if (!bytes) return CMLB_EINVAL;
    const std::string why = validate(p);
    if (!why.empty()) { g_create_error = why; return CMLB_EINVAL; }
    *bytes = state_bytes_of(p);
    return CMLB_OK;
}

int cmlb_state_layout(const cmlb_params* p, uint64_t* pitch, uint64_t* plane) {
    if (!pitch || !plane) return CMLB_EINVAL;
    const std::string why = validate(p);
    if (!why.empty()) { g_create_error = why; return CMLB_EINVAL; }
    *pitch = cmlb::state_pitch(p->lattice, p->storage, (uint32_t)p->nx);
    *plane = state_plane_of(p);
    return CMLB_OK;
}

int cmlb_create(const cmlb_params* p, cmlb_ctx** out) { return create_impl(p, nullptr, nullptr, out); }

int cmlb_create_external(const cmlb_params* p, void* f_a, void* f_b, cmlb_ctx** out) {
    if (!f_a || !f_b) {
        g_create_error = "external buffers must not be NULL";
        if (out) *out = nullptr;
        return CMLB_EINVAL;
    }
    return create_impl(p, f_a, f_b, out);
}

const char* cmlb_create_error(void) { return g_create_error.c_str(); }

void cmlb_destroy(cmlb_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->p.device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->owns)
        for (int k = 0; k < 2; ++k)
            if (c->f[k]) (void)hipFree(c->f[k]);
    if (c->red_u) (void)hipFree(c->red_u);
    if (c->red_p) (void)hipFree(c->red_p);
    if (c->red_out) (void)hipFree(c->red_out);
    if (c->cl_params) (void)hipFree(c->cl_params);
    if (c->cl_net) (void)hipFree(c->cl_net);
    if (c->cl_partials) (void)hipFree(c->cl_partials);
    if (c->cl_grad) (void)hipFree(c->cl_grad);
    if (c->cl_f1) (void)hipFree(c->cl_f1);
    if (c->cl_D) (void)hipFree(c->cl_D);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->ev) (void)hipEventDestroy(c->ev);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* cmlb_last_error(const cmlb_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

int cmlb_set_tau(cmlb_ctx* c, const double* tau, int n) {
    if (!c) return CMLB_EINVAL;
    if (!tau || n < 1 || n > 6) return fail(c, CMLB_EINVAL, "tau array must hold 1..6 orders (2..7)");
    for (int k = 0; k < n; ++k)
        if (!(tau[k] > 0.0) || !std::isfinite(tau[k])) return fail(c, CMLB_EINVAL, "tau must be positive and finite");
    for (int k = 0; k < n; ++k) c->p.tau[k + 2] = tau[k];
    set_omegas(c);
    graph_drop(c);   // the rates are kernel arguments
    return CMLB_OK;
}

static int init_device_fields(cmlb_ctx* c, const double* rho, const double* u, const double* theta) {
    StepArgs a = base_args(c);
    a.dst = c->f[c->cur];
    FieldArgs fa{};
    fa.rho = rho;
    fa.u = u;
    fa.theta = theta;
    if (launch_init(c->p.lattice, c->p.storage, a, fa, c->stream)) return fail(c, CMLB_EINVAL, "unsupported configuration");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "init kernel launch");
    c->initialised = true;
    c->steps = 0;
    return CMLB_OK;
}

int cmlb_init_fields_device(cmlb_ctx* c, const double* rho, const double* u, const double* theta) {
    if (!c) return CMLB_EINVAL;
    if (!rho || !u) return fail(c, CMLB_EINVAL, "rho and u are required");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    return init_device_fields(c, rho, u, theta);
}

int cmlb_init_fields(cmlb_ctx* c, const double* rho, const double* u, const double* theta) {
    if (!c) return CMLB_EINVAL;
    if (!rho || !u) return fail(c, CMLB_EINVAL, "rho and u are required");
    for (uint64_t n = 0; n < c->nodes; ++n)
        if (!(rho[n] > 0.0) || !std::isfinite(rho[n])) return fail(c, CMLB_EINVAL, "rho must be positive and finite");
    if (theta)
        for (uint64_t n = 0; n < c->nodes; ++n)
            if (!(theta[n] > 0.0) || !std::isfinite(theta[n])) return fail(c, CMLB_EINVAL, "theta must be positive and finite");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    const int D = c->L.D;
    const size_t fb = c->nodes * sizeof(double);
    DevBuf buf;
    hipError_t e = hipMalloc(&buf.p, fb * (D + 2));
    if (e != hipSuccess) { (void)hipGetLastError(); return fail(c, CMLB_ENOMEM, "staging allocation failed"); }
    double* d_rho = (double*)buf.p;
    double* d_u = d_rho + c->nodes;
    double* d_th = d_u + (size_t)D * c->nodes;
    if ((e = hipMemcpyAsync(d_rho, rho, fb, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return hip_fail(c, e, "copy rho");
    if ((e = hipMemcpyAsync(d_u, u, fb * D, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return hip_fail(c, e, "copy u");
    if (theta && (e = hipMemcpyAsync(d_th, theta, fb, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return hip_fail(c, e, "copy theta");
    int rc = init_device_fields(c, d_rho, d_u, theta ? d_th : nullptr);
    if (rc) return rc;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "init");
    return CMLB_OK;
}

// Enqueue n steps on the context stream, one or two steps per launch.
static int enqueue_steps(cmlb_ctx* c, int64_t n) {
    StepArgs a = base_args(c);
    for (int64_t k = 0; k < n;) {
        a.src = c->f[c->cur];
        a.dst = c->f[1 - c->cur];
        int adv = 1;
        if (c->closure_on) {
            launch_step_closure(a, c->cl_net, c->stream);
        } else if (c->fuse != 1 && n - k >= 2 &&
                   launch_step2(c->p.lattice, c->p.storage, c->p.model, a, c->fuse, c->stream) == 0) {
            adv = 2;
        } else if (launch_step(c->p.lattice, c->p.storage, c->p.model, a, c->stream)) {
            return fail(c, CMLB_EINVAL, "unsupported configuration");
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(c, e, "step kernel launch");
        c->cur = 1 - c->cur;
        c->steps += adv;
        k += adv;
    }
    return CMLB_OK;
}

// Capture graph_steps steps from the current buffer parity into c->gexec.
static int graph_capture(cmlb_ctx* c) {
    graph_drop(c);
    const int cur0 = c->cur;
    const int64_t steps0 = c->steps;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(c, e, "graph capture begin");
    int rc = enqueue_steps(c, c->graph_steps);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->stream, &g);
    const bool back = c->cur == cur0;   // an even number of launches
    c->cur = cur0;                       // nothing ran yet
    c->steps = steps0;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "graph capture end");
    if (!back) {
        (void)hipGraphDestroy(g);
        return fail(c, CMLB_EINVAL, "graph steps must give an even number of launches");
    }
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return hip_fail(c, e, "graph instantiate");
    }
    c->graph_cur = cur0;
    return CMLB_OK;
}

int cmlb_step(cmlb_ctx* c, int64_t n) {
    if (!c) return CMLB_EINVAL;
    if (n < 0) return fail(c, CMLB_EINVAL, "negative step count");
    if (!c->initialised) return fail(c, CMLB_ESTATE, "state not initialised");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    if (c->graph_steps > 0 && n >= c->graph_steps) {
        if (!c->gexec || c->graph_cur != c->cur) {
            int rc = graph_capture(c);
            if (rc) return rc;
        }
        const int64_t reps = n / c->graph_steps;
        for (int64_t r = 0; r < reps; ++r) {
            hipError_t e = hipGraphLaunch(c->gexec, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "graph launch");
            c->steps += c->graph_steps;
        }
        n -= reps * c->graph_steps;
    }
    return enqueue_steps(c, n);
}

int cmlb_step_batch(cmlb_ctx* const* ctxs, int count, int64_t n) {
    if (!ctxs || count < 1 || !ctxs[0]) return CMLB_EINVAL;
    cmlb_ctx* c0 = ctxs[0];
    if (count > CMLB_MAX_BATCH) return fail(c0, CMLB_EINVAL, "more than CMLB_MAX_BATCH contexts in a batch");
    if (n < 0) return fail(c0, CMLB_EINVAL, "negative step count");
    const cmlb_params& p0 = c0->p;
    const int Q = c0->L.Q;
    for (int k = 0; k < count; ++k) {
        const cmlb_ctx* c = ctxs[k];
        if (!c) return fail(c0, CMLB_EINVAL, "NULL context in batch");
        for (int j = 0; j < k; ++j)
            if (ctxs[j] == c) return fail(c0, CMLB_EINVAL, "a context appears twice in the batch");
        if (!c->initialised) return fail(c0, CMLB_ESTATE, "state not initialised");
        if (c->closure_on) return fail(c0, CMLB_EINVAL, "the learned closure is not batched");
        const cmlb_params& p = c->p;
        if (p.lattice != p0.lattice || p.storage != p0.storage || p.model != p0.model || p.thermal != p0.thermal ||
            p.nx != p0.nx || p.ny != p0.ny || p.nz != p0.nz || p.rho0 != p0.rho0 || p.theta0 != p0.theta0 ||
            p.device != p0.device)
            return fail(c0, CMLB_EINVAL, "batched contexts differ in lattice, storage, model, grid, rho0, "
                                         "theta0 or device");
        for (int i = 0; i < Q; ++i)
            if (c->s[i] != c0->s[i]) return fail(c0, CMLB_EINVAL, "batched contexts differ in storage scales");
    }
    if (hipSetDevice(p0.device) != hipSuccess) return fail(c0, CMLB_EDEVICE, "hipSetDevice failed");
    if (n == 0) return CMLB_OK;
    hipError_t e = hipSuccess;
    auto event_of = [&](cmlb_ctx* c) {
        if (!c->ev) e = hipEventCreateWithFlags(&c->ev, hipEventDisableTiming);
        return e == hipSuccess;
    };
    // the launches go on the first context's stream, after the work already
    // enqueued on the others' streams
    bool other_streams = false;
    for (int k = 1; k < count; ++k) {
        cmlb_ctx* c = ctxs[k];
        if (c->stream == c0->stream) continue;
        other_streams = true;
        if (!event_of(c) || (e = hipEventRecord(c->ev, c->stream)) != hipSuccess ||
            (e = hipStreamWaitEvent(c0->stream, c->ev, 0)) != hipSuccess)
            return hip_fail(c0, e, "batch stream ordering");
    }
    BatchArgs A;
    std::memset(&A, 0, sizeof(A));
    A.a = base_args(c0);
    for (int k = 0; k < count; ++k)
        for (int m = 0; m < 8; ++m) A.l[k].omega[m] = ctxs[k]->omega[m];
    for (int64_t t = 0; t < n; ++t) {
        for (int k = 0; k < count; ++k) {
            A.l[k].src = ctxs[k]->f[ctxs[k]->cur];
            A.l[k].dst = ctxs[k]->f[1 - ctxs[k]->cur];
        }
        if (launch_step_batch(p0.lattice, p0.storage, p0.model, A, count, c0->stream))
            return fail(c0, CMLB_EINVAL, "unsupported configuration");
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(c0, e, "batched step kernel launch");
        for (int k = 0; k < count; ++k) {
            ctxs[k]->cur = 1 - ctxs[k]->cur;
            ctxs[k]->steps += 1;
        }
    }
    // later work on the other contexts' streams waits for the batch
    if (other_streams) {
        if (!event_of(c0) || (e = hipEventRecord(c0->ev, c0->stream)) != hipSuccess)
            return hip_fail(c0, e, "batch stream ordering");
        for (int k = 1; k < count; ++k)
            if (ctxs[k]->stream != c0->stream && (e = hipStreamWaitEvent(ctxs[k]->stream, c0->ev, 0)) != hipSuccess)
                return hip_fail(c0, e, "batch stream ordering");
    }
    return CMLB_OK;
}

int cmlb_set_graph_steps(cmlb_ctx* c, int steps) {
    if (!c) return CMLB_EINVAL;
    if (steps < 0 || steps % 4 != 0) return fail(c, CMLB_EINVAL, "graph steps must be 0 or a positive multiple of 4");
    graph_drop(c);
    c->graph_steps = steps;
    return CMLB_OK;
}

int cmlb_set_step_fusion(cmlb_ctx* c, int steps_per_launch) {
    if (!c) return CMLB_EINVAL;
    if (steps_per_launch < 0 || steps_per_launch > 3)
        return fail(c, CMLB_EINVAL, "steps per launch must be 0 (automatic), 1, 2 or 3");
    c->fuse = steps_per_launch;
    graph_drop(c);
    return CMLB_OK;
}

int cmlb_sync(cmlb_ctx* c) {
    if (!c) return CMLB_EINVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "sync");
    return CMLB_OK;
}

int cmlb_get_moments(cmlb_ctx* c, double* rho, double* u, double* theta) {
    if (!c) return CMLB_EINVAL;
    if (!c->initialised) return fail(c, CMLB_ESTATE, "state not initialised");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    const int D = c->L.D;
    const size_t fb = c->nodes * sizeof(double);
    DevBuf buf;
    hipError_t e = hipMalloc(&buf.p, fb * (D + 2));
    if (e != hipSuccess) { (void)hipGetLastError(); return fail(c, CMLB_ENOMEM, "staging allocation failed"); }
    StepArgs a = base_args(c);
    a.src = c->f[c->cur];
    FieldArgs fa{};
    fa.out_rho = (double*)buf.p;
    fa.out_u = fa.out_rho + c->nodes;
    fa.out_theta = fa.out_u + (size_t)D * c->nodes;
    launch_moments(c->p.lattice, c->p.storage, a, fa, c->stream);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "moments kernel launch");
    if (rho && (e = hipMemcpyAsync(rho, fa.out_rho, fb, hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return hip_fail(c, e, "copy rho");
    if (u && (e = hipMemcpyAsync(u, fa.out_u, fb * D, hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return hip_fail(c, e, "copy u");
    if (theta && (e = hipMemcpyAsync(theta, fa.out_theta, fb, hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return hip_fail(c, e, "copy theta");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "moments");
    return CMLB_OK;
}

int cmlb_get_moments_device(cmlb_ctx* c, double* rho, double* u, double* theta) {
    if (!c) return CMLB_EINVAL;
    if (!c->initialised) return fail(c, CMLB_ESTATE, "state not initialised");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    StepArgs a = base_args(c);
    a.src = c->f[c->cur];
    FieldArgs fa{};
    fa.out_rho = rho;
    fa.out_u = u;
    fa.out_theta = theta;
    launch_moments(c->p.lattice, c->p.storage, a, fa, c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "moments kernel launch");
    return CMLB_OK;
}

static int codec(cmlb_ctx* c, double* f, bool decode) {
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    const size_t bytes = c->nodes * c->L.Q * sizeof(double);
    DevBuf buf;
    hipError_t e = hipMalloc(&buf.p, bytes);
    if (e != hipSuccess) { (void)hipGetLastError(); return fail(c, CMLB_ENOMEM, "staging allocation failed"); }
    StepArgs a = base_args(c);
    if (!decode && (e = hipMemcpyAsync(buf.p, f, bytes, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copy populations");
    launch_codec(c->p.lattice, c->p.storage, decode, c->f[c->cur], (double*)buf.p, a, c->L.w, c->stream);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "codec kernel launch");
    if (decode && (e = hipMemcpyAsync(f, buf.p, bytes, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copy populations");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "codec");
    return CMLB_OK;
}

int cmlb_get_populations(cmlb_ctx* c, double* f) {
    if (!c) return CMLB_EINVAL;
    if (!f) return fail(c, CMLB_EINVAL, "f is NULL");
    if (!c->initialised) return fail(c, CMLB_ESTATE, "state not initialised");
    return codec(c, f, true);
}

int cmlb_set_populations(cmlb_ctx* c, const double* f) {
    if (!c) return CMLB_EINVAL;
    if (!f) return fail(c, CMLB_EINVAL, "f is NULL");
    int rc = codec(c, const_cast<double*>(f), false);
    if (rc == CMLB_OK) {
        c->initialised = true;
        c->steps = 0;
    }
    return rc;
}

// Launch the reduction kernels with the given scratch (uf: 3 x nodes
// doubles; p1, p2: reduce_blocks(nodes) x kRedVals doubles each; out:
// kRedVals doubles), read the sums back and fill *out.  Every scratch entry
// is written before it is read, so nothing needs clearing between calls.
static int reduce_with(cmlb_ctx* c, double* uf, double* p1, double* p2, double* out_dev, cmlb_globals* out) {
    hipError_t e;
    StepArgs a = base_args(c);
    a.src = c->f[c->cur];
    launch_reduce(c->p.lattice, c->p.storage, a, uf, p1, p2, out_dev, c->stream);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "reduce kernel launch");
    double v[kRedVals];
    if ((e = hipMemcpyAsync(v, out_dev, sizeof(v), hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return hip_fail(c, e, "copy");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "reduce");
    double we2 = 0.0;
    for (int i = 0; i < c->L.Q; ++i)
        we2 += c->L.w[i] * (c->L.e[i][0] * c->L.e[i][0] + c->L.e[i][1] * c->L.e[i][1] + c->L.e[i][2] * c->L.e[i][2]);
    out->mass = c->p.rho0 * (double)c->nodes + v[0];
    out->momentum[0] = v[1];
    out->momentum[1] = v[2];
    out->momentum[2] = v[3];
    out->energy = 0.5 * (v[4] + c->p.rho0 * we2 * (double)c->nodes);
    out->kinetic_energy = v[5];
    out->enstrophy = v[6];
    out->n_nonfinite = (int64_t)v[7];
    out->rho_min = c->p.rho0 - v[8];
    out->rho_max = c->p.rho0 + v[9];
    out->u_max = std::sqrt(v[10]);
    if (out->n_nonfinite > 0) return fail(c, CMLB_EUNSTABLE, "non-finite populations in the state");
    return CMLB_OK;
}

int cmlb_reduce(cmlb_ctx* c, cmlb_globals* out) {
    if (!c) return CMLB_EINVAL;
    if (!out) return fail(c, CMLB_EINVAL, "out is NULL");
    if (!c->initialised) return fail(c, CMLB_ESTATE, "state not initialised");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    hipError_t e;
    const int nb = reduce_blocks(c->nodes);
    if (!c->red_u) {
        if ((e = hipMalloc(&c->red_u, c->nodes * 3 * sizeof(double))) != hipSuccess) { (void)hipGetLastError(); c->red_u = nullptr; return fail(c, CMLB_ENOMEM, "reduction scratch"); }
        if ((e = hipMalloc(&c->red_p, (size_t)nb * 2 * kRedVals * sizeof(double))) != hipSuccess) { (void)hipGetLastError(); c->red_p = nullptr; return fail(c, CMLB_ENOMEM, "reduction scratch"); }
        if ((e = hipMalloc(&c->red_out, kRedVals * sizeof(double))) != hipSuccess) { (void)hipGetLastError(); c->red_out = nullptr; return fail(c, CMLB_ENOMEM, "reduction scratch"); }
    }
    return reduce_with(c, c->red_u, c->red_p, c->red_p + (size_t)nb * kRedVals, c->red_out, out);
}

// ---------------------------------------------------------------------------
// Allocation-free reduction: the same kernels with their scratch in a
// file-scope device array.  In host code `scratch` names a host-side stand-in,
// not device memory; its device address on each GPU comes from
// hipGetSymbolAddress (taken once per device, with that device current) and
// only that address is ever passed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[CMLB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 256;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kScratchDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device address of this device's scratch array (the device must be current).
int scratch_address(cmlb_ctx* c, unsigned char** out) {
    const int dev = c->p.device;
    if (dev < 0 || dev >= kScratchDevices) return fail(c, CMLB_EINVAL, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(c, CMLB_EDEVICE, std::string("scratch symbol address: ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return CMLB_OK;
}
}  // namespace

int cmlb_reduce_noalloc(cmlb_ctx* c, cmlb_globals* out) {
    if (!c) return CMLB_EINVAL;
    if (!out) return fail(c, CMLB_EINVAL, "out is NULL");
    if (!c->initialised) return fail(c, CMLB_ESTATE, "state not initialised");
    if (c->nodes > (uint64_t)CMLB_NOALLOC_MAX_NODES)
        return fail(c, CMLB_EINVAL, "grid of " + std::to_string(c->nodes) + " nodes exceeds the allocation-free "
                    "scratch (at most " + std::to_string(CMLB_NOALLOC_MAX_NODES) + " nodes)");
    const int nb = reduce_blocks(c->nodes);
    const size_t off_p1 = align256(c->nodes * 3 * sizeof(double));
    const size_t off_p2 = off_p1 + align256((size_t)nb * kRedVals * sizeof(double));
    const size_t off_out = off_p2 + align256((size_t)nb * kRedVals * sizeof(double));
    if (off_out + kRedVals * sizeof(double) > (size_t)CMLB_NOALLOC_SCRATCH_BYTES)
        return fail(c, CMLB_EINVAL, "reduction scratch larger than the allocation-free array");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    unsigned char* base = nullptr;
    if (int rc = scratch_address(c, &base)) return rc;
    return reduce_with(c, reinterpret_cast<double*>(base), reinterpret_cast<double*>(base + off_p1),
                       reinterpret_cast<double*>(base + off_p2), reinterpret_cast<double*>(base + off_out), out);
}

int cmlb_state(cmlb_ctx* c, void** f_cur, size_t* bytes, void** stream) {
    if (!c) return CMLB_EINVAL;
    if (f_cur) *f_cur = c->f[c->cur];
    if (bytes) *bytes = state_bytes_of(&c->p);
    if (stream) *stream = (void*)c->stream;
    return CMLB_OK;
}

int64_t cmlb_step_count(const cmlb_ctx* c) { return c ? c->steps : -1; }

int cmlb_set_step_count(cmlb_ctx* c, int64_t steps) {
    if (!c) return CMLB_EINVAL;
    if (steps < 0) return fail(c, CMLB_EINVAL, "negative step count");
    c->steps = steps;
    return CMLB_OK;
}

int cmlb_get_tau(const cmlb_ctx* c, double* tau) {
    if (!c || !tau) return CMLB_EINVAL;
    for (int k = 0; k < 8; ++k) tau[k] = c->p.tau[k];
    return CMLB_OK;
}

int cmlb_store_state_device(cmlb_ctx* c, void* dst) {
    if (!c) return CMLB_EINVAL;
    if (!dst) return fail(c, CMLB_EINVAL, "dst is NULL");
    if (!c->initialised) return fail(c, CMLB_ESTATE, "state not initialised");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    const size_t bytes = state_bytes_of(&c->p);
    hipError_t e = hipMemcpyAsync(dst, c->f[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "store state");
    return CMLB_OK;
}

int cmlb_load_state_device(cmlb_ctx* c, const void* src) {
    if (!c) return CMLB_EINVAL;
    if (!src) return fail(c, CMLB_EINVAL, "src is NULL");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    const size_t bytes = state_bytes_of(&c->p);
    hipError_t e = hipMemcpyAsync(c->f[c->cur], src, bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "load state");
    c->initialised = true;
    c->steps = 0;
    return CMLB_OK;
}

int cmlb_load_deviations_device(cmlb_ctx* c, const float* src) {
    if (!c) return CMLB_EINVAL;
    if (!src) return fail(c, CMLB_EINVAL, "src is NULL");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    StepArgs a = base_args(c);
    launch_encode_deviations(c->p.lattice, c->p.storage, c->f[c->cur], src, a, c->stream);
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "encode kernel launch");
    c->initialised = true;
    c->steps = 0;
    return CMLB_OK;
}

int cmlb_box_filter(cmlb_ctx* c, int factor, void* dst) {
    if (!c) return CMLB_EINVAL;
    if (!dst) return fail(c, CMLB_EINVAL, "dst is NULL");
    if (c->p.lattice != CMLB_D3Q27) return fail(c, CMLB_EINVAL, "box filter is for D3Q27 contexts");
    if (factor < 1 || c->p.nx % factor || c->p.ny % factor || c->p.nz % factor)
        return fail(c, CMLB_EINVAL, "grid sizes must be multiples of the filter factor");
    if (!c->initialised) return fail(c, CMLB_ESTATE, "state not initialised");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    StepArgs a = base_args(c);
    a.src = c->f[c->cur];
    launch_box_filter(c->p.storage, a, factor, static_cast<float*>(dst), c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "box filter launch");
    return CMLB_OK;
}

static int closure_ready(cmlb_ctx* c, bool need_loaded) {
    if (c->p.lattice != CMLB_D3Q27 || c->p.storage != CMLB_F32 || c->p.model != CMLB_MODEL_CM)
        return fail(c, CMLB_EINVAL, "the learned closure needs a D3Q27 CM context with FP32 storage");
    if (need_loaded && !c->closure_loaded) return fail(c, CMLB_ESTATE, "no closure loaded");
    if (hipSetDevice(c->p.device) != hipSuccess) return fail(c, CMLB_EDEVICE, "hipSetDevice failed");
    return CMLB_OK;
}

int cmlb_closure_load(cmlb_ctx* c, const float* params, const float* sigma) {
    if (!c) return CMLB_EINVAL;
    if (!params || !sigma) return fail(c, CMLB_EINVAL, "params and sigma are required");
    int rc = closure_ready(c, false);
    if (rc) return rc;
    for (int k = 0; k < CMLB_CLOSURE_NPARAM; ++k)
        if (!std::isfinite(params[k])) return fail(c, CMLB_EINVAL, "parameters must be finite");
    for (int k = 0; k < 27; ++k)
        if (!(sigma[k] > 0.0f) || !std::isfinite(sigma[k])) return fail(c, CMLB_EINVAL, "sigma must be positive");
    hipError_t e;
    if (!c->cl_params) {
        if ((e = hipMalloc(&c->cl_params, (3 * CMLB_CLOSURE_NPARAM + 32) * sizeof(float))) != hipSuccess ||
            (e = hipMalloc(&c->cl_net, closure_net_bytes())) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, CMLB_ENOMEM, "closure allocation failed");
        }
    }
    float* P = c->cl_params;
    float* sig = P + 3 * CMLB_CLOSURE_NPARAM;
    if ((e = hipMemcpyAsync(P, params, CMLB_CLOSURE_NPARAM * sizeof(float), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copy params");
    if ((e = hipMemsetAsync(P + CMLB_CLOSURE_NPARAM, 0, 2 * CMLB_CLOSURE_NPARAM * sizeof(float), c->stream)) != hipSuccess)
        return hip_fail(c, e, "clear optimiser state");
    if ((e = hipMemcpyAsync(sig, sigma, 27 * sizeof(float), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copy sigma");
    launch_closure_pack(P, sig, c->cl_tie_even, c->cl_net, c->stream);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "pack launch");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "closure load");
    c->closure_loaded = true;
    c->cl_step = 0;
    return CMLB_OK;
}

int cmlb_closure_enable(cmlb_ctx* c, int on) {
    if (!c) return CMLB_EINVAL;
    if (on) {
        int rc = closure_ready(c, true);
        if (rc) return rc;
    }
    c->closure_on = on != 0;
    graph_drop(c);
    return CMLB_OK;
}

int cmlb_closure_tie_even(cmlb_ctx* c, int on) {
    if (!c) return CMLB_EINVAL;
    int rc = closure_ready(c, true);
    if (rc) return rc;
    c->cl_tie_even = on != 0;
    float* P = c->cl_params;
    launch_closure_pack(P, P + 3 * CMLB_CLOSURE_NPARAM, c->cl_tie_even, c->cl_net, c->stream);
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "pack launch");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "tie even");
    return CMLB_OK;
}

int cmlb_closure_get(cmlb_ctx* c, float* params) {
    if (!c) return CMLB_EINVAL;
    if (!params) return fail(c, CMLB_EINVAL, "params is NULL");
    int rc = closure_ready(c, true);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(params, c->cl_params, CMLB_CLOSURE_NPARAM * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy params");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "closure get");
    return CMLB_OK;
}

static int closure_gradient(cmlb_ctx* c, const cmlb_batch* b) {
    if (!b || !b->state || !b->target || b->n_pairs < 1) return fail(c, CMLB_EINVAL, "bad batch");
    if (c->p.nx % 64) return fail(c, CMLB_EINVAL, "closure training needs nx to be a multiple of 64");
    hipError_t e;
    if (!c->cl_partials) {
        c->cl_blocks = 1024;
        if ((e = hipMalloc(&c->cl_partials, (size_t)c->cl_blocks * closure_partial_stride() * sizeof(float))) != hipSuccess ||
            (e = hipMalloc(&c->cl_grad, closure_partial_stride() * sizeof(float))) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, CMLB_ENOMEM, "closure training scratch");
        }
    }
    StepArgs a = base_args(c);
    const float* target = static_cast<const float*>(b->target);
    int mode = 0;
    if (c->cl_objective == CMLB_CLOSURE_OBJ_MOMENTUM) {
        // the closure step of each pair's state, then the momentum mismatch
        // field D that the training kernel takes as its adjoint input
        const uint64_t N = nodes_of(a.g);
        if (b->n_pairs > c->cl_pairs_cap) {
            if (c->cl_f1) (void)hipFree(c->cl_f1);
            if (c->cl_D) (void)hipFree(c->cl_D);
            c->cl_f1 = c->cl_D = nullptr;
            c->cl_pairs_cap = 0;
            if ((e = hipMalloc(&c->cl_f1, (size_t)b->n_pairs * 27 * N * sizeof(float))) != hipSuccess ||
                (e = hipMalloc(&c->cl_D, (size_t)b->n_pairs * 3 * N * sizeof(float))) != hipSuccess) {
                (void)hipGetLastError();
                return fail(c, CMLB_ENOMEM, "momentum objective scratch");
            }
            c->cl_pairs_cap = b->n_pairs;
        }
        for (int64_t k = 0; k < b->n_pairs; ++k) {
            StepArgs sa = a;
            sa.g.plane = N;                    // batch arrays are unpadded [27][z][y][x],
            sa.pitch = (uint32_t)c->p.nx;      // not in the state's own layout
            sa.src = static_cast<const float*>(b->state) + (uint64_t)k * 27 * N;
            sa.dst = c->cl_f1 + (uint64_t)k * 27 * N;
            launch_step_closure(sa, c->cl_net, c->stream);
        }
        launch_closure_momentum(c->cl_f1, target, b->n_pairs, a.g, c->cl_D, c->stream);
        target = c->cl_D;
        mode = 1;
    }
    launch_closure_train(static_cast<const float*>(b->state), target, b->n_pairs, a.g, (float)c->p.rho0,
                         (float)c->omega[2], c->cl_net, c->cl_partials, c->cl_blocks, c->cl_grad, mode, c->stream);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "closure training launch");
    return CMLB_OK;
}

int cmlb_closure_set_objective(cmlb_ctx* c, int kind) {
    if (!c) return CMLB_EINVAL;
    int rc = closure_ready(c, false);
    if (rc) return rc;
    if (kind != CMLB_CLOSURE_OBJ_POPULATIONS && kind != CMLB_CLOSURE_OBJ_MOMENTUM)
        return fail(c, CMLB_EINVAL, "objective must be CMLB_CLOSURE_OBJ_POPULATIONS or CMLB_CLOSURE_OBJ_MOMENTUM");
    c->cl_objective = kind;
    return CMLB_OK;
}

int cmlb_closure_set_adam(cmlb_ctx* c, double beta1, double beta2, double eps) {
    if (!c) return CMLB_EINVAL;
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return fail(c, CMLB_EINVAL, "beta1 and beta2 must lie in [0, 1)");
    if (!(eps >= 1.17549435e-38 && eps <= 3.4e38))
        return fail(c, CMLB_EINVAL, "eps must be a positive normal FP32 number");
    c->cl_beta1 = (float)beta1;
    c->cl_beta2 = (float)beta2;
    c->cl_eps = (float)eps;
    return CMLB_OK;
}

int cmlb_closure_freeze(cmlb_ctx* c, int mask) {
    if (!c) return CMLB_EINVAL;
    if (mask < 0 || mask > 15) return fail(c, CMLB_EINVAL, "freeze mask must lie in [0, 15]");
    c->cl_frozen = mask;
    return CMLB_OK;
}

int cmlb_closure_objective(cmlb_ctx* c, const cmlb_batch* b, float* objective, float* grad) {
    if (!c) return CMLB_EINVAL;
    if (!objective) return fail(c, CMLB_EINVAL, "objective is NULL");
    int rc = closure_ready(c, true);
    if (rc) return rc;
    if ((rc = closure_gradient(c, b))) return rc;
    hipError_t e;
    if ((e = hipMemcpyAsync(objective, c->cl_grad + CMLB_CLOSURE_NPARAM, sizeof(float), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copy objective");
    if (grad && (e = hipMemcpyAsync(grad, c->cl_grad, CMLB_CLOSURE_NPARAM * sizeof(float), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copy gradient");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "closure objective");
    return CMLB_OK;
}

int cmlb_closure_train_step(cmlb_ctx* c, const cmlb_batch* b, float lr, float* objective) {
    if (!c) return CMLB_EINVAL;
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(c, CMLB_EINVAL, "lr must be positive");
    int rc = closure_ready(c, true);
    if (rc) return rc;
    if ((rc = closure_gradient(c, b))) return rc;
    float* P = c->cl_params;
    c->cl_step++;
    launch_closure_adam(P, P + CMLB_CLOSURE_NPARAM, P + 2 * CMLB_CLOSURE_NPARAM, c->cl_grad, lr, c->cl_beta1,
                        c->cl_beta2, c->cl_eps, c->cl_frozen, c->cl_step, c->stream);
    launch_closure_pack(P, P + 3 * CMLB_CLOSURE_NPARAM, c->cl_tie_even, c->cl_net, c->stream);
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "adam launch");
    if (objective) {
        if ((e = hipMemcpyAsync(objective, c->cl_grad + CMLB_CLOSURE_NPARAM, sizeof(float), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
            return hip_fail(c, e, "copy objective");
        if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "train step");
    }
    return CMLB_OK;
}

int cmlb_get_scale(const cmlb_ctx* c, double* scale) {
    if (!c || !scale) return CMLB_EINVAL;
    for (int i = 0; i < c->L.Q; ++i) scale[i] = c->s[i];
    return CMLB_OK;
}

}  // extern "C"
