/* Drives every exported function of the FP64 oracle on small inputs, with
 * buffers of exactly the sizes its Python wrapper allocates, so that a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer reports any
 * out-of-bounds access, use of freed memory or undefined arithmetic.
 * Test infrastructure: compiled together with oracle/cmlb_oracle.c by
 * tests/test_oracle_sanitizers.py; it shares nothing with the HIP library. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int lattice, model, thermal, pad;
    double theta0;
    double omega[8];
    double delta_coef;
} orc_cfg;

int orc_lattice_info(int kind, int *D, int *Q, int *e, double *w, double *r, double *resid);
int orc_hermite(int D, int nmax, const double *xi, double *H);
int orc_symprod(int D, int n, const double *A, int m, const double *B, double *out);
int orc_maxwell_coeffs(int D, int nmax, double rho, const double *u_xi, double theta, double *a);
int orc_equilibrium(int kind, double rho, const double *u_lat, double theta, double *f0);
int orc_collide(const orc_cfg *cfg, int n_nodes, const double *f, double *out);
int orc_collide_definitional(const orc_cfg *cfg, int n_nodes, const double *f, double *out);
int orc_run(const orc_cfg *cfg, long nx, long ny, long nz, double *S, long nsteps, int nthreads);
int orc_step_nodes(const orc_cfg *cfg, long nx, long ny, long nz, const double *S, long n_nodes,
                   const int64_t *nodes, double *out, int nthreads);
int orc_init_equilibrium(const orc_cfg *cfg, long nx, long ny, long nz, const double *rho, const double *u,
                         const double *theta, double *S, int nthreads);
int orc_moments(int kind, long n_nodes, const double *S, double *rho, double *u, double *theta);
int orc_mlp_nparam(void);
int orc_mlp_forward(const double *params, int n, const double *x, double *omega);
int orc_closure_inputs(int n, const double *f, const double *norm, double *x);
int orc_collide_closure(const orc_cfg *cfg, int n, const double *f, const double *params, const double *norm,
                        int tie_even, double *out, double *omega_out);
int orc_closure_loss_grad(const orc_cfg *cfg, int n, const double *f, const double *fbar, const double *params,
                          const double *norm, int tie_even, double *loss_out, double *grad);
int orc_gather_nodes(int kind, long nx, long ny, long nz, const double *S, long n_nodes, const int64_t *nodes,
                     double *out);

static unsigned seed = 12345u;
static double urand(void) { /* uniform in [-1, 1) */
    seed = seed * 1664525u + 1013904223u;
    return ((seed >> 8) & 0xFFFFFF) / 8388608.0 - 1.0;
}

static double *alloc(size_t n) {
    double *p = malloc(n * sizeof(double));
    if (!p) { puts("allocation failed"); exit(2); }
    for (size_t k = 0; k < n; ++k) p[k] = 0.0;
    return p;
}

#define CHECK(call) do { if ((call) != 0) { printf("failed: %s\n", #call); return 1; } } while (0)

static int lattice_runs(int kind) {
    int D, Q, e[37 * 3];
    double w[37], r, resid;
    CHECK(orc_lattice_info(kind, &D, &Q, e, w, &r, &resid));
    const long nx = kind == 1 ? 5 : 7, ny = kind == 1 ? 4 : 6, nz = kind == 1 ? 3 : 1;
    const long n = nx * ny * nz;
    const int models = kind == 2 ? 3 : 1;
    for (int model = 0; model < models; ++model)
        for (int thermal = 0; thermal < (kind == 2 ? 2 : 1); ++thermal) {
            orc_cfg cfg = {kind, model, thermal, 0, 1.0, {0, 0, 1.6, 1.1, 1.3, 0.9, 1.2, 1.0}, 6.0};
            double *rho = alloc(n), *u = alloc((size_t)D * n), *th = alloc(n);
            for (long k = 0; k < n; ++k) {
                rho[k] = 1.0 + 0.02 * urand();
                th[k] = 1.0 + 0.02 * urand();
                for (int d = 0; d < D; ++d) u[d * n + k] = 0.04 * urand();
            }
            double *S = alloc((size_t)Q * n);
            CHECK(orc_init_equilibrium(&cfg, nx, ny, nz, rho, u, thermal ? th : NULL, S, 1));
            for (long k = 0; k < (long)Q * n; ++k) S[k] *= 1.0 + 0.01 * urand();
            CHECK(orc_run(&cfg, nx, ny, nz, S, 3, 1));
            const int64_t nodes[3] = {0, n - 1, n / 2};
            double *out = alloc(3 * (size_t)Q), *pulled = alloc(3 * (size_t)Q), *col = alloc(3 * (size_t)Q);
            CHECK(orc_step_nodes(&cfg, nx, ny, nz, S, 3, nodes, out, 1));
            CHECK(orc_gather_nodes(kind, nx, ny, nz, S, 3, nodes, pulled));
            CHECK(orc_collide(&cfg, 3, pulled, col));
            CHECK(orc_collide_definitional(&cfg, 3, pulled, col));
            CHECK(orc_moments(kind, n, S, rho, u, th));
            for (long k = 0; k < n; ++k)
                if (!isfinite(rho[k])) { puts("non-finite density"); return 1; }
            free(rho); free(u); free(th); free(S); free(out); free(pulled); free(col);
        }
    double f0[37], ul[3] = {0.03, -0.02, 0.01};
    CHECK(orc_equilibrium(kind, 1.01, ul, 1.02, f0));
    return 0;
}

int main(void) {
    for (int kind = 0; kind < 3; ++kind)
        if (lattice_runs(kind)) return 1;

    double xi[3] = {0.3, -1.2, 0.7};
    double *H = alloc(1 + 3 + 9 + 27 + 81);                /* ranks 0..4 in three dimensions */
    CHECK(orc_hermite(3, 4, xi, H));
    double *A = alloc(9), *B = alloc(9), *AB = alloc(81);  /* Sym(A (x) B), ranks 2 + 2 */
    for (int k = 0; k < 9; ++k) { A[k] = urand(); B[k] = urand(); }
    CHECK(orc_symprod(3, 2, A, 2, B, AB));
    double u2[3] = {0.1, -0.2, 0.0};
    double *a = alloc(1 + 2 + 4 + 8 + 16);                 /* ranks 0..4 in two dimensions */
    CHECK(orc_maxwell_coeffs(2, 4, 1.1, u2, 1.05, a));

    const int np = orc_mlp_nparam(), nn = 5;
    double *P = alloc(np), *norm = alloc(27), *f = alloc(27 * nn), *fb = alloc(27 * nn);
    double *x = alloc(27 * nn), *om = alloc(4 * nn), *fo = alloc(27 * nn), *grad = alloc(np), loss = 0.0;
    for (int k = 0; k < np; ++k) P[k] = 0.3 * urand();
    for (int k = 0; k < 27; ++k) norm[k] = 0.01 + 0.005 * (urand() + 1.0);
    int D, Q, e[37 * 3];
    double w[37], r, resid;
    CHECK(orc_lattice_info(1, &D, &Q, e, w, &r, &resid));
    for (int k = 0; k < nn; ++k)
        for (int i = 0; i < 27; ++i) {
            f[27 * k + i] = w[i] * (1.0 + 0.05 * urand());
            fb[27 * k + i] = w[i] * (1.0 + 0.05 * urand());
        }
    orc_cfg cfg = {1, 0, 0, 0, 1.0, {0, 0, 1.6, 1.0, 1.0, 1.0, 1.0, 1.0}, 6.0};
    CHECK(orc_closure_inputs(nn, f, norm, x));
    CHECK(orc_mlp_forward(P, nn, x, om));
    for (int tie = 0; tie < 2; ++tie) {
        CHECK(orc_collide_closure(&cfg, nn, f, P, norm, tie, fo, om));
        CHECK(orc_closure_loss_grad(&cfg, nn, f, fb, P, norm, tie, &loss, grad));
    }
    if (!isfinite(loss)) { puts("non-finite loss"); return 1; }
    free(H); free(A); free(B); free(AB); free(a);
    free(P); free(norm); free(f); free(fb); free(x); free(om); free(fo); free(grad);
    puts("oracle sanitize driver: ok");
    return 0;
}
