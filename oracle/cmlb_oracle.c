/*
 * FP64 CPU oracle for the central-moment multiple-relaxation-time (CM-MRT)
 * lattice Boltzmann update of X. Shan, "A central-moment multiple-relaxation-
 * time collision model" (arXiv:1808.04406).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * execute this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the HIP library; it derives every table itself.
 *
 * Everything is double precision, written for readability rather than speed:
 * symmetric tensors are stored with all D^n index components, symmetrisation
 * averages over all n! index permutations, and linear systems are solved by
 * Gaussian elimination with partial pivoting.
 *
 * Units.  Lattice velocities e_i are integer vectors; the abscissas of the
 * quadrature are xi_i = r e_i (Sec. II.A, eq:quad).  The Hermite machinery
 * works in xi-units, where the reference temperature is theta = 1.  The API
 * exchanges velocities in lattice units (cells per step): u_lat = u_xi / r.
 *
 * Parity: every function below is pinned by the CPU test suite against
 * closed forms, library quadrature, brute force or the paper's printed
 * constants; the learned-closure network (not in the paper) is pinned by an
 * independent FP64 implementation of its layers and by finite differences
 * of its training objective.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQ 37
#define ORC_MAXN 6   /* highest tensor rank handled */

/* Lattice kinds.  ORC_D2Q37 is the ninth-degree 37-velocity rule on the
 * shells with |e|^2 <= 10 (called E9 A here); E9 B-D and E7 A-D are the other
 * minimal on-lattice rules of Sec. III.A (Fig. 2), see make_hermite_rule. */
enum { ORC_D2Q9 = 0, ORC_D3Q27 = 1, ORC_D2Q37 = 2, ORC_E9B = 3, ORC_E9C = 4, ORC_E9D = 5,
       ORC_E7A = 6, ORC_E7B = 7, ORC_E7C = 8, ORC_E7D = 9, ORC_NKIND = 10 };
enum { ORC_CM = 0, ORC_RAW_MRT = 1, ORC_REG_BGK = 2 };

typedef struct {
    int D, Q;
    int e[ORC_MAXQ][3];
    double w[ORC_MAXQ];
    double r;
    int N;                      /* Hermite truncation N = M (0: complete tensor-product basis) */
    double H[ORC_MAXQ][31];     /* H^(0..4)(xi_i) of a Hermite-truncated 2D lattice */
} orc_lattice;

/* Collision configuration (passed from Python as a flat struct). */
typedef struct {
    int lattice;       /* ORC_D2Q9 / ORC_D3Q27 / ORC_D2Q37 and the other 2D rules */
    int model;         /* ORC_CM (this paper), ORC_RAW_MRT (eq:regnmrt, right), ORC_REG_BGK (eq:lbgk-reg) */
    int thermal;       /* 1: theta is computed from f; 0: theta is frozen at theta0 (Sec. III.B) */
    int pad;
    double theta0;     /* frozen temperature (isothermal runs) */
    double omega[8];   /* omega[n]: relaxation frequency of order n; n = 0, 1 unused */
    double delta_coef; /* coefficient of the delta term in the fourth-order relaxation; 6 satisfies eq:omega, 72 is as printed */
} orc_cfg;

/* ------------------------------------------------------------------------- */
/* Dense linear algebra                                                      */
/* ------------------------------------------------------------------------- */

/* Solve A x = b in place (A is n x n row-major and is destroyed; b becomes x).
 * Returns 0, or -1 if A is numerically singular. */
static int solve_dense(int n, double *A, double *b)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); piv = i; }
        if (best == 0.0) return -1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double m = A[i * n + k] / A[k * n + k];
            if (m == 0.0) continue;
            for (int j = k; j < n; ++j) A[i * n + j] -= m * A[k * n + j];
            b[i] -= m * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * b[j];
        b[k] = s / A[k * n + k];
    }
    return 0;
}

static double determinant(int n, double *A)
{
    double det = 1.0;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (A[piv * n + k] == 0.0) return 0.0;
        if (piv != k) {
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            det = -det;
        }
        det *= A[k * n + k];
        for (int i = k + 1; i < n; ++i) {
            double m = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= m * A[k * n + j];
        }
    }
    return det;
}

static double factorial(int n) { double f = 1.0; for (int k = 2; k <= n; ++k) f *= k; return f; }
static double binom(int n, int k) { return factorial(n) / (factorial(k) * factorial(n - k)); }
static int ipow(int b, int e) { int p = 1; while (e-- > 0) p *= b; return p; }

/* ------------------------------------------------------------------------- */
/* Lattices (quadratures, Sec. II.A eq:quad)                                  */
/* ------------------------------------------------------------------------- */

/* 1D Gaussian moment E[X^p], X ~ N(0,1): (p-1)!! for even p, 0 for odd p. */
static double gauss_moment(int p)
{
    if (p % 2) return 0.0;
    double m = 1.0;
    for (int k = p - 1; k > 0; k -= 2) m *= k;
    return m;
}

/* All distinct images of (a, b) under sign changes and axis exchange. */
static int shell_images(int a, int b, int out[8][2])
{
    int n = 0;
    int base[2][2] = {{a, b}, {b, a}};
    for (int t = 0; t < 2; ++t)
        for (int sx = 1; sx >= -1; sx -= 2)
            for (int sy = 1; sy >= -1; sy -= 2) {
                int x = sx * base[t][0], y = sy * base[t][1], dup = 0;
                for (int k = 0; k < n; ++k) if (out[k][0] == x && out[k][1] == y) dup = 1;
                if (!dup) { out[n][0] = x; out[n][1] = y; ++n; }
            }
    return n;
}

/* On-lattice 2D rules from their velocity shells (Sec. II.A, eq:quad).  A
 * rule of degree Q integrates every polynomial of degree <= Q against the
 * Gaussian weight; with the symmetry of the shells (all sign changes and the
 * axis exchange) the odd moments vanish and the conditions are
 * sum_i w_i xi_x^p xi_y^q = E[X^p] E[Y^q] for even p >= q, p + q < Q.  The
 * shell weights and the scale r solve them: with x = 1/r^2 they read
 * A w = b(x), b_k = E[X^p]E[Y^q] x^((p+q)/2), which has a solution where
 * det[A | b(x)] = 0.  The roots are located by a scan over x and bisection;
 * the first root whose weights are all positive is taken.  The weights
 * come from a square subsystem (the last condition dropped), and the
 * dropped condition is the consistency check (resid_out).
 *
 * The rules of Sec. III.A (Fig. 2) are the minimal ones: 17 velocities for
 * degree 7, 37 for degree 9.  A degree-7 rule has 6 conditions, so rest plus
 * four 4-velocity shells; a degree-9 rule has 9, so rest plus five
 * 4-velocity and two 8-velocity shells.  Among shells whose velocity
 * components are at most 3, moment matching yields exactly four positive
 * rules of each degree, matching the paper's count (their A-D letters are
 * not recoverable from the text; the order here is by the shell lists):
 *   E9 A = D2Q37: (1,0),(2,0),(3,0),(1,1),(2,2),(2,1),(3,1)   (|e|^2 <= 10)
 *   E9 B:         (1,0),(2,0),(3,0),(1,1),(2,2),(2,1),(3,2)
 *   E9 C:         (1,0),(2,0),(3,0),(1,1),(3,3),(2,1),(3,1)
 *   E9 D:         (1,0),(2,0),(3,0),(1,1),(3,3),(2,1),(3,2)
 *   E7 A:         (1,0),(3,0),(1,1),(2,2)
 *   E7 B:         (1,0),(3,0),(1,1),(3,3)
 *   E7 C:         (2,0),(3,0),(1,1),(3,3)
 *   E7 D:         (3,0),(1,1),(2,2),(3,3)
 * The degree-9 rules carry the order-4 truncation N = M = 4 of Sec. III; a
 * degree-7 rule resolves eq:an exactly for orders up to 7 - N, so it
 * carries N = M = 3. */
static const int g_shells[ORC_NKIND][8][2] = {
    [ORC_D2Q37] = {{0,0},{1,0},{2,0},{3,0},{1,1},{2,2},{2,1},{3,1}},
    [ORC_E9B]   = {{0,0},{1,0},{2,0},{3,0},{1,1},{2,2},{2,1},{3,2}},
    [ORC_E9C]   = {{0,0},{1,0},{2,0},{3,0},{1,1},{3,3},{2,1},{3,1}},
    [ORC_E9D]   = {{0,0},{1,0},{2,0},{3,0},{1,1},{3,3},{2,1},{3,2}},
    [ORC_E7A]   = {{0,0},{1,0},{3,0},{1,1},{2,2}},
    [ORC_E7B]   = {{0,0},{1,0},{3,0},{1,1},{3,3}},
    [ORC_E7C]   = {{0,0},{2,0},{3,0},{1,1},{3,3}},
    [ORC_E7D]   = {{0,0},{3,0},{1,1},{2,2},{3,3}},
};

static int make_hermite_rule(int kind, orc_lattice *L, double *resid_out)
{
    const int degree = (kind >= ORC_E7A) ? 7 : 9;
    const int ns = (degree == 7) ? 5 : 8;
    /* conditions (p, q), p >= q even, p + q < degree; the last is dropped from the square system */
    static const int mons9[9][2] = {{0,0},{2,0},{4,0},{2,2},{6,0},{4,2},{6,2},{4,4},{8,0}};
    static const int mons7[6][2] = {{0,0},{2,0},{4,0},{2,2},{4,2},{6,0}};
    const int (*mons)[2] = (degree == 7) ? mons7 : mons9;
    const int nm = ns + 1;
    int img[8][8][2], nimg[8];
    double A[9][8];
    for (int k = 0; k < ns; ++k) nimg[k] = shell_images(g_shells[kind][k][0], g_shells[kind][k][1], img[k]);
    for (int k = 0; k < nm; ++k)
        for (int c = 0; c < ns; ++c) {
            double acc = 0.0;
            for (int j = 0; j < nimg[c]; ++j)
                acc += pow(img[c][j][0], mons[k][0]) * pow(img[c][j][1], mons[k][1]);
            A[k][c] = acc;
        }
    double M[81];
#define AUGDET(x, out) do {                                                   \
        for (int k_ = 0; k_ < nm; ++k_) {                                     \
            for (int s_ = 0; s_ < ns; ++s_) M[k_ * nm + s_] = A[k_][s_];      \
            M[k_ * nm + ns] = gauss_moment(mons[k_][0]) * gauss_moment(mons[k_][1]) \
                          * pow((x), (mons[k_][0] + mons[k_][1]) / 2);        \
        }                                                                     \
        (out) = determinant(nm, M);                                           \
    } while (0)
    double wv[8], x = 0.0;
    int found = 0;
    double prev_x = 0.05, prev_f;
    AUGDET(prev_x, prev_f);
    for (int k = 1; k <= 4000 && !found; ++k) {
        double xs = 0.05 + k * 0.001, fx;
        AUGDET(xs, fx);
        if ((fx < 0) != (prev_f < 0)) {
            double lo = prev_x, hi = xs, flo = prev_f;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi), fm;
                AUGDET(mid, fm);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
            }
            x = 0.5 * (lo + hi);
            double S[64];
            for (int r_ = 0; r_ < ns; ++r_) {
                for (int c = 0; c < ns; ++c) S[r_ * ns + c] = A[r_][c];
                wv[r_] = gauss_moment(mons[r_][0]) * gauss_moment(mons[r_][1]) * pow(x, (mons[r_][0] + mons[r_][1]) / 2);
            }
            int pos = !solve_dense(ns, S, wv);
            for (int c = 0; c < ns && pos; ++c) pos = wv[c] > 0.0;
            found = pos;
        }
        prev_x = xs; prev_f = fx;
    }
#undef AUGDET
    if (!found) return -1;
    double rlast = -gauss_moment(mons[ns][0]) * gauss_moment(mons[ns][1]) * pow(x, (mons[ns][0] + mons[ns][1]) / 2);
    for (int c = 0; c < ns; ++c) rlast += A[ns][c] * wv[c];
    if (resid_out) *resid_out = rlast;
    /* populations ordered by (e_y, e_x) lexicographically */
    L->D = 2; L->Q = (degree == 7) ? 17 : 37; L->r = 1.0 / sqrt(x); L->N = (degree == 7) ? 3 : 4;
    int q = 0;
    for (int ey = -3; ey <= 3; ++ey)
        for (int ex = -3; ex <= 3; ++ex)
            for (int c = 0; c < ns; ++c)
                for (int j = 0; j < nimg[c]; ++j)
                    if (img[c][j][0] == ex && img[c][j][1] == ey) {
                        L->e[q][0] = ex; L->e[q][1] = ey; L->e[q][2] = 0;
                        L->w[q] = wv[c];
                        ++q;
                    }
    return q == L->Q ? 0 : -1;
}

/* D2Q9 and D3Q27: the tensor products of the three-point Gauss-Hermite rule
 * {0, +-sqrt(3)} with weights {2/3, 1/6, 1/6}; degree 5 per axis.  Populations
 * are ordered lexicographically with e_x fastest, i = (ex+1) + 3(ey+1) + 9(ez+1). */
static void make_tensor_lattice(int D, orc_lattice *L)
{
    static const double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    L->D = D; L->Q = ipow(3, D); L->r = sqrt(3.0);
    for (int i = 0; i < L->Q; ++i) {
        int ix = i % 3, iy = (i / 3) % 3, iz = (D == 3) ? i / 9 : 1;
        L->e[i][0] = ix - 1; L->e[i][1] = iy - 1; L->e[i][2] = (D == 3) ? iz - 1 : 0;
        L->w[i] = w1[ix] * w1[iy] * (D == 3 ? w1[iz] : 1.0);
    }
    L->N = 0;
}

static int get_lattice(int kind, orc_lattice *L)
{
    if (kind == ORC_D2Q9) { make_tensor_lattice(2, L); return 0; }
    if (kind == ORC_D3Q27) { make_tensor_lattice(3, L); return 0; }
    if (kind >= ORC_D2Q37 && kind < ORC_NKIND) return make_hermite_rule(kind, L, NULL);
    return -1;
}

/* Lattice tables are built once per kind. */
static orc_lattice g_lat[ORC_NKIND];
static int g_lat_ok[ORC_NKIND];

static void build_tables(orc_lattice *L, int kind);

/* Lattice and its Hermite tables; built on first use, before any parallel region. */
static const orc_lattice *lattice(int kind)
{
    if (kind < 0 || kind >= ORC_NKIND) return NULL;
    if (!g_lat_ok[kind]) {
        orc_lattice L;
        if (get_lattice(kind, &L)) return NULL;
        g_lat[kind] = L;
        build_tables(&g_lat[kind], kind);
        g_lat_ok[kind] = 1;
    }
    return &g_lat[kind];
}

int orc_lattice_info(int kind, int *D, int *Q, int *e, double *w, double *r, double *resid)
{
    const orc_lattice *L = lattice(kind);
    if (!L) return -1;
    *D = L->D; *Q = L->Q; *r = L->r;
    for (int i = 0; i < L->Q; ++i) {
        w[i] = L->w[i];
        for (int d = 0; d < 3; ++d) e[3 * i + d] = L->e[i][d];
    }
    if (resid) {
        *resid = 0.0;
        if (kind >= ORC_D2Q37) { orc_lattice T; make_hermite_rule(kind, &T, resid); }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Symmetric tensors (Sec. II, definitions of Sym and the symmetric product)  */
/* ------------------------------------------------------------------------- */
/* A rank-n tensor in D dimensions is stored with all D^n components, index
 * (i_0, ..., i_{n-1}) at offset sum_k i_k D^(n-1-k). */

static int next_perm(int n, int *p)
{
    int i = n - 2;
    while (i >= 0 && p[i] >= p[i + 1]) --i;
    if (i < 0) return 0;
    int j = n - 1;
    while (p[j] <= p[i]) --j;
    int t = p[i]; p[i] = p[j]; p[j] = t;
    for (int a = i + 1, b = n - 1; a < b; ++a, --b) { t = p[a]; p[a] = p[b]; p[b] = t; }
    return 1;
}

/* Sym(A): average of A over the n! permutations of its indices. */
static void t_sym(int D, int n, const double *A, double *out)
{
    int size = ipow(D, n);
    if (n <= 1) { memcpy(out, A, sizeof(double) * size); return; }
    double nf = factorial(n);
    for (int I = 0; I < size; ++I) {
        int idx[ORC_MAXN], perm[ORC_MAXN];
        for (int k = n - 1, t = I; k >= 0; --k) { idx[k] = t % D; t /= D; }
        for (int k = 0; k < n; ++k) perm[k] = k;
        double acc = 0.0;
        do {
            int J = 0;
            for (int k = 0; k < n; ++k) J = J * D + idx[perm[k]];
            acc += A[J];
        } while (next_perm(n, perm));
        out[I] = acc / nf;
    }
}

/* Ordinary tensor product A (rank n) (x) B (rank m). */
static void t_outer(int D, int n, const double *A, int m, const double *B, double *out)
{
    int sa = ipow(D, n), sb = ipow(D, m);
    for (int i = 0; i < sa; ++i)
        for (int j = 0; j < sb; ++j) out[i * sb + j] = A[i] * B[j];
}

/* Symmetric product AB = Sym(A (x) B). */
static void t_symprod(int D, int n, const double *A, int m, const double *B, double *out)
{
    double tmp[729];
    t_outer(D, n, A, m, B, tmp);
    t_sym(D, n + m, tmp, out);
}

static double t_contract(int D, int n, const double *A, const double *B)
{
    int s = ipow(D, n);
    double acc = 0.0;
    for (int i = 0; i < s; ++i) acc += A[i] * B[i];
    return acc;
}

static void t_delta(int D, double *out)
{
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) out[i * D + j] = (i == j) ? 1.0 : 0.0;
}

/* Offsets of ranks 0..nmax packed one after another. */
static int t_offset(int D, int n) { int o = 0; for (int k = 0; k < n; ++k) o += ipow(D, k); return o; }

/* Tensor Hermite polynomials H^(0..nmax)(xi) by the recursion of Appendix A:
 * xi H^(n) = H^(n+1) + n delta H^(n-1), all products symmetric. */
static void hermite_tensors(int D, int nmax, const double *xi, double *H)
{
    double delta[9], t1[729], t2[729];
    t_delta(D, delta);
    H[0] = 1.0;
    if (nmax >= 1) for (int d = 0; d < D; ++d) H[1 + d] = xi[d];
    for (int n = 1; n < nmax; ++n) {
        double *Hn = H + t_offset(D, n), *Hm = H + t_offset(D, n - 1), *Hp = H + t_offset(D, n + 1);
        t_symprod(D, 1, xi, n, Hn, t1);
        t_symprod(D, 2, delta, n - 1, Hm, t2);
        int s = ipow(D, n + 1);
        for (int i = 0; i < s; ++i) Hp[i] = t1[i] - n * t2[i];
    }
}

int orc_hermite(int D, int nmax, const double *xi, double *H)
{
    if (D < 1 || D > 3 || nmax < 0 || nmax > ORC_MAXN) return -1;
    hermite_tensors(D, nmax, xi, H);
    return 0;
}

int orc_symprod(int D, int n, const double *A, int m, const double *B, double *out)
{
    if (n + m > ORC_MAXN) return -1;
    t_symprod(D, n, A, m, B, out);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Maxwellian Hermite coefficients (eq:maxwellian, Appendix A eq:trans-a)     */
/* ------------------------------------------------------------------------- */
/* In the frame moving with u the Maxwellian of temperature theta has Hermite
 * coefficients b^(0) = rho, b^(1) = b^(3) = 0, b^(2) = rho (theta-1) delta,
 * b^(4) = 3 rho (theta-1)^2 delta delta (Gaussian moments of H^(n)(c)).  The
 * absolute-frame coefficients follow from the binomial transform
 * a^(n) = sum_i C(n,i) b^(i) u^(n-i). */
static void maxwell_coeffs(int D, int nmax, double rho, const double *u_xi, double theta, double *a)
{
    double b[1 + 3 + 9 + 27 + 81];
    double delta[9] = {0}, dd[81];
    t_delta(D, delta);
    t_symprod(D, 2, delta, 2, delta, dd);
    memset(b, 0, sizeof(b));
    b[t_offset(D, 0)] = rho;
    if (nmax >= 2) for (int i = 0; i < D * D; ++i) b[t_offset(D, 2) + i] = rho * (theta - 1.0) * delta[i];
    if (nmax >= 4) for (int i = 0; i < ipow(D, 4); ++i) b[t_offset(D, 4) + i] = 3.0 * rho * (theta - 1.0) * (theta - 1.0) * dd[i];
    /* powers u^k as symmetric tensors */
    double upow[5][81];
    upow[0][0] = 1.0;
    for (int k = 1; k <= nmax; ++k) t_symprod(D, k - 1, upow[k - 1], 1, u_xi, upow[k]);
    for (int n = 0; n <= nmax; ++n) {
        double *an = a + t_offset(D, n);
        int s = ipow(D, n);
        for (int j = 0; j < s; ++j) an[j] = 0.0;
        for (int i = 0; i <= n; ++i) {
            double tmp[729];
            t_symprod(D, i, b + t_offset(D, i), n - i, upow[n - i], tmp);
            double c = binom(n, i);
            for (int j = 0; j < s; ++j) an[j] += c * tmp[j];
        }
    }
}

int orc_maxwell_coeffs(int D, int nmax, double rho, const double *u_xi, double theta, double *a)
{
    if (nmax > 4) return -1;
    maxwell_coeffs(D, nmax, rho, u_xi, theta, a);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Moments of one node (Sec. II.A, eq. after eq:fi)                           */
/* ------------------------------------------------------------------------- */
static void node_moments(const orc_lattice *L, const double *f, double *rho, double *u_xi, double *theta)
{
    double m0 = 0.0, m1[3] = {0, 0, 0}, m2 = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        double xi2 = 0.0;
        m0 += f[i];
        for (int d = 0; d < L->D; ++d) {
            double xi = L->r * L->e[i][d];
            m1[d] += f[i] * xi;
            xi2 += xi * xi;
        }
        m2 += f[i] * xi2;
    }
    *rho = m0;
    double uu = 0.0;
    for (int d = 0; d < 3; ++d) { u_xi[d] = (d < L->D) ? m1[d] / m0 : 0.0; uu += u_xi[d] * u_xi[d]; }
    /* rho (u^2 + D theta) = sum f xi^2 */
    *theta = (m2 / m0 - uu) / L->D;
}

/* ------------------------------------------------------------------------- */
/* Per-axis (tensor-product) Hermite basis for D2Q9 and D3Q27 (Sec. II.A)     */
/* ------------------------------------------------------------------------- */
/* On the lattices {-1,0,1}^D the complete set of Q functions used is
 * H_p(xi) = prod_d He_{p_d}(xi_d), p_d <= 2, with He_0 = 1, He_1 = x,
 * He_2 = x^2 - 1 (H^(0..2) of Appendix A in one dimension).  They are the
 * components of the tensor Hermite polynomials with at most two equal
 * indices and are orthogonal under the quadrature with norm prod p_d!. */
static double he1d(int p, double x)
{
    /* He_{p+1} = x He_p - p He_{p-1} (the one-dimensional recursion) */
    double hm = 1.0, h = x;
    if (p == 0) return 1.0;
    for (int k = 1; k < p; ++k) { double hn = x * h - k * hm; hm = h; h = hn; }
    return h;
}

static int n_tp(int D) { return ipow(3, D); }
static void tp_index(int D, int p, int *pd) { pd[0] = p % 3; pd[1] = (p / 3) % 3; pd[2] = (D == 3) ? p / 9 : 0; }

static double tp_hermite(int D, int p, const double *xi);

/* H_p(xi_i) for every basis function p and velocity i, built once per lattice. */
static double g_Htp[2][27][27];
static int g_Htp_ok[2];

static const double (*tp_table(const orc_lattice *L))[27]
{
    int k = (L->D == 3) ? 1 : 0;
    if (!g_Htp_ok[k]) {
        for (int p = 0; p < n_tp(L->D); ++p)
            for (int i = 0; i < L->Q; ++i) {
                double xi[3] = {L->r * L->e[i][0], L->r * L->e[i][1], L->r * L->e[i][2]};
                g_Htp[k][p][i] = tp_hermite(L->D, p, xi);
            }
        g_Htp_ok[k] = 1;
    }
    return (const double (*)[27])g_Htp[k];
}

static double tp_hermite(int D, int p, const double *xi)
{
    int pd[3];
    tp_index(D, p, pd);
    double h = 1.0;
    for (int d = 0; d < D; ++d) h *= he1d(pd[d], xi[d]);
    return h;
}

/* Per-axis 3x3 map from Hermite coefficients (He_0..He_2 in the absolute
 * frame) to central monomial moments (c^0, c^1, c^2), c = xi - u.  Built from
 * eq:binomial-transform, He_k(c) = sum_i (-1)^(k-i) C(k,i) He_i(xi) u^(k-i),
 * and eq:hermite-r, c^2 = He_2(c) + He_0(c). */
static void axis_herm_to_central(double u, double P[3][3])
{
    double B[3][3] = {{0}};  /* He_k(c) in terms of He_i(xi) */
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i <= k; ++i) B[k][i] = ((k - i) % 2 ? -1.0 : 1.0) * binom(k, i) * pow(u, k - i);
    double Mh[3][3] = {{1, 0, 0}, {0, 1, 0}, {1, 0, 1}};  /* c^k in terms of He_j(c) */
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += Mh[k][j] * B[j][i];
            P[k][i] = s;
        }
}

/* Inverse of the above: central monomials back to absolute-frame Hermite
 * coefficients, from He_2(c) = c^2 - 1 and He_n(xi) = sum_i C(n,i) He_i(c) u^(n-i). */
static void axis_central_to_herm(double u, double P[3][3])
{
    double Hm[3][3] = {{1, 0, 0}, {0, 1, 0}, {-1, 0, 1}};  /* He_k(c) in terms of c^j */
    double Bi[3][3] = {{0}};                                /* He_k(xi) in terms of He_i(c) */
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i <= k; ++i) Bi[k][i] = binom(k, i) * pow(u, k - i);
    /* a_xi[k] = sum f He_k(xi) = sum_i Bi[k][i] b[i], b[i] = sum f He_i(c) = sum_j Hm[i][j] kappa[j] */
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) s += Bi[k][i] * Hm[i][j];
            P[k][j] = s;
        }
}

/* Coefficient-space maps are linear over the basis; on the tensor-product
 * basis a coefficient vector indexed by p transforms with the Kronecker
 * product of the per-axis maps. */
static void tp_apply(int D, const double P[3][3][3], const double *in, double *out)
{
    int n = n_tp(D);
    for (int p = 0; p < n; ++p) {
        int pd[3];
        tp_index(D, p, pd);
        double acc = 0.0;
        for (int q = 0; q < n; ++q) {
            int qd[3];
            tp_index(D, q, qd);
            double m = 1.0;
            for (int d = 0; d < D; ++d) m *= P[d][pd[d]][qd[d]];
            acc += m * in[q];
        }
        out[p] = acc;
    }
}

static int tp_order(int D, int p) { int pd[3]; tp_index(D, p, pd); return pd[0] + pd[1] + pd[2]; }
static double tp_norm(int D, int p) { int pd[3]; tp_index(D, p, pd); double n = 1.0; for (int d = 0; d < D; ++d) n *= factorial(pd[d]); return n; }

/* Hermite coefficients on the tensor-product basis of a complete-basis
 * equilibrium: a_p = rho prod_d E[He_{p_d}(X_d)], X_d ~ N(u_d, theta), i.e.
 * per axis 1, u, u^2 + theta - 1 (the components of eq:trans-a applied to the
 * relative-frame Maxwellian coefficients). */
static void tp_maxwell(int D, double rho, const double *u_xi, double theta, double *a)
{
    for (int p = 0; p < n_tp(D); ++p) {
        int pd[3];
        tp_index(D, p, pd);
        double v = rho;
        for (int d = 0; d < D; ++d) {
            double u = u_xi[d];
            v *= (pd[d] == 0) ? 1.0 : (pd[d] == 1 ? u : u * u + theta - 1.0);
        }
        a[p] = v;
    }
}

/* ------------------------------------------------------------------------- */
/* Equilibria                                                                */
/* ------------------------------------------------------------------------- */

/* Discrete equilibrium f0_i, eq:fi applied to the Maxwellian coefficients:
 *   D2Q9/D3Q27: complete tensor-product basis (every resolved central moment
 *               is the Maxwellian's);
 *   2D rules:   Hermite truncation at order M = N of the lattice (4 on the
 *               37-velocity rules, 3 on the 17-velocity rules; Sec. II.B). */
static void equilibrium(const orc_lattice *L, int kind, double rho, const double *u_xi, double theta, double *f0)
{
    (void)kind;
    if (L->N > 0) {
        const int D = 2, M = L->N;
        double a[1 + 2 + 4 + 8 + 16];
        maxwell_coeffs(D, M, rho, u_xi, theta, a);
        for (int i = 0; i < L->Q; ++i) {
            const double *H = L->H[i];  /* H^(0..4)(xi_i) */
            double s = 0.0;
            for (int n = 0; n <= M; ++n) s += t_contract(D, n, a + t_offset(D, n), H + t_offset(D, n)) / factorial(n);
            f0[i] = L->w[i] * s;
        }
    } else {
        int D = L->D;
        double a[27];
        const double (*Ht)[27] = tp_table(L);
        tp_maxwell(D, rho, u_xi, theta, a);
        for (int i = 0; i < L->Q; ++i) {
            double s = 0.0;
            for (int p = 0; p < n_tp(D); ++p) s += a[p] * Ht[p][i] / tp_norm(D, p);
            f0[i] = L->w[i] * s;
        }
    }
}

int orc_equilibrium(int kind, double rho, const double *u_lat, double theta, double *f0)
{
    const orc_lattice *L = lattice(kind);
    if (!L) return -1;
    double u_xi[3] = {0, 0, 0};
    for (int d = 0; d < L->D; ++d) u_xi[d] = L->r * u_lat[d];
    equilibrium(L, kind, rho, u_xi, theta, f0);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Collision, D2Q9 / D3Q27 (complete basis)                                  */
/* ------------------------------------------------------------------------- */

/* Paper's route (Sec. II.C, last paragraph): f1 = f - f0 -> Hermite
 * coefficients a1 (eq:an) -> a_Omega -> Omega_i (eq:fi) -> f* = f^ + Omega.
 * On the complete basis f^ = f, and eq:omega "for all n" fixes a_Omega:
 * map a1 to central monomial moments with the binomial transform, scale
 * each by -omega_{|p|}, and map back.  On the raw-MRT switch a_Omega =
 * -omega_n a1 (eq:regnmrt); on regularised BGK every order uses omega[2]. */
static void collide_tp(const orc_lattice *L, const orc_cfg *cfg, const double *f, double *out)
{
    int D = L->D, n = n_tp(D);
    double rho, u[3], th;
    node_moments(L, f, &rho, u, &th);
    if (!cfg->thermal) th = cfg->theta0;
    const double (*Ht)[27] = tp_table(L);
    double af[27], aeq[27], a1[27], k1[27], kO[27], aO[27];
    for (int p = 0; p < n; ++p) {
        double s = 0.0;
        for (int i = 0; i < L->Q; ++i) s += f[i] * Ht[p][i];   /* eq:an */
        af[p] = s;
    }
    tp_maxwell(D, rho, u, th, aeq);
    for (int p = 0; p < n; ++p) a1[p] = af[p] - aeq[p];
    double om[8];
    for (int k = 0; k < 8; ++k) om[k] = (cfg->model == ORC_REG_BGK) ? cfg->omega[2] : cfg->omega[k];
    om[0] = om[1] = 0.0;  /* mass and momentum are conserved: a1 vanishes there */
    if (cfg->model == ORC_CM) {
        double P[3][3][3], Pi[3][3][3];
        for (int d = 0; d < 3; ++d) { axis_herm_to_central(u[d], P[d]); axis_central_to_herm(u[d], Pi[d]); }
        tp_apply(D, (const double(*)[3][3])P, a1, k1);
        for (int p = 0; p < n; ++p) kO[p] = -om[tp_order(D, p)] * k1[p];
        tp_apply(D, (const double(*)[3][3])Pi, kO, aO);
    } else {
        for (int p = 0; p < n; ++p) aO[p] = -om[tp_order(D, p)] * a1[p];
    }
    for (int i = 0; i < L->Q; ++i) {
        double s = 0.0;
        for (int p = 0; p < n; ++p) s += (af[p] + aO[p]) * Ht[p][i] / tp_norm(D, p);   /* eq:fi */
        out[i] = L->w[i] * s;
    }
}

/* Definition (eq:omega for every central moment the lattice resolves): with
 * K_{p,i} = prod_d (e_{i,d} - u_d)^{p_d} (lattice units), kappa = K f and
 * kappa_eq,p = rho prod_d m(p_d), m = (1, 0, theta/r^2), the post-collision
 * state solves K f* = kappa - omega_{|p|} (kappa - kappa_eq). */
static int collide_tp_definitional(const orc_lattice *L, const orc_cfg *cfg, const double *f, double *out)
{
    int D = L->D, Q = L->Q;
    double rho, u[3], th;
    node_moments(L, f, &rho, u, &th);
    if (!cfg->thermal) th = cfg->theta0;
    double ul[3] = {u[0] / L->r, u[1] / L->r, u[2] / L->r};
    double K[27 * 27], ks[27];
    for (int p = 0; p < Q; ++p) {
        int pd[3];
        tp_index(D, p, pd);
        double kap = 0.0, keq = rho;
        for (int i = 0; i < Q; ++i) {
            double m = 1.0;
            for (int d = 0; d < D; ++d) m *= pow(L->e[i][d] - ul[d], pd[d]);
            K[p * Q + i] = m;
            kap += m * f[i];
        }
        for (int d = 0; d < D; ++d) keq *= (pd[d] == 0) ? 1.0 : (pd[d] == 1 ? 0.0 : th / (L->r * L->r));
        int ord = pd[0] + pd[1] + pd[2];
        double om = (ord < 2) ? 0.0 : ((cfg->model == ORC_REG_BGK) ? cfg->omega[2] : cfg->omega[ord]);
        ks[p] = kap - om * (kap - keq);
    }
    if (solve_dense(Q, K, ks)) return -1;
    for (int i = 0; i < Q; ++i) out[i] = ks[i];
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Collision, D2Q37 (N = M = 4, Sec. II.C)                                   */
/* ------------------------------------------------------------------------- */

/* Hermite tensors H^(0..4) of the abscissas of a 2D rule. */
static void hermite_init(orc_lattice *L)
{
    for (int i = 0; i < L->Q; ++i) {
        double xi[2] = {L->r * L->e[i][0], L->r * L->e[i][1]};
        hermite_tensors(2, 4, xi, L->H[i]);
    }
}

/* The paper's procedure for the truncated basis (N = M = L->N):
 *  1. rho, u, theta (theta frozen at theta0 when isothermal);
 *  2. f0 = the order-N Hermite equilibrium;
 *  3. a1^(n) = sum_i (f_i - f0_i) H^(n)(xi_i), n = 2 .. N (eq:an);
 *  4. a_Omega^(n) from eq:mrt (its terms up to order N), with the delta
 *     term of the fourth order carrying cfg->delta_coef (6 satisfies
 *     eq:omega; the paper prints 72); raw MRT uses -omega_n a1^(n),
 *     regularised BGK -omega a1^(n) (eq:regnmrt);
 *  5. f*_i = f^_i + Omega_i, where f^ is the order-N projection of eq:reg and
 *     Omega_i = w_i sum_n a_Omega^(n):H^(n)(xi_i)/n! (eq:fi). */
static void collide_hermite(const orc_lattice *L, const orc_cfg *cfg, const double *f, double *out)
{
    const int D = 2, N = L->N;
    double rho, u[3], th;
    node_moments(L, f, &rho, u, &th);
    if (!cfg->thermal) th = cfg->theta0;
    double f0[ORC_MAXQ], af[31], a1[31], aO[31];
    equilibrium(L, cfg->lattice, rho, u, th, f0);
    memset(af, 0, sizeof(af));
    memset(a1, 0, sizeof(a1));
    const int nk = t_offset(D, N + 1);
    for (int i = 0; i < L->Q; ++i)
        for (int k = 0; k < nk; ++k) {
            af[k] += f[i] * L->H[i][k];
            a1[k] += (f[i] - f0[i]) * L->H[i][k];
        }
    memset(aO, 0, sizeof(aO));
    const double *A2 = a1 + t_offset(D, 2), *A3 = a1 + t_offset(D, 3), *A4 = a1 + t_offset(D, 4);
    double *O2 = aO + t_offset(D, 2), *O3 = aO + t_offset(D, 3), *O4 = aO + t_offset(D, 4);
    if (cfg->model == ORC_CM) {
        double w2 = cfg->omega[2], w3 = cfg->omega[3], w4 = cfg->omega[4];
        double delta[4], uu[4], ua2[8], ua3[16], uua2[16], da2[16];
        t_delta(D, delta);
        t_symprod(D, 1, u, 1, u, uu);
        t_symprod(D, 1, u, 2, A2, ua2);
        t_symprod(D, 1, u, 3, A3, ua3);
        t_symprod(D, 2, uu, 2, A2, uua2);
        t_symprod(D, 2, delta, 2, A2, da2);
        for (int k = 0; k < 4; ++k) O2[k] = -w2 * A2[k];                                   /* eq:mrt-a */
        for (int k = 0; k < 8; ++k) O3[k] = -w3 * A3[k] + 3.0 * (w3 - w2) * ua2[k];         /* eq:mrt-b */
        if (N >= 4)
            for (int k = 0; k < 16; ++k)
                O4[k] = -w4 * A4[k] + 4.0 * (w4 - w3) * ua3[k]
                      - 6.0 * (w4 + w2 - 2.0 * w3) * uua2[k] - cfg->delta_coef * (w4 - w2) * da2[k];
    } else {
        for (int n = 2; n <= N; ++n) {
            double om = (cfg->model == ORC_REG_BGK) ? cfg->omega[2] : cfg->omega[n];
            for (int k = t_offset(D, n); k < t_offset(D, n + 1); ++k) aO[k] = -om * a1[k];
        }
    }
    for (int i = 0; i < L->Q; ++i) {
        double s = 0.0;
        for (int n = 0; n <= N; ++n) {
            int o = t_offset(D, n);
            s += t_contract(D, n, af + o, L->H[i] + o) / factorial(n);
            s += t_contract(D, n, aO + o, L->H[i] + o) / factorial(n);
        }
        out[i] = L->w[i] * s;
    }
}

/* Definitional form for the 2D rules: f* lies in the span of w_i H_m(xi_i)
 * (the (N+1)(N+2)/2 components of order <= N: 15 for N = 4, 10 for N = 3)
 * and its central monomial moments of order <= N are
 * sum_i f*_i c_i^p = (1 - omega_{|p|}) sum_i f_i c_i^p + omega_{|p|} rho mu_px mu_py,
 * with mu the Gaussian central moments (1, 0, theta, 0, 3 theta^2) (eq:omega
 * for every resolved order).  Solved as a square system. */
static int collide_hermite_definitional(const orc_lattice *L, const orc_cfg *cfg, const double *f, double *out)
{
    double rho, u[3], th;
    node_moments(L, f, &rho, u, &th);
    if (!cfg->thermal) th = cfg->theta0;
    int basis[15][2], nb = 0;
    for (int n = 0; n <= L->N; ++n)
        for (int k = 0; k <= n; ++k) { basis[nb][0] = k; basis[nb][1] = n - k; ++nb; }
    double mu[5] = {1.0, 0.0, th, 0.0, 3.0 * th * th};
    double A[225], rhs[15];
    for (int row = 0; row < nb; ++row) {
        int px = basis[row][0], py = basis[row][1], ord = px + py;
        double kap = 0.0;
        for (int i = 0; i < L->Q; ++i) {
            double cx = L->r * L->e[i][0] - u[0], cy = L->r * L->e[i][1] - u[1];
            kap += f[i] * pow(cx, px) * pow(cy, py);
        }
        double om = (ord < 2) ? 0.0 : ((cfg->model == ORC_REG_BGK) ? cfg->omega[2] : cfg->omega[ord]);
        rhs[row] = (1.0 - om) * kap + om * rho * mu[px] * mu[py];
        for (int col = 0; col < nb; ++col) {
            double s = 0.0;
            for (int i = 0; i < L->Q; ++i) {
                double xx = L->r * L->e[i][0], yy = L->r * L->e[i][1];
                double phi = L->w[i] * he1d(basis[col][0], xx) * he1d(basis[col][1], yy);
                s += phi * pow(xx - u[0], px) * pow(yy - u[1], py);
            }
            A[row * nb + col] = s;
        }
    }
    if (solve_dense(nb, A, rhs)) return -1;
    for (int i = 0; i < L->Q; ++i) {
        double xx = L->r * L->e[i][0], yy = L->r * L->e[i][1], s = 0.0;
        for (int col = 0; col < nb; ++col) s += rhs[col] * L->w[i] * he1d(basis[col][0], xx) * he1d(basis[col][1], yy);
        out[i] = s;
    }
    return 0;
}

static void build_tables(orc_lattice *L, int kind)
{
    if (L->N > 0) hermite_init(L);
    else (void)tp_table(L);
    (void)kind;
}

static int collide_node(const orc_lattice *L, const orc_cfg *cfg, const double *f, double *out)
{
    if (L->N > 0) collide_hermite(L, cfg, f, out);
    else collide_tp(L, cfg, f, out);
    return 0;
}

int orc_collide(const orc_cfg *cfg, int n_nodes, const double *f, double *out)
{
    const orc_lattice *L = lattice(cfg->lattice);
    if (!L) return -1;
    for (int k = 0; k < n_nodes; ++k) collide_node(L, cfg, f + (size_t)k * L->Q, out + (size_t)k * L->Q);
    return 0;
}

int orc_collide_definitional(const orc_cfg *cfg, int n_nodes, const double *f, double *out)
{
    const orc_lattice *L = lattice(cfg->lattice);
    if (!L) return -1;
    for (int k = 0; k < n_nodes; ++k) {
        int rc = (L->N > 0)
            ? collide_hermite_definitional(L, cfg, f + (size_t)k * L->Q, out + (size_t)k * L->Q)
            : collide_tp_definitional(L, cfg, f + (size_t)k * L->Q, out + (size_t)k * L->Q);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Periodic grid: state, streaming, steps (eq:lbgk update form)              */
/* ------------------------------------------------------------------------- */
/* State S_t: post-collision populations, layout S[i][z][y][x] (x fastest).
 * One step: S_{t+1}(x)_i = C[ S_t(x - e_i)_i ]  (pull, then collide), which is
 * the update f_i(x + xi_i, t + 1) = f*_i(x, t) re-indexed. */

static inline size_t wrap(long v, long n) { v %= n; if (v < 0) v += n; return (size_t)v; }

static void gather(const orc_lattice *L, long nx, long ny, long nz, const double *S, long x, long y, long z, double *f)
{
    size_t plane = (size_t)nx * ny * nz;
    for (int i = 0; i < L->Q; ++i) {
        size_t xs = wrap(x - L->e[i][0], nx), ys = wrap(y - L->e[i][1], ny), zs = wrap(z - L->e[i][2], nz);
        f[i] = S[i * plane + (zs * ny + ys) * nx + xs];
    }
}

int orc_run(const orc_cfg *cfg, long nx, long ny, long nz, double *S, long nsteps, int nthreads)
{
    const orc_lattice *L = lattice(cfg->lattice);
    if (!L || nx < 1 || ny < 1 || nz < 1) return -1;
    if (L->D == 2 && nz != 1) return -1;
    size_t plane = (size_t)nx * ny * nz;
    double *T = (double *)malloc(sizeof(double) * plane * L->Q);
    if (!T) return -2;
    for (long s = 0; s < nsteps; ++s) {
        #pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads)
        for (long z = 0; z < nz; ++z)
            for (long y = 0; y < ny; ++y)
                for (long x = 0; x < nx; ++x) {
                    double f[ORC_MAXQ], o[ORC_MAXQ];
                    gather(L, nx, ny, nz, S, x, y, z, f);
                    collide_node(L, cfg, f, o);
                    size_t node = ((size_t)z * ny + y) * nx + x;
                    for (int i = 0; i < L->Q; ++i) T[i * plane + node] = o[i];
                }
        memcpy(S, T, sizeof(double) * plane * L->Q);
    }
    free(T);
    return 0;
}

/* One step evaluated only at the listed nodes (flat index (z*ny+y)*nx+x);
 * out[k*Q + i] receives population i of node k. */
int orc_step_nodes(const orc_cfg *cfg, long nx, long ny, long nz, const double *S,
                   long n_nodes, const int64_t *nodes, double *out, int nthreads)
{
    const orc_lattice *L = lattice(cfg->lattice);
    if (!L) return -1;
    #pragma omp parallel for schedule(static) num_threads(nthreads)
    for (long k = 0; k < n_nodes; ++k) {
        long idx = (long)nodes[k];
        long x = idx % nx, y = (idx / nx) % ny, z = idx / (nx * ny);
        double f[ORC_MAXQ];
        gather(L, nx, ny, nz, S, x, y, z, f);
        collide_node(L, cfg, f, out + (size_t)k * L->Q);
    }
    return 0;
}

/* Equilibrium initial state S_0 = f0(rho, u, theta); u in lattice units,
 * fields laid out [comp][z][y][x]; theta may be NULL (then cfg->theta0). */
int orc_init_equilibrium(const orc_cfg *cfg, long nx, long ny, long nz,
                         const double *rho, const double *u, const double *theta, double *S, int nthreads)
{
    const orc_lattice *L = lattice(cfg->lattice);
    if (!L) return -1;
    size_t plane = (size_t)nx * ny * nz;
    #pragma omp parallel for schedule(static) num_threads(nthreads)
    for (long n = 0; n < (long)plane; ++n) {
        double ux[3] = {0, 0, 0}, f0[ORC_MAXQ];
        for (int d = 0; d < L->D; ++d) ux[d] = L->r * u[d * plane + n];
        equilibrium(L, cfg->lattice, rho[n], ux, theta ? theta[n] : cfg->theta0, f0);
        for (int i = 0; i < L->Q; ++i) S[i * plane + n] = f0[i];
    }
    return 0;
}

/* Macroscopic fields of a state: rho, u (lattice units, [d][node]) and theta. */
int orc_moments(int kind, long n_nodes, const double *S, double *rho, double *u, double *theta)
{
    const orc_lattice *L = lattice(kind);
    if (!L) return -1;
    for (long n = 0; n < n_nodes; ++n) {
        double f[ORC_MAXQ], r_, ux[3], th;
        for (int i = 0; i < L->Q; ++i) f[i] = S[i * n_nodes + n];
        node_moments(L, f, &r_, ux, &th);
        rho[n] = r_;
        for (int d = 0; d < L->D; ++d) u[d * n_nodes + n] = ux[d] / L->r;
        if (theta) theta[n] = th;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Learned closure (D3Q27): a per-node MLP sets omega_3..omega_6             */
/* ------------------------------------------------------------------------- */
/* Not part of the paper; the rates it sets are the paper's omega_n of
 * eq:omega for n >= 3.  Network: x (27) -> GELU(W1 x + b1) (32) ->
 * GELU(W2 h1 + b2) (32) -> z = W3 h2 + b3 (4), omega_{n} = 0.5 + 1.45
 * sigmoid(z_{n-3}).  GELU is the exact erf form.  Parameters are packed as
 * W1[32][27], b1[32], W2[32][32], b2[32], W3[4][32], b3[4] (2084 values,
 * row-major [out][in]).  Inputs are the non-equilibrium central moments
 * x_p = (kappa_p - kappa_eq,p) / (rho sigma_p), p = px + 3 py + 9 pz,
 * kappa_p = sum_i f_i prod_d (e_{i,d} - u_d)^{p_d} (lattice units) and
 * kappa_eq,p = rho prod_d m(p_d), m = (1, 0, 1/3). */

#define MLP_NIN 27
#define MLP_NH 32
#define MLP_NOUT 4
#define MLP_NPARAM (MLP_NH * MLP_NIN + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NOUT * MLP_NH + MLP_NOUT)
#define MLP_NQ (MLP_NIN + 2 * MLP_NH)   /* rounded quantities of one node: x, h1, h2 */

static double gelu(double a) { return 0.5 * a * (1.0 + erf(a / sqrt(2.0))); }
static double gelu_grad(double a)
{
    const double pi = 3.14159265358979323846;
    return 0.5 * (1.0 + erf(a / sqrt(2.0))) + a * exp(-0.5 * a * a) / sqrt(2.0 * pi);
}
static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Optional rounding of the network's operands.  The library evaluates the
 * network with BF16 weights, inputs and hidden activations (8 significant
 * bits, round to nearest with ties to even).  With bits = 8 the oracle
 * rounds the same quantities: the weights W1, W2, W3, the inputs x and the
 * activations h1 = GELU(a1), h2 = GELU(a2); biases, pre-activations and
 * everything downstream of z stay exact.  The derivative of the objective
 * passes through a rounding unchanged (the rounding error is a constant of
 * the evaluation), so the backward pass uses the rounded weights and the
 * rounded activations.
 *   offset: per rounded quantity, add this constant instead of rounding, with
 *           the weights as given (the network whose exact gradient the
 *           rounded network's gradient is);
 *   xset:   the rounded inputs take these values (one of the roundings that
 *           another evaluation may arrive at). */
typedef struct {
    int bits;
    const double *offset;
    const double *xset;
} mlp_round;

/* Nearest value with `bits` significant bits, ties to even; *lo and *hi
 * receive the two such values bracketing v (equal if v is one). */
static double round_sig(double v, int bits, double *lo, double *hi)
{
    if (v == 0.0 || !isfinite(v)) {
        if (lo) *lo = v;
        if (hi) *hi = v;
        return v;
    }
    int e;
    const double m = frexp(fabs(v), &e);      /* |v| = m 2^e, 0.5 <= m < 1 */
    const double sc = ldexp(m, bits);         /* in [2^(bits-1), 2^bits) */
    const double fl = floor(sc), sign = v < 0 ? -1.0 : 1.0;
    const double a = sign * ldexp(fl, e - bits), b = sign * ldexp(fl == sc ? fl : fl + 1.0, e - bits);
    if (lo) *lo = a;
    if (hi) *hi = b;
    const double frac = sc - fl;
    if (frac < 0.5) return a;
    if (frac > 0.5) return b;
    return fmod(fl, 2.0) == 0.0 ? a : b;
}

static double mlp_weight(const mlp_round *q, double w)
{
    return (q && !q->offset && q->bits > 0) ? round_sig(w, q->bits, NULL, NULL) : w;
}

static double mlp_q(const mlp_round *q, int k, double v)
{
    if (!q) return v;
    if (q->offset) return v + q->offset[k];
    if (q->bits <= 0) return v;
    return round_sig(v, q->bits, NULL, NULL);
}

/* pre-rounding values (x, h1, h2), the values used (xr, h1r, h2r), the
 * pre-activations and the logits of one node */
typedef struct {
    double x[MLP_NIN], xr[MLP_NIN];
    double a1[MLP_NH], h1[MLP_NH], h1r[MLP_NH], s1[MLP_NH];
    double a2[MLP_NH], h2[MLP_NH], h2r[MLP_NH], s2[MLP_NH];
    double z[MLP_NOUT], s3[MLP_NOUT];
} mlp_trace;

/* s1, s2: |b| + sum |W in| of each pre-activation (the scale of its sum) */
static void mlp_forward(const double *P, const double *x, const mlp_round *q, mlp_trace *t)
{
    const double *W1 = P, *b1 = W1 + MLP_NH * MLP_NIN, *W2 = b1 + MLP_NH, *b2 = W2 + MLP_NH * MLP_NH;
    const double *W3 = b2 + MLP_NH, *b3 = W3 + MLP_NOUT * MLP_NH;
    for (int k = 0; k < MLP_NIN; ++k) {
        t->x[k] = x[k];
        t->xr[k] = (q && q->xset) ? q->xset[k] : mlp_q(q, k, x[k]);
    }
    for (int j = 0; j < MLP_NH; ++j) {
        double s = b1[j], m = fabs(b1[j]);
        for (int k = 0; k < MLP_NIN; ++k) {
            const double term = mlp_weight(q, W1[j * MLP_NIN + k]) * t->xr[k];
            s += term;
            m += fabs(term);
        }
        t->a1[j] = s;
        t->s1[j] = m;
        t->h1[j] = gelu(s);
        t->h1r[j] = mlp_q(q, MLP_NIN + j, t->h1[j]);
    }
    for (int j = 0; j < MLP_NH; ++j) {
        double s = b2[j], m = fabs(b2[j]);
        for (int k = 0; k < MLP_NH; ++k) {
            const double term = mlp_weight(q, W2[j * MLP_NH + k]) * t->h1r[k];
            s += term;
            m += fabs(term);
        }
        t->a2[j] = s;
        t->s2[j] = m;
        t->h2[j] = gelu(s);
        t->h2r[j] = mlp_q(q, MLP_NIN + MLP_NH + j, t->h2[j]);
    }
    for (int j = 0; j < MLP_NOUT; ++j) {
        double s = b3[j], m = fabs(b3[j]);
        for (int k = 0; k < MLP_NH; ++k) {
            const double term = mlp_weight(q, W3[j * MLP_NH + k]) * t->h2r[k];
            s += term;
            m += fabs(term);
        }
        t->z[j] = s;
        t->s3[j] = m;
    }
}

static double rate_from_logit(double z) { return 0.5 + 1.45 * sigmoid(z); }

int orc_mlp_nparam(void) { return MLP_NPARAM; }

int orc_mlp_forward(const double *params, int n, const double *x, double *omega)
{
    for (int k = 0; k < n; ++k) {
        mlp_trace t;
        mlp_forward(params, x + (size_t)k * MLP_NIN, NULL, &t);
        for (int j = 0; j < MLP_NOUT; ++j) omega[(size_t)k * MLP_NOUT + j] = rate_from_logit(t.z[j]);
    }
    return 0;
}

int orc_round_sig(int n, const double *in, int bits, double *out)
{
    for (int k = 0; k < n; ++k) out[k] = round_sig(in[k], bits, NULL, NULL);
    return 0;
}

/* Network inputs of one D3Q27 node (central moments by their definition). */
static void closure_inputs(const orc_lattice *L, const double *f, const double *norm, double *x)
{
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < 27; ++i) {
        rho += f[i];
        for (int d = 0; d < 3; ++d) j[d] += f[i] * L->e[i][d];
    }
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    for (int p = 0; p < 27; ++p) {
        int pd[3];
        tp_index(3, p, pd);
        double kap = 0.0, keq = rho;
        for (int i = 0; i < 27; ++i) {
            double m = 1.0;
            for (int d = 0; d < 3; ++d) m *= pow(L->e[i][d] - u[d], pd[d]);
            kap += m * f[i];
        }
        for (int d = 0; d < 3; ++d) keq *= (pd[d] == 0) ? 1.0 : (pd[d] == 1 ? 0.0 : 1.0 / 3.0);
        x[p] = (kap - keq) / (rho * norm[p]);
    }
}

int orc_closure_inputs(int n, const double *f, const double *norm, double *x)
{
    const orc_lattice *L = lattice(ORC_D3Q27);
    for (int k = 0; k < n; ++k) closure_inputs(L, f + (size_t)k * 27, norm, x + (size_t)k * 27);
    return 0;
}

/* One node of the closure collision.  f: pulled populations; fbar: target
 * (NULL for the collision alone); inv_n: weight of the node in the mean.
 * Outputs f* (fs), the rates omega_3..6 (om), the node's share of the
 * objective (*loss) and of its gradient (grad, accumulated; NULL to skip).
 *
 * Objective: L = (1/n) sum_nodes sum_i (f*_i - fbar_i)^2 / w_i.  f* is
 * affine in each omega_m (kappa* = kappa + omega_{|p|} (kappa_eq - kappa)),
 * so the derivative of f* with respect to omega_m is the difference of two
 * collisions with omega_m = 1 and omega_m = 0; the rest is the chain rule
 * through the sigmoid map and the two GELU layers. */
static void closure_node(const orc_lattice *L, const orc_cfg *cfg, const double *f, const double *fbar,
                         const double *P, const double *norm, int tie_even, double inv_n, const mlp_round *q,
                         mlp_trace *t, double *fs, double *om, double *loss, double *grad)
{
    double x[27];
    closure_inputs(L, f, norm, x);
    mlp_forward(P, x, q, t);
    orc_cfg c = *cfg;
    for (int j = 0; j < MLP_NOUT; ++j) c.omega[3 + j] = rate_from_logit(t->z[j]);
    if (tie_even) c.omega[4] = c.omega[6] = cfg->omega[2];
    if (om)
        for (int j = 0; j < MLP_NOUT; ++j) om[j] = c.omega[3 + j];
    collide_tp(L, &c, f, fs);
    if (!fbar) return;
    double r[27], l = 0.0;
    for (int i = 0; i < 27; ++i) {
        const double e = fs[i] - fbar[i];
        l += e * e / L->w[i] * inv_n;
        r[i] = 2.0 * e / L->w[i] * inv_n;
    }
    *loss = l;
    if (!grad) return;
    const double *W2 = P + MLP_NH * MLP_NIN + MLP_NH;
    const double *W3 = W2 + MLP_NH * MLP_NH + MLP_NH;
    double dz[MLP_NOUT];
    for (int j = 0; j < MLP_NOUT; ++j) {
        if (tie_even && (j == 1 || j == 3)) { dz[j] = 0.0; continue; }
        orc_cfg c1 = c, c0 = c;
        c1.omega[3 + j] = 1.0;
        c0.omega[3 + j] = 0.0;
        double g1[27], g0[27], dw = 0.0;
        collide_tp(L, &c1, f, g1);
        collide_tp(L, &c0, f, g0);
        for (int i = 0; i < 27; ++i) dw += r[i] * (g1[i] - g0[i]);
        const double s = sigmoid(t->z[j]);
        dz[j] = dw * 1.45 * s * (1.0 - s);
    }
    double *gW1 = grad, *gb1 = gW1 + MLP_NH * MLP_NIN, *gW2 = gb1 + MLP_NH, *gb2 = gW2 + MLP_NH * MLP_NH;
    double *gW3 = gb2 + MLP_NH, *gb3 = gW3 + MLP_NOUT * MLP_NH;
    double da2[MLP_NH], da1[MLP_NH];
    for (int j = 0; j < MLP_NOUT; ++j) {
        gb3[j] += dz[j];
        for (int m = 0; m < MLP_NH; ++m) gW3[j * MLP_NH + m] += dz[j] * t->h2r[m];
    }
    for (int m = 0; m < MLP_NH; ++m) {
        double dh = 0.0;
        for (int j = 0; j < MLP_NOUT; ++j) dh += mlp_weight(q, W3[j * MLP_NH + m]) * dz[j];
        da2[m] = dh * gelu_grad(t->a2[m]);
    }
    for (int j = 0; j < MLP_NH; ++j) {
        gb2[j] += da2[j];
        for (int m = 0; m < MLP_NH; ++m) gW2[j * MLP_NH + m] += da2[j] * t->h1r[m];
    }
    for (int m = 0; m < MLP_NH; ++m) {
        double dh = 0.0;
        for (int j = 0; j < MLP_NH; ++j) dh += mlp_weight(q, W2[j * MLP_NH + m]) * da2[j];
        da1[m] = dh * gelu_grad(t->a1[m]);
    }
    for (int j = 0; j < MLP_NH; ++j) {
        gb1[j] += da1[j];
        for (int m = 0; m < MLP_NIN; ++m) gW1[j * MLP_NIN + m] += da1[j] * t->xr[m];
    }
}

/* Collision with the network's rates for orders 3..6 (omega_2 from cfg).
 * With tie_even, orders 4 and 6 relax at omega_2 instead (the network's
 * outputs for them are unused). */
int orc_collide_closure(const orc_cfg *cfg, int n, const double *f, const double *params, const double *norm,
                        int tie_even, double *out, double *omega_out)
{
    const orc_lattice *L = lattice(ORC_D3Q27);
    if (cfg->lattice != ORC_D3Q27 || cfg->model != ORC_CM) return -1;
    for (int k = 0; k < n; ++k) {
        mlp_trace t;
        closure_node(L, cfg, f + (size_t)k * 27, NULL, params, norm, tie_even, 0.0, NULL, &t,
                     out + (size_t)k * 27, omega_out ? omega_out + (size_t)k * MLP_NOUT : NULL, NULL, NULL);
    }
    return 0;
}

/* Training objective and its gradient for pulled pre-collision states f and
 * targets fbar (n nodes each, [node][i]), the network in FP64. */
int orc_closure_loss_grad(const orc_cfg *cfg, int n, const double *f, const double *fbar, const double *params,
                          const double *norm, int tie_even, double *loss_out, double *grad)
{
    const orc_lattice *L = lattice(ORC_D3Q27);
    if (cfg->lattice != ORC_D3Q27 || cfg->model != ORC_CM || n < 1) return -1;
    memset(grad, 0, sizeof(double) * MLP_NPARAM);
    double loss = 0.0;
    for (int k = 0; k < n; ++k) {
        mlp_trace t;
        double fs[27], l;
        closure_node(L, cfg, f + (size_t)k * 27, fbar + (size_t)k * 27, params, norm, tie_even, 1.0 / n, NULL,
                     &t, fs, NULL, &l, grad);
        loss += l;
    }
    *loss_out = loss;
    return 0;
}

/* The objective of the network whose operands are shifted by constant
 * offsets instead of rounded (offsets[k * MLP_NQ + q] for node k: x, h1, h2),
 * with the weights as given.  At offsets equal to the rounding errors of a
 * rounded evaluation it takes the same value, and its exact gradient is the
 * gradient the rounded evaluation reports. */
int orc_closure_loss_offsets(const orc_cfg *cfg, int n, const double *f, const double *fbar, const double *params,
                             const double *norm, int tie_even, const double *offsets, double *loss_out)
{
    const orc_lattice *L = lattice(ORC_D3Q27);
    if (cfg->lattice != ORC_D3Q27 || cfg->model != ORC_CM || n < 1) return -1;
    double loss = 0.0;
    for (int k = 0; k < n; ++k) {
        mlp_round q = {0, offsets + (size_t)k * MLP_NQ, NULL};
        mlp_trace t;
        double fs[27], l;
        closure_node(L, cfg, f + (size_t)k * 27, fbar + (size_t)k * 27, params, norm, tie_even, 1.0 / n, &q, &t,
                     fs, NULL, &l, NULL);
        loss += l;
    }
    *loss_out = loss;
    return 0;
}

/* Deviation of a rounded quantity: the other evaluation computes v with an
 * error of at most d, so its rounded value lies between the roundings of
 * v - d and v + d; returns the largest distance of those from `used` (0 if
 * both equal it). */
static double rounding_spread(double v, double d, double used, int bits)
{
    const double lo = round_sig(v - d, bits, NULL, NULL), hi = round_sig(v + d, bits, NULL, NULL);
    return fmax(fabs(lo - used), fabs(hi - used));
}

/* Bounds of one node's outputs when its rounded inputs may deviate by dx
 * and the later operands follow the error model (see
 * orc_closure_eval_rounded), by propagating deviation bounds through the
 * rounded network and its backward pass: each product |a b| deviates by at
 * most |da| |b| + |a| |db| + |da| |db|, each sum by the sum of |coefficient|
 * times the deviations, a smooth map by its derivative times the deviation
 * plus half its largest second derivative times the deviation squared
 * (|GELU''| <= 0.8, |sigmoid''| <= 0.1).  f* is affine in each omega_j with
 * slopes D_ij that do not depend on the rates, so its deviation is exactly
 * sum_j |D_ij| |d omega_j|. */
static void interval_bounds(const orc_lattice *L, const orc_cfg *cfg, const double *f, const double *fbar,
                            const double *P, int tie_even, double inv_n, int bits, const double *err,
                            const mlp_trace *t, const double *fs, const double *dx, double *bfs, double *bgrad)
{
    const double *W1 = P, *W2 = W1 + MLP_NH * MLP_NIN + MLP_NH, *W3 = W2 + MLP_NH * MLP_NH + MLP_NH;
    const mlp_round q = {bits, NULL, NULL};
    const double G2 = 0.8, S2 = 0.1;
    /* layer 1 */
    double da1[MLP_NH], dh1[MLP_NH];
    for (int j = 0; j < MLP_NH; ++j) {
        double s = 0.0;
        for (int m = 0; m < MLP_NIN; ++m) s += fabs(mlp_weight(&q, W1[j * MLP_NIN + m])) * dx[m];
        da1[j] = s;
        const double d = fabs(gelu_grad(t->a1[j])) * s + 0.5 * G2 * s * s + err[1] * fabs(t->a1[j]) + err[2] * t->s1[j];
        dh1[j] = rounding_spread(t->h1[j], d, t->h1r[j], bits);
    }
    /* layer 2 */
    double da2[MLP_NH], dh2[MLP_NH];
    for (int j = 0; j < MLP_NH; ++j) {
        double s = 0.0;
        for (int m = 0; m < MLP_NH; ++m) s += fabs(mlp_weight(&q, W2[j * MLP_NH + m])) * dh1[m];
        da2[j] = s;
        const double d = fabs(gelu_grad(t->a2[j])) * s + 0.5 * G2 * s * s + err[1] * fabs(t->a2[j]) + err[2] * t->s2[j];
        dh2[j] = rounding_spread(t->h2[j], d, t->h2r[j], bits);
    }
    /* logits and rates */
    double dz[MLP_NOUT], dom[MLP_NOUT], sg[MLP_NOUT];
    for (int j = 0; j < MLP_NOUT; ++j) {
        double s = err[2] * t->s3[j];
        for (int m = 0; m < MLP_NH; ++m) s += fabs(mlp_weight(&q, W3[j * MLP_NH + m])) * dh2[m];
        dz[j] = s;
        const double sj = sigmoid(t->z[j]);
        sg[j] = sj * (1.0 - sj);
        dom[j] = 1.45 * (sg[j] * s + 0.5 * S2 * s * s);
        if (tie_even && (j == 1 || j == 3)) dom[j] = 0.0;
    }
    /* slopes of f* in each rate, and the deviation of f* */
    orc_cfg c = *cfg;
    for (int j = 0; j < MLP_NOUT; ++j) c.omega[3 + j] = rate_from_logit(t->z[j]);
    if (tie_even) c.omega[4] = c.omega[6] = cfg->omega[2];
    double D[MLP_NOUT][27], dfs[27];
    for (int j = 0; j < MLP_NOUT; ++j) {
        orc_cfg c1 = c, c0 = c;
        c1.omega[3 + j] = 1.0;
        c0.omega[3 + j] = 0.0;
        double g1[27], g0[27];
        collide_tp(L, &c1, f, g1);
        collide_tp(L, &c0, f, g0);
        for (int i = 0; i < 27; ++i) D[j][i] = g1[i] - g0[i];
    }
    for (int i = 0; i < 27; ++i) {
        double s = 0.0;
        for (int j = 0; j < MLP_NOUT; ++j) s += fabs(D[j][i]) * dom[j];
        dfs[i] = s;
        if (bfs) bfs[i] += s;
    }
    if (!fbar || !bgrad) return;
    /* objective and residuals */
    double r[27], dr[27], dl = 0.0;
    for (int i = 0; i < 27; ++i) {
        const double e = fs[i] - fbar[i];
        r[i] = 2.0 * e / L->w[i] * inv_n;
        dr[i] = 2.0 * dfs[i] / L->w[i] * inv_n;
        dl += (2.0 * fabs(e) * dfs[i] + dfs[i] * dfs[i]) / L->w[i] * inv_n;
    }
    bgrad[MLP_NPARAM] += dl;
    /* backward: d objective / d z and its deviation */
    double gz[MLP_NOUT], dgz[MLP_NOUT];
    for (int j = 0; j < MLP_NOUT; ++j) {
        double G = 0.0, dG = 0.0;
        for (int i = 0; i < 27; ++i) {
            G += r[i] * D[j][i];
            dG += dr[i] * fabs(D[j][i]);
        }
        const double s = 1.45 * sg[j], ds = 1.45 * S2 * dz[j];
        gz[j] = G * s;
        dgz[j] = dG * fabs(s) + fabs(G) * ds + dG * ds;
        if (tie_even && (j == 1 || j == 3)) gz[j] = dgz[j] = 0.0;
    }
    double *bW1 = bgrad, *bb1 = bW1 + MLP_NH * MLP_NIN, *bW2 = bb1 + MLP_NH, *bb2 = bW2 + MLP_NH * MLP_NH;
    double *bW3 = bb2 + MLP_NH, *bb3 = bW3 + MLP_NOUT * MLP_NH;
    for (int j = 0; j < MLP_NOUT; ++j) {
        bb3[j] += dgz[j];
        for (int m = 0; m < MLP_NH; ++m)
            bW3[j * MLP_NH + m] += dgz[j] * fabs(t->h2r[m]) + fabs(gz[j]) * dh2[m] + dgz[j] * dh2[m];
    }
    /* layer 2 backward */
    double g2[MLP_NH], dg2[MLP_NH];
    for (int m = 0; m < MLP_NH; ++m) {
        double hsum = 0.0, dhsum = 0.0;
        for (int j = 0; j < MLP_NOUT; ++j) {
            const double w = mlp_weight(&q, W3[j * MLP_NH + m]);
            hsum += w * gz[j];
            dhsum += fabs(w) * dgz[j];
        }
        const double gp = gelu_grad(t->a2[m]), dgp = G2 * da2[m] + err[3];
        g2[m] = hsum * gp;
        dg2[m] = dhsum * fabs(gp) + fabs(hsum) * dgp + dhsum * dgp;
    }
    for (int j = 0; j < MLP_NH; ++j) {
        bb2[j] += dg2[j];
        for (int m = 0; m < MLP_NH; ++m)
            bW2[j * MLP_NH + m] += dg2[j] * fabs(t->h1r[m]) + fabs(g2[j]) * dh1[m] + dg2[j] * dh1[m];
    }
    /* layer 1 backward */
    double g1v[MLP_NH], dg1[MLP_NH];
    for (int m = 0; m < MLP_NH; ++m) {
        double hsum = 0.0, dhsum = 0.0;
        for (int j = 0; j < MLP_NH; ++j) {
            const double w = mlp_weight(&q, W2[j * MLP_NH + m]);
            hsum += w * g2[j];
            dhsum += fabs(w) * dg2[j];
        }
        const double gp = gelu_grad(t->a1[m]), dgp = G2 * da1[m] + err[3];
        g1v[m] = hsum * gp;
        dg1[m] = dhsum * fabs(gp) + fabs(hsum) * dgp + dhsum * dgp;
    }
    for (int j = 0; j < MLP_NH; ++j) {
        bb1[j] += dg1[j];
        for (int m = 0; m < MLP_NIN; ++m)
            bW1[j * MLP_NIN + m] += dg1[j] * fabs(t->xr[m]) + fabs(g1v[j]) * dx[m] + dg1[j] * dx[m];
    }
}

/* Bounds of one node's outputs under the error model.  The inputs x are
 * where a different rounding moves the network most (one step of x moves
 * every pre-activation of layer 1), so their alternatives are enumerated:
 * every input whose error interval rounds to other values than x_r takes
 * each of them in turn (all combinations, at most 3^5), the node is
 * evaluated for each, and its bound is the largest of |change| plus the
 * propagated bound of that evaluation.  With more ambiguous inputs the
 * input deviations are propagated as intervals instead. */
static void closure_node_bounds(const orc_lattice *L, const orc_cfg *cfg, const double *f, const double *fbar,
                                const double *P, const double *norm, int tie_even, double inv_n, int bits,
                                double rho0, const double *err, const mlp_trace *t, const double *fs,
                                const double *g0, double *bfs, double *bgrad)
{
    const int ng = MLP_NPARAM + 1;
    double rho = 0.0, dev = 0.0;
    for (int i = 0; i < 27; ++i) {
        rho += f[i];
        dev += fabs(f[i] - L->w[i] * rho0);
    }
    int amb[MLP_NIN], na = 0;
    double alt[MLP_NIN][3];
    int nalt[MLP_NIN];
    double dx[MLP_NIN];
    for (int m = 0; m < MLP_NIN; ++m) {
        const double d = err[0] * dev / (rho * norm[m]);
        dx[m] = rounding_spread(t->x[m], d, t->xr[m], bits);
        if (dx[m] == 0.0) continue;
        /* the representable values in the interval, the one used first */
        const double lo = round_sig(t->x[m] - d, bits, NULL, NULL), hi = round_sig(t->x[m] + d, bits, NULL, NULL);
        nalt[m] = 0;
        alt[m][nalt[m]++] = t->xr[m];
        if (lo != t->xr[m]) alt[m][nalt[m]++] = lo;
        if (hi != t->xr[m] && hi != lo) alt[m][nalt[m]++] = hi;
        amb[na++] = m;
    }
    double zero[MLP_NIN];
    memset(zero, 0, sizeof zero);
    int combos = 1;
    for (int a = 0; a < na && combos <= 243; ++a) combos *= nalt[amb[a]];
    if (na == 0 || combos > 243) {
        interval_bounds(L, cfg, f, fbar, P, tie_even, inv_n, bits, err, t, fs, na ? dx : zero, bfs, bgrad);
        return;
    }
    double *gc = (double *)calloc((size_t)ng, sizeof(double));
    double *bgc = (double *)calloc((size_t)ng, sizeof(double));
    double *worst = (double *)calloc((size_t)ng, sizeof(double));
    if (!gc || !bgc || !worst) {   /* out of memory: fall back to the interval form */
        free(gc); free(bgc); free(worst);
        interval_bounds(L, cfg, f, fbar, P, tie_even, inv_n, bits, err, t, fs, dx, bfs, bgrad);
        return;
    }
    double wfs[27];
    memset(wfs, 0, sizeof wfs);
    for (int c = 0; c < combos; ++c) {
        double xs[MLP_NIN];
        memcpy(xs, t->xr, sizeof xs);
        for (int a = 0, rem = c; a < na; ++a) {
            const int m = amb[a];
            xs[m] = alt[m][rem % nalt[m]];
            rem /= nalt[m];
        }
        const mlp_round q = {bits, NULL, xs};
        mlp_trace tc;
        double fsc[27], bfc[27], lc = 0.0;
        memset(gc, 0, sizeof(double) * ng);
        memset(bgc, 0, sizeof(double) * ng);
        memset(bfc, 0, sizeof bfc);
        closure_node(L, cfg, f, fbar, P, norm, tie_even, inv_n, &q, &tc, fsc, NULL, &lc, (fbar && bgrad) ? gc : NULL);
        gc[MLP_NPARAM] = lc;
        interval_bounds(L, cfg, f, fbar, P, tie_even, inv_n, bits, err, &tc, fsc, zero, bfc, (fbar && bgrad) ? bgc : NULL);
        for (int i = 0; i < 27; ++i) wfs[i] = fmax(wfs[i], fabs(fsc[i] - fs[i]) + bfc[i]);
        if (fbar && bgrad)
            for (int e = 0; e < ng; ++e) worst[e] = fmax(worst[e], fabs(gc[e] - g0[e]) + bgc[e]);
    }
    if (bfs)
        for (int i = 0; i < 27; ++i) bfs[i] += wfs[i];
    if (fbar && bgrad)
        for (int e = 0; e < ng; ++e) bgrad[e] += worst[e];
    free(gc);
    free(bgc);
    free(worst);
}

/* The closure collision (and, with fbar, the objective and its gradient)
 * with the network's operands rounded to `bits` significant bits, plus
 * per-element bounds on how far an evaluation of the same network may land
 * from these values when it computes what it rounds, and the derivative of
 * GELU, with small errors of its own.  Error model err[4] of that
 * evaluation, before each rounding:
 *   x_p:  err[0] * sum_i |f_i - w_i rho0| / (rho sigma_p)
 *   h:    err[1] * |a| + err[2] * (|b| + sum |W in|)   (a the pre-activation;
 *         the logits z carry err[2] * (|b| + sum |W h|))
 *   GELU'(a): err[3] (absolute).
 * Where the error interval of a quantity rounds to other values than this
 * evaluation's, their distance is carried forward (closure_node_bounds).
 * bound_fs[n][27], bound_grad[MLP_NPARAM] (objective) and bound_grad[0..]
 * receive the propagated bounds; abs_grad accumulates |node share| per
 * entry (the scale of the FP32 rounding of the other evaluation's sums).
 * offsets (optional, [n][MLP_NQ]) receives the rounding errors used. */
int orc_closure_eval_rounded(const orc_cfg *cfg, int n, const double *f, const double *fbar, const double *params,
                             const double *norm, int tie_even, int bits, double rho0, const double *err,
                             double *fs_out, double *omega_out, double *loss_out, double *grad,
                             double *bound_fs, double *bound_grad, double *abs_grad, double *offsets)
{
    const orc_lattice *L = lattice(ORC_D3Q27);
    if (cfg->lattice != ORC_D3Q27 || cfg->model != ORC_CM || n < 1 || bits < 1) return -1;
    const int ng = MLP_NPARAM + 1;
    if (grad) memset(grad, 0, sizeof(double) * MLP_NPARAM);
    if (bound_grad) memset(bound_grad, 0, sizeof(double) * ng);
    if (abs_grad) memset(abs_grad, 0, sizeof(double) * ng);
    if (bound_fs) memset(bound_fs, 0, sizeof(double) * 27 * (size_t)n);
    double *g0 = (double *)malloc(sizeof(double) * ng);
    if (!g0) return -2;
    double loss = 0.0;
    for (int k = 0; k < n; ++k) {
        const double *fk = f + (size_t)k * 27, *tk = fbar ? fbar + (size_t)k * 27 : NULL;
        const mlp_round q = {bits, NULL, NULL};
        mlp_trace t;
        double fs[27], l0 = 0.0;
        memset(g0, 0, sizeof(double) * ng);
        closure_node(L, cfg, fk, tk, params, norm, tie_even, 1.0 / n, &q, &t, fs, omega_out + (size_t)k * MLP_NOUT,
                     &l0, (tk && grad) ? g0 : NULL);
        g0[MLP_NPARAM] = l0;
        memcpy(fs_out + (size_t)k * 27, fs, sizeof fs);
        loss += l0;
        if (tk && grad)
            for (int e = 0; e < MLP_NPARAM; ++e) grad[e] += g0[e];
        if (tk && abs_grad)
            for (int e = 0; e < ng; ++e) abs_grad[e] += fabs(g0[e]);
        if (offsets) {
            double *o = offsets + (size_t)k * MLP_NQ;
            for (int m = 0; m < MLP_NIN; ++m) o[m] = t.xr[m] - t.x[m];
            for (int m = 0; m < MLP_NH; ++m) {
                o[MLP_NIN + m] = t.h1r[m] - t.h1[m];
                o[MLP_NIN + MLP_NH + m] = t.h2r[m] - t.h2[m];
            }
        }
        if (bound_fs || bound_grad)
            closure_node_bounds(L, cfg, fk, tk, params, norm, tie_even, 1.0 / n, bits, rho0, err, &t, fs, g0,
                                bound_fs ? bound_fs + (size_t)k * 27 : NULL, tk ? bound_grad : NULL);
    }
    if (loss_out) *loss_out = loss;
    free(g0);
    return 0;
}

/* Pulled (pre-collision) populations of the listed nodes: out[k*Q + i] =
 * S_i(x_k - e_i) on the periodic grid. */
int orc_gather_nodes(int kind, long nx, long ny, long nz, const double *S, long n_nodes, const int64_t *nodes,
                     double *out)
{
    const orc_lattice *L = lattice(kind);
    if (!L) return -1;
    for (long k = 0; k < n_nodes; ++k) {
        long idx = (long)nodes[k];
        long x = idx % nx, y = (idx / nx) % ny, z = idx / (nx * ny);
        gather(L, nx, ny, nz, S, x, y, z, out + (size_t)k * L->Q);
    }
    return 0;
}
