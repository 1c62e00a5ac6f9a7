// Central-moment collision on the 2D Hermite rules: the ninth-degree
// 37-velocity rules with order-4 truncation (N = M = 4, Sec. II.B-C) and the
// seventh-degree 17-velocity rules with N = M = 3, thermal or isothermal.
//
// The paper's update f* = f^ + Omega keeps the Hermite components of order
// <= N (eq:reg) and relaxes them so that eq:omega holds for n <= N.  On these
// rules the raw moments of order <= N of f and of its projection f^ agree
// (the quadrature degree is at least 2N + 1), so the kernel works with
// moments throughout:
//   1. integer lattice moments M_kl = sum_i h_i e_x^k e_y^l (k + l <= N),
//      paired over +-e so even orders use h_i + h_-i and odd ones h_i - h_-i;
//   2. xi-unit raw moments m_kl = r^(k+l) M_kl, then rho, u, theta;
//   3. central moments by a per-axis binomial shift (Appendix A, eq:trans-a);
//   4. relax order n = k + l >= 2 at omega_n towards the Maxwellian central
//      moments rho mu_k mu_l, mu = (1, 0, theta, 0, 3 theta^2);
//   5. shift back, convert raw moments to Hermite coefficients a_kl
//      (He_0..He_4 of Appendix A) and reconstruct with eq:fi,
//      f*_i = w_i sum a_kl He_k(xi_x) He_l(xi_y) / (k! l!), evaluated as a
//      polynomial in the integer velocity components.
// With the coefficient 6 in the delta term of the fourth order (the value
// eq:omega requires) the paper's absolute-frame formula eq:mrt is exactly
// step 4 seen through the binomial transform, so this is the same operator.
// The raw-moment MRT of eq:regnmrt instead relaxes the a_kl themselves.
//
// Everything is carried on deviations h = f - w rho0: their moments are the
// moments of f minus rho0 times the standard-normal moments (exact to the
// rule's degree), and the deviation equilibrium is assembled from small
// differences only.
#pragma once

#include "common.hpp"

namespace cmlb {

// Triangle of multi-indices (k, l), k + l <= N <= 4, stored in a 5x5 array.
template <class R>
struct Tri {
    R v[5][5];
};

// Binomial coefficient table for n <= 4.
__host__ __device__ constexpr int binom4(int n, int k) {
    return (k < 0 || k > n) ? 0 : (n == 0 ? 1 : (k == 0 || k == n) ? 1 : binom4(n - 1, k - 1) + binom4(n - 1, k));
}

// Coefficient of x^a in He_k(x) (probabilists' Hermite polynomials).
__host__ __device__ constexpr int he_coef(int k, int a) {
    constexpr int t[5][5] = {{1, 0, 0, 0, 0}, {0, 1, 0, 0, 0}, {-1, 0, 1, 0, 0},
                             {0, -3, 0, 1, 0}, {3, 0, -6, 0, 1}};
    return t[k][a];
}

__host__ __device__ constexpr int ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }
__host__ __device__ constexpr int fact_c(int n) { return n <= 1 ? 1 : n * fact_c(n - 1); }

// 1. lattice moments of the deviation populations.
template <int LAT, class R>
__device__ __forceinline__ Tri<R> h2_moments(const R (&h)[H2<LAT>::Q]) {
    using L = H2<LAT>;
    Tri<R> M;
    static_for<0, 5>([&](auto K) {
        static_for<0, 5>([&](auto L_) { M.v[decltype(K)::value][decltype(L_)::value] = R(0); });
    });
    M.v[0][0] = h[L::rest];
    static_for<L::rest + 1, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = L::tab.ex[i], ey = L::tab.ey[i];
        const R s = h[i] + h[L::Q - 1 - i];
        const R d = h[i] - h[L::Q - 1 - i];
        static_for<0, 5>([&](auto K) {
            static_for<0, 5>([&](auto L_) {
                constexpr int k = decltype(K)::value, l = decltype(L_)::value;
                if constexpr (k + l <= L::N) {
                    constexpr int c = ipow_c(ex, k) * ipow_c(ey, l);
                    if constexpr (c != 0) {
                        if constexpr ((k + l) % 2 == 0) M.v[k][l] += R(c) * s;
                        else M.v[k][l] += R(c) * d;
                    }
                }
            });
        });
    });
    return M;
}

// Per-axis binomial shift of a triangle: out_kl = sum_a C(k,a) t^(k-a) in_al
// along x (AXIS = 0) or along y (AXIS = 1).  t = -u gives central moments
// from raw ones, t = +u the inverse.
template <int N, int AXIS, class R>
__device__ __forceinline__ Tri<R> h2_shift(const Tri<R>& in, R t) {
    const R tp[5] = {R(1), t, t * t, t * t * t, (t * t) * (t * t)};
    Tri<R> out;
    static_for<0, 5>([&](auto K) {
        static_for<0, 5>([&](auto L) {
            constexpr int k = decltype(K)::value, l = decltype(L)::value;
            if constexpr (k + l <= N) {
                constexpr int n = AXIS == 0 ? k : l;
                R acc = in.v[k][l];
                static_for<0, n>([&](auto A) {
                    constexpr int a = decltype(A)::value;
                    constexpr int c = binom4(n, a);
                    const R src = AXIS == 0 ? in.v[a][l] : in.v[k][a];
                    acc += R(c) * tp[n - a] * src;
                });
                out.v[k][l] = acc;
            }
        });
    });
    return out;
}

template <class R>
struct H2State {
    R drho, rho, ux, uy, dtheta;  // xi-units velocity, theta - 1
};

// 2. macroscopic state from the xi-unit raw moments of the deviations.
template <class R>
__device__ __forceinline__ H2State<R> h2_state(const Tri<R>& m, R rho0, bool thermal, R theta0) {
    H2State<R> st;
    st.drho = m.v[0][0];
    st.rho = rho0 + st.drho;
    const R inv = recip<R>(st.rho);
    st.ux = m.v[1][0] * inv;
    st.uy = m.v[0][1] * inv;
    if (thermal) {
        // rho (|u|^2 + 2 theta) = sum f |xi|^2 = sum h |xi|^2 + 2 rho0
        st.dtheta = R(0.5) * ((m.v[2][0] + m.v[0][2] - R(2) * st.drho) * inv - (st.ux * st.ux + st.uy * st.uy));
    } else {
        st.dtheta = theta0 - R(1);
    }
    return st;
}

// Deviation equilibrium central moments rho mu_k mu_l - rho0 mu'_k mu'_l, with
// mu' the central moments of the standard normal about u, written as
// drho mu_k mu_l + rho0 (Delta_k mu_l + mu'_k Delta_l), Delta = mu - mu'.
template <class R>
__device__ __forceinline__ void h2_eq_factors(R u, R dth, R (&mu)[5], R (&mup)[5], R (&del)[5]) {
    const R th = R(1) + dth, u2 = u * u;
    mu[0] = R(1); mu[1] = R(0); mu[2] = th; mu[3] = R(0); mu[4] = R(3) * th * th;
    mup[0] = R(1); mup[1] = -u; mup[2] = R(1) + u2; mup[3] = -u * (u2 + R(3)); mup[4] = u2 * (u2 + R(6)) + R(3);
    del[0] = R(0); del[1] = u; del[2] = dth - u2; del[3] = u * (u2 + R(3));
    del[4] = R(3) * dth * (R(2) + dth) - u2 * (u2 + R(6));
}

// 5. raw xi-moments of f* - w rho0 -> coefficients C_ab of the polynomial
// sum_ab C_ab e_x^a e_y^b = sum_kl a_kl He_k(r e_x) He_l(r e_y) / (k! l!).
template <int N, class R>
__device__ __forceinline__ Tri<R> h2_poly_from_raw(const Tri<R>& m, R r) {
    // a_kl = sum_ab he(k,a) he(l,b) m_ab
    Tri<R> t, a, c, C;
    static_for<0, 5>([&](auto K) {
        static_for<0, 5>([&](auto L) {
            constexpr int k = decltype(K)::value, l = decltype(L)::value;
            if constexpr (k + l <= N) {
                R acc = R(0);
                static_for<0, k + 1>([&](auto A) {
                    constexpr int aa = decltype(A)::value;
                    constexpr int c = he_coef(k, aa);
                    if constexpr (c != 0) acc += R(c) * m.v[aa][l];
                });
                t.v[k][l] = acc;
            }
        });
    });
    static_for<0, 5>([&](auto K) {
        static_for<0, 5>([&](auto L) {
            constexpr int k = decltype(K)::value, l = decltype(L)::value;
            if constexpr (k + l <= N) {
                R acc = R(0);
                static_for<0, l + 1>([&](auto B) {
                    constexpr int b = decltype(B)::value;
                    constexpr int c = he_coef(l, b);
                    if constexpr (c != 0) acc += R(c) * t.v[k][b];
                });
                constexpr int kl = fact_c(k) * fact_c(l);
                a.v[k][l] = acc * R(1.0 / kl);
            }
        });
    });
    // C_ab = r^(a+b) sum_{k>=a, l>=b} a_kl he(k,a) he(l,b)
    static_for<0, 5>([&](auto A) {
        static_for<0, 5>([&](auto L) {
            constexpr int aa = decltype(A)::value, l = decltype(L)::value;
            if constexpr (aa + l <= N) {
                R acc = R(0);
                static_for<aa, N + 1 - l>([&](auto K) {
                    constexpr int k = decltype(K)::value;
                    constexpr int c = he_coef(k, aa);
                    if constexpr (c != 0) acc += R(c) * a.v[k][l];
                });
                c.v[aa][l] = acc;
            }
        });
    });
    const R rp[5] = {R(1), r, r * r, r * r * r, (r * r) * (r * r)};
    static_for<0, 5>([&](auto A) {
        static_for<0, 5>([&](auto B) {
            constexpr int aa = decltype(A)::value, b = decltype(B)::value;
            if constexpr (aa + b <= N) {
                R acc = R(0);
                static_for<b, N + 1 - aa>([&](auto L) {
                    constexpr int l = decltype(L)::value;
                    constexpr int cc = he_coef(l, b);
                    if constexpr (cc != 0) acc += R(cc) * c.v[aa][l];
                });
                C.v[aa][b] = acc * rp[aa + b];
            }
        });
    });
    return C;
}

// Reconstruct deviation populations from the polynomial coefficients.
template <int LAT, class R>
__device__ __forceinline__ void h2_reconstruct(R (&h)[H2<LAT>::Q], const Tri<R>& C, const R (&wc)[8]) {
    using L = H2<LAT>;
    h[L::rest] = wc[0] * C.v[0][0];
    static_for<L::rest + 1, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = L::tab.ex[i], ey = L::tab.ey[i];
        R ev = R(0), od = R(0);
        static_for<0, 5>([&](auto A) {
            static_for<0, 5>([&](auto B) {
                constexpr int a = decltype(A)::value, b = decltype(B)::value;
                if constexpr (a + b <= L::N) {
                    constexpr int c = ipow_c(ex, a) * ipow_c(ey, b);
                    if constexpr (c != 0) {
                        if constexpr ((a + b) % 2 == 0) ev += R(c) * C.v[a][b];
                        else od += R(c) * C.v[a][b];
                    }
                }
            });
        });
        const R w = wc[L::tab.cls[i]];
        h[i] = w * (ev + od);
        h[L::Q - 1 - i] = w * (ev - od);
    });
}

// Collision of one node from the lattice moments M of its deviation
// populations (step 1 done), writing the post-collision deviations to h.
template <int LAT, int MODEL, class R>
__device__ __forceinline__ void h2_collide_moments(Tri<R> M, R (&h)[H2<LAT>::Q], R rho0, const R* om, R r,
                                                   const R (&wc)[8], bool thermal, R theta0) {
    constexpr int N = H2<LAT>::N;
    static_assert(MODEL == kCM || N == 4, "raw-moment MRT and regularised BGK are built for the order-4 rules");
    const R rp[5] = {R(1), r, r * r, r * r * r, (r * r) * (r * r)};
    static_for<0, 5>([&](auto K) {
        static_for<0, 5>([&](auto L) {
            constexpr int k = decltype(K)::value, l = decltype(L)::value;
            if constexpr (k + l <= N) M.v[k][l] *= rp[k + l];
        });
    });
    const H2State<R> st = h2_state<R>(M, rho0, thermal, theta0);
    Tri<R> mstar;
    if constexpr (MODEL == kRawMRT) {
        // Relax absolute-frame Hermite coefficients a_kl of the raw moments:
        // a_kl = sum he he m; work through central moments of u = 0 is the raw
        // basis, so use the Hermite combination directly on m.
        // equilibrium a'_kl = rho g_k(ux) g_l(uy) - rho0 [k = l = 0],
        // g = E[He_k(X)], X ~ N(u, theta).
        auto gk = [&](R u, R dth, R (&g)[5]) {
            const R u2 = u * u;
            g[0] = R(1); g[1] = u; g[2] = u2 + dth; g[3] = u * (u2 + R(3) * dth);
            g[4] = u2 * (u2 + R(6) * dth) + R(3) * dth * dth;
        };
        R gx[5], gy[5];
        gk(st.ux, st.dtheta, gx);
        gk(st.uy, st.dtheta, gy);
        // Hermite coefficients of the deviations (no 1/k!l! here)
        Tri<R> t, a;
        static_for<0, 5>([&](auto K) {
            static_for<0, 5>([&](auto L) {
                constexpr int k = decltype(K)::value, l = decltype(L)::value;
                if constexpr (k + l <= 4) {
                    R acc = R(0);
                    static_for<0, k + 1>([&](auto A) {
                        constexpr int aa = decltype(A)::value;
                        constexpr int c = he_coef(k, aa);
                        if constexpr (c != 0) acc += R(c) * M.v[aa][l];
                    });
                    t.v[k][l] = acc;
                }
            });
        });
        static_for<0, 5>([&](auto K) {
            static_for<0, 5>([&](auto L) {
                constexpr int k = decltype(K)::value, l = decltype(L)::value;
                if constexpr (k + l <= 4) {
                    R acc = R(0);
                    static_for<0, l + 1>([&](auto B) {
                        constexpr int b = decltype(B)::value;
                        constexpr int c = he_coef(l, b);
                        if constexpr (c != 0) acc += R(c) * t.v[k][b];
                    });
                    a.v[k][l] = acc;
                    if constexpr (k + l >= 2) {
                        const R aeq = st.rho * gx[k] * gy[l];
                        a.v[k][l] += om[k + l] * (aeq - a.v[k][l]);
                    }
                }
            });
        });
        // back to raw moments: m_ab = sum_kl mono(a,k) mono(b,l) a_kl, where
        // x^a = sum_k mono(a,k) He_k(x) (eq:hermite-r)
        constexpr int mono[5][5] = {{1, 0, 0, 0, 0}, {0, 1, 0, 0, 0}, {1, 0, 1, 0, 0},
                                    {0, 3, 0, 1, 0}, {3, 0, 6, 0, 1}};
        Tri<R> t2;
        static_for<0, 5>([&](auto A) {
            static_for<0, 5>([&](auto L) {
                constexpr int aa = decltype(A)::value, l = decltype(L)::value;
                if constexpr (aa + l <= 4) {
                    R acc = R(0);
                    static_for<0, aa + 1>([&](auto K) {
                        constexpr int k = decltype(K)::value;
                        constexpr int c = mono[aa][k];
                        if constexpr (c != 0) acc += R(c) * a.v[k][l];
                    });
                    t2.v[aa][l] = acc;
                }
            });
        });
        static_for<0, 5>([&](auto A) {
            static_for<0, 5>([&](auto B) {
                constexpr int aa = decltype(A)::value, b = decltype(B)::value;
                if constexpr (aa + b <= 4) {
                    R acc = R(0);
                    static_for<0, b + 1>([&](auto L) {
                        constexpr int l = decltype(L)::value;
                        constexpr int c = mono[b][l];
                        if constexpr (c != 0) acc += R(c) * t2.v[aa][l];
                    });
                    mstar.v[aa][b] = acc;
                }
            });
        });
    } else {
        // central moments of the deviations
        Tri<R> kap = h2_shift<N, 1, R>(h2_shift<N, 0, R>(M, -st.ux), -st.uy);
        R mux[5], mupx[5], delx[5], muy[5], mupy[5], dely[5];
        h2_eq_factors<R>(st.ux, st.dtheta, mux, mupx, delx);
        h2_eq_factors<R>(st.uy, st.dtheta, muy, mupy, dely);
        static_for<0, 5>([&](auto K) {
            static_for<0, 5>([&](auto L) {
                constexpr int k = decltype(K)::value, l = decltype(L)::value;
                if constexpr (k + l >= 2 && k + l <= N) {
                    const R keq = st.drho * mux[k] * muy[l] + rho0 * (delx[k] * muy[l] + mupx[k] * dely[l]);
                    kap.v[k][l] += om[k + l] * (keq - kap.v[k][l]);
                }
            });
        });
        mstar = h2_shift<N, 1, R>(h2_shift<N, 0, R>(kap, st.ux), st.uy);
    }
    const Tri<R> C = h2_poly_from_raw<N, R>(mstar, r);
    h2_reconstruct<LAT, R>(h, C, wc);
}

// Full collision of one node (in place on deviation populations).
template <int LAT, int MODEL, class R>
__device__ __forceinline__ void h2_collide(R (&h)[H2<LAT>::Q], R rho0, const R* om, R r, const R (&wc)[8],
                                           bool thermal, R theta0) {
    h2_collide_moments<LAT, MODEL, R>(h2_moments<LAT, R>(h), h, rho0, om, r, wc, thermal, theta0);
}

// Deviation equilibrium populations: the order-N Hermite equilibrium has the
// Maxwellian's central moments up to order N.
template <int LAT, class R>
__device__ __forceinline__ void h2_equilibrium(R (&h)[H2<LAT>::Q], R drho, R rho0, R ux_xi, R uy_xi, R dtheta,
                                               R r, const R (&wc)[8]) {
    constexpr int N = H2<LAT>::N;
    R mux[5], mupx[5], delx[5], muy[5], mupy[5], dely[5];
    h2_eq_factors<R>(ux_xi, dtheta, mux, mupx, delx);
    h2_eq_factors<R>(uy_xi, dtheta, muy, mupy, dely);
    Tri<R> kap;
    static_for<0, 5>([&](auto K) {
        static_for<0, 5>([&](auto L) {
            constexpr int k = decltype(K)::value, l = decltype(L)::value;
            if constexpr (k + l <= N)
                kap.v[k][l] = drho * mux[k] * muy[l] + rho0 * (delx[k] * muy[l] + mupx[k] * dely[l]);
        });
    });
    const Tri<R> m = h2_shift<N, 1, R>(h2_shift<N, 0, R>(kap, ux_xi), uy_xi);
    const Tri<R> C = h2_poly_from_raw<N, R>(m, r);
    h2_reconstruct<LAT, R>(h, C, wc);
}

}  // namespace cmlb
