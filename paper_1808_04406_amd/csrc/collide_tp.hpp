// Central-moment collision on the tensor-product lattices D2Q9 and D3Q27.
//
// The complete basis {0,1,2}^D of per-axis central monomials is resolved
// exactly by the lattices {-1,0,1}^D, so relaxing every central moment
// kappa_p = sum_i f_i prod_d (e_{i,d} - u_d)^{p_d} at the rate of its order
// |p| (eq:omega, required "for all n") and transforming back determines the
// post-collision populations uniquely.  In lattice units the equilibrium
// central moments are rho prod_d m(p_d), m = (1, 0, c_s^2) with
// c_s^2 = theta / r^2 = 1/3 (the complete-basis Maxwellian).
//
// The transform factorises into D sweeps of the 3-point map
// (f_-, f_0, f_+) -> (kappa_0, kappa_1, kappa_2) along each axis, done as raw
// moments first (whose lowest orders are rho and rho u) and then a per-axis
// binomial shift to the central frame; the inverse is analytic.  All arithmetic is on deviations h_i = f_i - w_i rho0: the
// transforms are linear, and the deviation equilibrium
// kappa'_eq = rho prod m - rho0 prod(m + d), d = (0, -u, u^2) (the central
// moments of w about u) is formed by a recursion over the axes that never
// subtracts two O(1) numbers.
#pragma once

#include "common.hpp"

namespace cmlb {

template <int D, class R>
struct TPMacro {
    R drho;  // rho - rho0
    R u[3];  // lattice units
};

// In place: populations (slot digit e+1 along each axis) -> raw moments
// (slot digit = order along each axis), i.e. the sums sum_e e^p f_e.
template <int D, class R>
__device__ __forceinline__ void tp_raw(R (&h)[TP<D>::Q]) {
    static_for<0, D>([&](auto Dd) {
        constexpr int d = decltype(Dd)::value;
        constexpr int s = (d == 0) ? 1 : (d == 1 ? 3 : 9);
        static_for<0, TP<D>::Q>([&](auto B) {
            constexpr int base = decltype(B)::value;
            if constexpr ((base / s) % 3 == 0) {
                const R hm = h[base], h0 = h[base + s], hp = h[base + 2 * s];
                const R sum = hm + hp;
                h[base] = sum + h0;        // e^0
                h[base + s] = hp - hm;     // e^1
                h[base + 2 * s] = sum;     // e^2
            }
        });
    });
}

// In place: raw moments -> central moments (binomial shift along each axis).
template <int D, class R>
__device__ __forceinline__ void tp_raw_to_central(R (&k)[TP<D>::Q], const R (&u)[3]) {
    static_for<0, D>([&](auto Dd) {
        constexpr int d = decltype(Dd)::value;
        constexpr int s = (d == 0) ? 1 : (d == 1 ? 3 : 9);
        static_for<0, TP<D>::Q>([&](auto B) {
            constexpr int base = decltype(B)::value;
            if constexpr ((base / s) % 3 == 0) {
                const R m0 = k[base], m1 = k[base + s], m2 = k[base + 2 * s];
                const R c1 = m1 - u[d] * m0;
                k[base + s] = c1;
                k[base + 2 * s] = m2 - u[d] * (m1 + c1);   // m2 - 2 u m1 + u^2 m0
            }
        });
    });
}

// rho - rho0 and u from the raw moments of the deviations (Sec. II.A moments).
template <int D, class R>
__device__ __forceinline__ TPMacro<D, R> tp_macro_raw(const R (&m)[TP<D>::Q], R rho0) {
    TPMacro<D, R> r;
    r.drho = m[0];
    const R inv = recip<R>(rho0 + m[0]);
    r.u[0] = m[1] * inv;
    r.u[1] = m[3] * inv;
    r.u[2] = (D == 3) ? m[9] * inv : R(0);
    return r;
}

// In place: central moments -> populations (inverse of the two maps above).
template <int D, class R>
__device__ __forceinline__ void tp_inverse(R (&h)[TP<D>::Q], const R (&u)[3]) {
    static_for<0, D>([&](auto Dd) {
        constexpr int d = decltype(Dd)::value;
        constexpr int s = (d == 0) ? 1 : (d == 1 ? 3 : 9);
        static_for<0, TP<D>::Q>([&](auto B) {
            constexpr int base = decltype(B)::value;
            if constexpr ((base / s) % 3 == 0) {
                const R k0 = h[base], k1 = h[base + s], k2 = h[base + 2 * s];
                const R m1 = k1 + u[d] * k0;          // raw first moment
                const R m2 = k2 + u[d] * (k1 + m1);   // raw second moment
                const R hm1 = R(0.5) * m1;
                h[base + s] = k0 - m2;                // e = 0
                h[base + 2 * s] = R(0.5) * m2 + hm1;  // e = +1
                h[base] = R(0.5) * m2 - hm1;          // e = -1
            }
        });
    });
}

// Deviation equilibrium central moment of multi-index p (digits = orders).
template <int D, int P, class R>
__device__ __forceinline__ R tp_keq(R drho, R rho0, const R (&u)[3], const R (&uu)[3]) {
    constexpr R cs2 = R(1) / R(3);
    R prod = R(1), diff = R(0);  // prod m, prod(m + d) - prod m
    static_for<0, D>([&](auto Dd) {
        constexpr int d = decltype(Dd)::value;
        constexpr int pd = (P / (d == 0 ? 1 : (d == 1 ? 3 : 9))) % 3;
        if constexpr (pd == 0) {
            // m = 1, d = 0: nothing changes
        } else if constexpr (pd == 1) {
            // m = 0, d = -u
            diff = -u[d] * (diff + prod);
            prod = R(0);
        } else {
            // m = c_s^2, d = u^2
            diff = (cs2 + uu[d]) * diff + uu[d] * prod;
            prod = cs2 * prod;
        }
    });
    return drho * prod - rho0 * diff;
}

// Relax central moments of order >= 2 towards equilibrium in place.
// om[n] = omega_n; orders 0 and 1 are conserved and left untouched.
template <int D, class R>
__device__ __forceinline__ void tp_relax(R (&k)[TP<D>::Q], R drho, R rho0, const R (&u)[3],
                                         const R* om) {
    R uu[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};
    static_for<0, TP<D>::Q>([&](auto Pc) {
        constexpr int p = decltype(Pc)::value;
        constexpr int order = p % 3 + (p / 3) % 3 + (D == 3 ? p / 9 : 0);
        if constexpr (order >= 2) {
            const R keq = tp_keq<D, p>(drho, rho0, u, uu);
            k[p] = k[p] + om[order] * (keq - k[p]);
        }
    });
}

// Full collision of one node on deviation populations (in place).
template <int D, class R>
__device__ __forceinline__ void tp_collide(R (&h)[TP<D>::Q], R rho0, const R* om) {
    tp_raw<D, R>(h);
    const TPMacro<D, R> m = tp_macro_raw<D, R>(h, rho0);
    tp_raw_to_central<D, R>(h, m.u);
    tp_relax<D, R>(h, m.drho, rho0, m.u, om);
    tp_inverse<D, R>(h, m.u);
}

// Deviation equilibrium populations for given rho - rho0 and u.
template <int D, class R>
__device__ __forceinline__ void tp_equilibrium(R (&h)[TP<D>::Q], R drho, R rho0, const R (&u)[3]) {
    R uu[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};
    static_for<0, TP<D>::Q>([&](auto Pc) {
        constexpr int p = decltype(Pc)::value;
        h[p] = tp_keq<D, p>(drho, rho0, u, uu);
    });
    tp_inverse<D, R>(h, u);
}

}  // namespace cmlb
