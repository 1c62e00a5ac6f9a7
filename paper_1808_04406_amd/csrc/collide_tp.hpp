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
// (f_-, f_0, f_+) -> (kappa_0, kappa_1, kappa_2) along each axis; its inverse
// is analytic.  All arithmetic is on deviations h_i = f_i - w_i rho0: the
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

// rho - rho0 and u from the deviation populations (Sec. II.A moments).
template <int D, class R>
__device__ __forceinline__ TPMacro<D, R> tp_macro(const R (&h)[TP<D>::Q], R rho0) {
    R s = R(0), j[3] = {R(0), R(0), R(0)};
    static_for<0, TP<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        s += h[i];
        if constexpr (TP<D>::ex(i) == 1) j[0] += h[i];
        if constexpr (TP<D>::ex(i) == -1) j[0] -= h[i];
        if constexpr (TP<D>::ey(i) == 1) j[1] += h[i];
        if constexpr (TP<D>::ey(i) == -1) j[1] -= h[i];
        if constexpr (TP<D>::ez(i) == 1) j[2] += h[i];
        if constexpr (TP<D>::ez(i) == -1) j[2] -= h[i];
    });
    TPMacro<D, R> m;
    m.drho = s;
    const R inv = R(1) / (rho0 + s);
    m.u[0] = j[0] * inv;
    m.u[1] = j[1] * inv;
    m.u[2] = (D == 3) ? j[2] * inv : R(0);
    return m;
}

// In place: populations (slot digit e+1 along each axis) -> central moments
// (slot digit = order along each axis).
template <int D, class R>
__device__ __forceinline__ void tp_forward(R (&h)[TP<D>::Q], const R (&u)[3]) {
    static_for<0, D>([&](auto Dd) {
        constexpr int d = decltype(Dd)::value;
        constexpr int s = (d == 0) ? 1 : (d == 1 ? 3 : 9);
        static_for<0, TP<D>::Q>([&](auto B) {
            constexpr int base = decltype(B)::value;
            if constexpr ((base / s) % 3 == 0) {
                const R hm = h[base], h0 = h[base + s], hp = h[base + 2 * s];
                const R sum = hm + hp, dif = hp - hm;
                const R k0 = sum + h0;
                const R k1 = dif - u[d] * k0;
                const R k2 = sum - u[d] * (dif + k1);
                h[base] = k0;
                h[base + s] = k1;
                h[base + 2 * s] = k2;
            }
        });
    });
}

// In place: central moments -> populations (inverse of tp_forward).
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
                h[base + s] = k0 - m2;                // e = 0
                h[base + 2 * s] = R(0.5) * (m2 + m1); // e = +1
                h[base] = R(0.5) * (m2 - m1);         // e = -1
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
    const TPMacro<D, R> m = tp_macro<D, R>(h, rho0);
    tp_forward<D, R>(h, m.u);
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
