"""Plain-definition analysis for the oracle (test infrastructure only).

* transport coefficients from relaxation times (Chapman-Enskog, Sec. II.C
  eq:sigma, with the lattice correction tau - 1/2);
* single-wavenumber mode amplitudes and exponential-decay fits (Sec. III.A);
* the closed-form dispersion relations eq:dr;
* global FP64 diagnostics of a state (mass, momentum, energy, kinetic energy,
  enstrophy, non-finite count).
"""
from __future__ import annotations

import numpy as np

from . import collide, equilibrium, lattice


def nu_lattice(kind: str, tau2: float, theta: float = 1.0) -> float:
    """Kinematic viscosity in lattice units: nu_xi = theta (tau2 - 1/2), nu_lat = nu_xi / r^2."""
    r = lattice(kind)["r"]
    return theta * (tau2 - 0.5) / r ** 2


def tau_from_nu_xi(nu_xi: float, theta: float = 1.0) -> float:
    """Relaxation time giving a diffusivity nu_xi (xi-units) at temperature theta."""
    return 0.5 + nu_xi / theta


def mode_amplitude(field: np.ndarray, kvec) -> complex:
    """(2/N) sum_x field(x) exp(-i k.x) for integer mode numbers kvec (x fastest)."""
    shape = field.shape
    idx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    coords = list(reversed(idx))
    phase = sum(2 * np.pi * kvec[d] * coords[d] / shape[::-1][d] for d in range(len(kvec)))
    return 2.0 * np.sum(field * np.exp(-1j * phase)) / field.size


def fit_decay(t, amp) -> float:
    """Least-squares slope of -ln|amp| against t (a positive decay rate)."""
    t = np.asarray(t, np.float64)
    y = np.log(np.abs(np.asarray(amp)))
    A = np.stack([t, np.ones_like(t)], 1)
    slope = np.linalg.lstsq(A, y, rcond=None)[0][0]
    return -slope


def fit_damped_cosine(t, a, alpha0: float, omega0: float):
    """Least-squares fit of a(t) = A exp(-alpha t) cos(Omega t + phi) (the
    standing acoustic wave of Sec. III.A, eq:modes); returns (alpha, Omega).
    alpha0 and omega0 start the iteration."""
    from scipy.optimize import least_squares
    t = np.asarray(t, np.float64)
    a = np.asarray(a, np.float64)
    p0 = [a[0], alpha0, omega0, 0.0]
    res = least_squares(lambda p: p[0] * np.exp(-p[1] * t) * np.cos(p[2] * t + p[3]) - a, p0,
                        x_scale=[abs(a[0]), abs(alpha0), abs(omega0), 1.0], xtol=1e-14, ftol=1e-14, gtol=1e-14)
    return res.x[1], res.x[2]


def dispersion(nu: float, kappa: float, theta0: float, k: float, D: int = 2):
    """Closed forms eq:dr (all quantities in xi-units).

    Returns (viscous decay rate, thermal decay rate, acoustic decay rate,
    acoustic angular frequency), rates positive; gamma = (D + 2) / D.
    """
    g = (D + 2.0) / D
    cs = np.sqrt(g * theta0)
    pr = nu / kappa
    lam = 1.0 + (g - 3.0) * pr
    pe = cs / (kappa * k)
    visc = nu * k * k
    therm = cs * k * (1.0 / pe + (g - 1.0) * lam / pe ** 3)
    ac_re = cs * k * ((g - lam) / (2 * pe) - (g - 1.0) * lam / (2 * pe ** 3))
    ac_im = cs * k * (1.0 - ((g + lam) ** 2 - 4 * lam) / (8 * pe ** 2))
    return visc, therm, ac_re, ac_im


def globals_of_state(kind: str, S: np.ndarray) -> dict:
    """FP64 global diagnostics: mass, momentum (lattice units), energy
    (sum f |e|^2 / 2, lattice units), kinetic energy 1/2 sum rho |u|^2,
    enstrophy 1/2 sum |curl u|^2 with second-order central differences on the
    periodic grid, and the count of non-finite populations."""
    L = lattice(kind)
    Q, D = L["Q"], L["D"]
    e = L["e"][:, :D].astype(np.float64)
    F = S.reshape(Q, -1)
    nonfinite = int((~np.isfinite(F)).sum())
    rho = F.sum(0)
    mom = e.T @ F
    u = mom / rho
    energy = 0.5 * ((e ** 2).sum(1) @ F).sum()
    ke = 0.5 * (rho * (u ** 2).sum(0)).sum()
    shape = S.shape[1:]
    uf = u.reshape((D,) + shape)

    def ddx(a, d):  # derivative along spatial direction d (0 = x = last axis)
        ax = a.ndim - 1 - d
        return 0.5 * (np.roll(a, -1, axis=ax) - np.roll(a, 1, axis=ax))

    if D == 2:
        wz = ddx(uf[1], 0) - ddx(uf[0], 1)
        ens = 0.5 * (wz ** 2).sum()
    else:
        wx = ddx(uf[2], 1) - ddx(uf[1], 2)
        wy = ddx(uf[0], 2) - ddx(uf[2], 0)
        wz = ddx(uf[1], 0) - ddx(uf[0], 1)
        ens = 0.5 * (wx ** 2 + wy ** 2 + wz ** 2).sum()
    return dict(mass=rho.sum(), momentum=mom.sum(1), energy=energy, ke=ke,
                enstrophy=ens, nonfinite=nonfinite)


def collision_jacobian(cfg, u_lat, theta=1.0, h=1e-6):
    """d f* / d f of the oracle collision at the equilibrium of (rho = 1, u),
    by central differences (linearised operator of Sec. II.C)."""
    L = lattice(cfg.lattice)
    Q = L["Q"]
    f0 = equilibrium(cfg.lattice, 1.0, u_lat, theta)
    plus = collide(cfg, f0[None] + h * np.eye(Q))
    minus = collide(cfg, f0[None] - h * np.eye(Q))
    return ((plus - minus) / (2 * h)).T


def spectral_radius(cfg, u_lat, theta=1.0, nk=9):
    """Largest |eigenvalue| of the linearised stream-and-collide update
    A(k) = diag(exp(-i k.e_i)) J over a grid of wave vectors k in [0, pi]^D
    (von Neumann analysis); > 1 means a growing mode."""
    L = lattice(cfg.lattice)
    D = L["D"]
    e = L["e"][:, :D]
    J = collision_jacobian(cfg, u_lat, theta)
    ks = np.linspace(0.0, np.pi, nk)
    best, arg = 0.0, None
    for k in np.stack(np.meshgrid(*[ks] * D, indexing="ij"), -1).reshape(-1, D):
        S = np.exp(-1j * (e @ k))
        r = np.abs(np.linalg.eigvals(S[:, None] * J)).max()
        if r > best:
            best, arg = r, k
    return best, arg
