"""Seeded synthetic inputs: initial macroscopic fields and random perturbations.

This module holds no lattice-Boltzmann arithmetic.  It produces the fields
(rho, u, theta) of the workloads (Taylor-Green vortices, decaying shear and
thermal waves, random-phase multi-mode velocity fields) and seeded random
arrays.  The HIP path and the FP64 oracle each turn these into populations
with their own code.

Conventions: fields are numpy float64 arrays shaped ``[(nz,) ny, nx]`` (x
fastest); velocities are ``[D, (nz,) ny, nx]`` in lattice units (cells per
step); node positions are the integer indices (x = i).
"""
from __future__ import annotations

import numpy as np


def grid(shape):
    """Integer coordinate arrays (x, y[, z]) for a grid shaped [(nz,) ny, nx]."""
    idx = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    return tuple(reversed(idx))


def tgv2d(nx: int, ny: int, u0: float, cs2: float = 1.0 / 3.0, rho0: float = 1.0):
    """2D Taylor-Green vortex with one period across the box.

    u = u0 (sin kx cos ky, -cos kx sin ky), rho from the pressure solution
    p = p0 - (rho0 u0^2 / 4)(cos 2kx + cos 2ky) with p = cs2 rho.
    """
    x, y = grid((ny, nx))
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    u = np.stack([u0 * np.sin(kx * x) * np.cos(ky * y), -u0 * np.cos(kx * x) * np.sin(ky * y)])
    rho = rho0 - rho0 * u0 ** 2 / (4 * cs2) * (np.cos(2 * kx * x) + np.cos(2 * ky * y))
    return rho, u


def tgv3d(n: int, u0: float, cs2: float = 1.0 / 3.0, rho0: float = 1.0, background=(0.0, 0.0, 0.0)):
    """3D Taylor-Green vortex on an n^3 periodic box, L = n / (2 pi).

    u = u0 (sin X cos Y cos Z, -cos X sin Y cos Z, 0) with X = x / L, plus a
    uniform background velocity; rho from the pressure solution
    p = p0 + (rho0 u0^2 / 16)(cos 2X + cos 2Y)(cos 2Z + 2), p = cs2 rho.
    """
    x, y, z = grid((n, n, n))
    X, Y, Z = (2 * np.pi / n) * x, (2 * np.pi / n) * y, (2 * np.pi / n) * z
    u = np.stack([u0 * np.sin(X) * np.cos(Y) * np.cos(Z) + background[0],
                  -u0 * np.cos(X) * np.sin(Y) * np.cos(Z) + background[1],
                  np.zeros_like(X) + background[2]])
    rho = rho0 + rho0 * u0 ** 2 / (16 * cs2) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2)
    return rho, u


def waves2d(nx: int, ny: int, shear_amp: float = 0.0, thermal_amp: float = 0.0,
            k=(1, 0), kt=None, background=(0.0, 0.0), rho0: float = 1.0, theta0: float = 1.0):
    """Decaying linear modes on an nx x ny periodic grid.

    Shear wave: velocity perpendicular to k, u_perp = shear_amp sin(k.x).
    Thermal wave (wave vector kt, default k): isobaric,
    theta = theta0 (1 + thermal_amp sin(kt.x)), rho = rho0 theta0 / theta.
    A uniform background velocity is added.  k are integer mode numbers.
    """
    kt = k if kt is None else kt
    x, y = grid((ny, nx))
    kv = np.array([2 * np.pi * k[0] / nx, 2 * np.pi * k[1] / ny])
    kvt = np.array([2 * np.pi * kt[0] / nx, 2 * np.pi * kt[1] / ny])
    phase = kv[0] * x + kv[1] * y
    phase_t = kvt[0] * x + kvt[1] * y
    perp = np.array([-kv[1], kv[0]]) / np.linalg.norm(kv)
    u = np.stack([background[0] + shear_amp * perp[0] * np.sin(phase),
                  background[1] + shear_amp * perp[1] * np.sin(phase)])
    theta = theta0 * (1.0 + thermal_amp * np.sin(phase_t))
    rho = rho0 * theta0 / theta
    return rho, u, theta


def nsf_modes(nu: float, kappa: float, theta0: float, k: float, dim: int = 2, rho0: float = 1.0):
    """Eigen-system of the Navier-Stokes-Fourier equations linearised about a
    uniform state at rest, for one wave e^(omega t + i k x) (Sec. III.A).

    Units are the paper's (velocities scaled by sqrt(kT/m), so p = rho theta,
    c_v = D/2, gamma = (D + 2)/D).  The monatomic stress has no bulk part,
    so the longitudinal viscosity is 2 (1 - 1/D) nu; heat conducts with
    diffusivity kappa = lambda / (rho c_p).  Variables (rho~, u~_par, theta~):

        omega rho~   = -i k rho0 u~_par
        omega u~_par = -i k (theta0 rho~ / rho0 + theta~) - 2 (1 - 1/D) nu k^2 u~_par
        omega theta~ = -i k (2/D) theta0 u~_par - gamma kappa k^2 theta~

    and omega = -nu k^2 for u~_perp.  Returns a dict with the thermal root
    (real), the acoustic pair (omega_plus with positive imaginary part) and
    their eigenvectors (rho~, u~_par, theta~), each scaled to rho~ = 1 for the
    acoustic pair and theta~ = 1 for the thermal mode.
    """
    g = (dim + 2.0) / dim
    A = np.array([[0.0, -1j * k * rho0, 0.0],
                  [-1j * k * theta0 / rho0, -2.0 * (1.0 - 1.0 / dim) * nu * k * k, -1j * k],
                  [0.0, -1j * k * (2.0 / dim) * theta0, -g * kappa * k * k]], dtype=complex)
    w, V = np.linalg.eig(A)
    it = int(np.argmin(np.abs(w.imag)))
    ip = int(np.argmax(w.imag))
    im = int(np.argmin(w.imag))
    return {"viscous": -nu * k * k,
            "thermal": w[it].real, "thermal_vec": V[:, it] / V[2, it],
            "plus": w[ip], "plus_vec": V[:, ip] / V[0, ip],
            "minus": w[im], "minus_vec": V[:, im] / V[0, im]}


def linear_modes(n: int, nu: float, kappa: float, theta0: float, r: float, amp=(0.001, 0.001, 0.001),
                 k_viscous=(1, 0), k_thermal=(1, 1), k_acoustic=(1, 0), background=(0.0, 0.0), rho0: float = 1.0):
    """Superposition of a viscous wave, a thermal wave and a standing acoustic
    wave on an n x n periodic grid, each built from the eigenvectors of
    ``nsf_modes`` (Sec. III.A, Fig. 1 setup), plus a uniform background
    velocity.

    Velocities are in the paper's units inside and are returned in lattice
    units (divided by r, the lattice scale of the quadrature); a mode number m
    along an axis is the wave number 2 pi m / (n r).  amp = (a_v, a_t, a_a):
    u~_perp = a_v (viscous); theta~ = a_t theta0 (thermal); rho~ = a_a rho0
    (acoustic, sum of the omega_plus and omega_minus waves, so the density
    is a_a rho0 cos(k.x) at t = 0).  The background velocity is in the
    paper's units too.
    """
    a_v, a_t, a_a = amp
    x, y = grid((n, n))
    rho = np.full((n, n), rho0)
    u = np.zeros((2, n, n))
    theta = np.full((n, n), theta0)

    def wave(m):
        kv = 2 * np.pi * np.array(m, float) / (n * r)
        kk = float(np.linalg.norm(kv))
        phase = 2 * np.pi * (m[0] * x + m[1] * y) / n
        return kv / kk, kk, np.exp(1j * phase)

    # viscous: u_perp only
    e, kk, ph = wave(k_viscous)
    perp = np.array([-e[1], e[0]])
    up = (a_v * ph).real
    u += perp[:, None, None] * up
    # thermal mode
    e, kk, ph = wave(k_thermal)
    vec = nsf_modes(nu, kappa, theta0, kk, 2, rho0)["thermal_vec"] * (a_t * theta0)
    rho += (vec[0] * ph).real
    u += e[:, None, None] * (vec[1] * ph).real
    theta += (vec[2] * ph).real
    # standing acoustic wave
    e, kk, ph = wave(k_acoustic)
    m = nsf_modes(nu, kappa, theta0, kk, 2, rho0)
    vec = 0.5 * (m["plus_vec"] + m["minus_vec"]) * (a_a * rho0)
    rho += (vec[0] * ph).real
    u += e[:, None, None] * (vec[1] * ph).real
    theta += (vec[2] * ph).real
    u[0] += background[0]
    u[1] += background[1]
    return rho, u / r, theta


def double_shear_layer(n: int, u0: float, sharpness: float = 80.0, delta: float = 0.05, rho0: float = 1.0,
                       theta0: float = 1.0):
    """Double shear layer on the unit square sampled at x = i/n, y = j/n
    (Sec. III.B): u_x = u0 tanh(sharpness (y - 1/4)) for y <= 1/2 and
    u0 tanh(sharpness (3/4 - y)) above; u_y = delta u0 sin(2 pi (x + 1/4));
    uniform rho and theta.  u0 is in the caller's velocity units."""
    x, y = grid((n, n))
    x, y = x / n, y / n
    ux = np.where(y <= 0.5, u0 * np.tanh(sharpness * (y - 0.25)), u0 * np.tanh(sharpness * (0.75 - y)))
    uy = delta * u0 * np.sin(2 * np.pi * (x + 0.25))
    return np.full((n, n), rho0), np.stack([ux, uy]), np.full((n, n), theta0)


def random_multimode(n: int, seed: int, kmax: int = 4, umax: float = 0.05, dim: int = 3):
    """Random-phase solenoidal velocity field on an n^dim periodic grid.

    Every integer mode k with 1 <= |k| <= kmax gets a complex Gaussian
    amplitude vector from ``numpy.random.default_rng(seed)`` (drawn on the
    (2 kmax + 1)^dim mode box, so the field does not depend on n), projected
    onto the plane normal to k; u is the real part of the mode sum, scaled so
    that max |u| = umax.  The sum is evaluated exactly by separable
    transforms (small DFTs along x and y, one matrix product along z).
    rho = 1.
    """
    rng = np.random.default_rng(seed)
    m = 2 * kmax + 1
    ks = np.arange(-kmax, kmax + 1)
    kk = np.stack(np.meshgrid(*[ks] * dim, indexing="ij"))[::-1]  # kk[d] along axis d (x first)
    kmag = np.sqrt((kk ** 2).sum(0))
    mask = (kmag >= 1) & (kmag <= kmax)
    amp = (rng.normal(size=(dim,) + (m,) * dim) + 1j * rng.normal(size=(dim,) + (m,) * dim)) * mask
    with np.errstate(invalid="ignore", divide="ignore"):
        kdotA = (kk * amp).sum(0) / np.where(kmag > 0, kmag ** 2, 1.0)
    amp = amp - kk * kdotA
    pos = np.arange(n)
    E = np.exp(2j * np.pi * np.outer(ks, pos) / n)           # [mode, position]
    u = np.empty((dim,) + (n,) * dim)
    for d in range(dim):
        a = amp[d]                                            # axes (kz,) ky, kx
        if dim == 3:
            b = np.einsum("zyk,kx->zyx", a, E)                # along x
            c = np.einsum("zkx,ky->zyx", b, E)                # along y: [kz, y, x]
            u[d] = (E.T @ c.reshape(m, n * n)).real.reshape(n, n, n)
        else:
            b = np.einsum("yk,kx->yx", a, E)
            u[d] = (E.T @ b).real
    u *= umax / np.sqrt((u ** 2).sum(0)).max()
    return np.ones((n,) * dim), u


def random_fields(shape, seed: int, drho: float = 0.05, umax: float = 0.05, dtheta: float = 0.0):
    """Independent random rho, u, theta per node (for one-step parity cases)."""
    rng = np.random.default_rng(seed)
    dim = len(shape)
    rho = 1.0 + drho * rng.uniform(-1, 1, size=shape)
    u = umax * rng.uniform(-1, 1, size=(dim,) + tuple(shape))
    theta = 1.0 + dtheta * rng.uniform(-1, 1, size=shape)
    return rho, u, theta


def perturbation(shape, seed: int, eps: float):
    """Seeded multiplicative noise 1 + eps N(0, 1) of the given shape."""
    rng = np.random.default_rng(seed)
    return 1.0 + eps * rng.normal(size=shape)
