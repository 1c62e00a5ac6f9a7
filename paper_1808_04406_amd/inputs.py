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
