"""Pins of the oracle's global diagnostics (oracle.analysis.globals_of_state).

The fields are trigonometric on anisotropic periodic grids, so every sum has
a closed form: for N >= 3 nodes along an axis, sum sin^2(2 pi x / N) =
sum cos^2 = N / 2 and sum sin cos = sum sin = 0.  The second-order central
difference (a(x+1) - a(x-1)) / 2 of sin(k x) is s cos(k x) with
s = sin(k), so the discrete vorticity is the continuous one with each
derivative scaled by its axis's s.  The states are the oracle's discrete
equilibria of these fields (whose rho, u and second moments are exact,
pinned elsewhere), so mass, momentum, energy, kinetic energy and enstrophy
are known exactly.

What each case catches (the grid sides differ, so s_x, s_y, s_z differ):
  * a Taylor-Green vortex in each coordinate plane: the sign inside each
    vorticity component (d_a u_b - d_b u_a gives (s_a + s_b)^2; a wrong sign
    gives (s_a - s_b)^2);
  * a field whose components each depend on one other axis only: which
    derivative enters which vorticity component (a transposed index swaps
    the s factors);
  * a uniform background velocity: the momentum sum and rho-weighting of
    the kinetic energy; a non-unit density: the rho factor.
"""
import math

import numpy as np
import pytest

from oracle.analysis import globals_of_state

SHAPE3 = (6, 10, 14)   # (nz, ny, nx)
SHAPE2 = (10, 14)      # (ny, nx)


def coords(shape):
    idx = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    xs = list(reversed(idx))   # x, y(, z)
    ns = list(reversed(shape))
    return [2 * math.pi * c / n for c, n in zip(xs, ns)], [math.sin(2 * math.pi / n) for n in ns]


def tgv_in_plane(shape, a, b, u0):
    """u_a = u0 sin A cos B cos C, u_b = -u0 cos A sin B cos C (C the third axis, 3D only)."""
    X, _ = coords(shape)
    D = len(shape)
    c = [d for d in range(D) if d not in (a, b)]
    cosC = np.cos(X[c[0]]) if c else 1.0
    u = np.zeros((D,) + shape)
    u[a] = u0 * np.sin(X[a]) * np.cos(X[b]) * cosC
    u[b] = -u0 * np.cos(X[a]) * np.sin(X[b]) * cosC
    return u


def state(orc, kind, rho, u, theta=None):
    cfg = orc.Cfg(lattice=kind, thermal=theta is not None)
    return orc.init_equilibrium(cfg, rho, u, theta)


def second_moment_trace(orc, kind, theta):
    """D c_s^2 in lattice units: sum_i w_i |e_i|^2 theta = D theta / r^2 (eq:quad, degree >= 2)."""
    L = orc.lattice(kind)
    return L["D"] * theta / L["r"] ** 2


@pytest.mark.parametrize("plane", [(0, 1), (1, 2), (2, 0)])
def test_tgv3d_each_plane(orc, plane):
    u0, c = 0.04, 1.3
    a, b = plane
    rho = np.full(SHAPE3, c)
    u = tgv_in_plane(SHAPE3, a, b, u0)
    g = globals_of_state("D3Q27", state(orc, "D3Q27", rho, u))
    V = float(np.prod(SHAPE3))
    _, s = coords(SHAPE3)
    third = 3 - a - b
    ke = c * u0 ** 2 * V / 8
    ens = 0.5 * u0 ** 2 * V / 8 * ((s[a] + s[b]) ** 2 + 2 * s[third] ** 2)
    assert g["mass"] == pytest.approx(c * V, rel=1e-13)
    assert np.abs(g["momentum"]).max() < 1e-13 * V
    assert g["ke"] == pytest.approx(ke, rel=1e-12)
    assert g["enstrophy"] == pytest.approx(ens, rel=1e-12)
    assert g["energy"] == pytest.approx(ke + 0.5 * c * V * second_moment_trace(orc, "D3Q27", 1.0), rel=1e-12)
    assert g["nonfinite"] == 0


def test_single_axis_fields_3d(orc):
    """u_x = a sin Y, u_y = b sin Z, u_z = c sin X plus a uniform U: the
    vorticity components are -b s_z cos Z, -c s_x cos X, -a s_y cos Y."""
    amp = (0.03, 0.02, 0.045)
    U = np.array([0.01, -0.02, 0.015])
    X, s = coords(SHAPE3)
    u = np.stack([amp[0] * np.sin(X[1]), amp[1] * np.sin(X[2]), amp[2] * np.sin(X[0])]) + U[:, None, None, None]
    rho = np.ones(SHAPE3)
    g = globals_of_state("D3Q27", state(orc, "D3Q27", rho, u))
    V = float(np.prod(SHAPE3))
    ens = 0.25 * V * (amp[1] ** 2 * s[2] ** 2 + amp[2] ** 2 * s[0] ** 2 + amp[0] ** 2 * s[1] ** 2)
    ke = 0.5 * V * (sum(a * a for a in amp) / 2 + U @ U)
    assert np.allclose(g["momentum"], V * U, rtol=1e-12, atol=0)
    assert g["ke"] == pytest.approx(ke, rel=1e-12)
    assert g["enstrophy"] == pytest.approx(ens, rel=1e-12)


@pytest.mark.parametrize("kind", ["D2Q9", "D2Q37"])
def test_tgv2d_and_single_axis(orc, kind):
    u0, c, theta0 = 0.03, 0.9, 1.1
    thermal = kind == "D2Q37"
    V = float(np.prod(SHAPE2))
    X, s = coords(SHAPE2)
    rho = np.full(SHAPE2, c)
    th = np.full(SHAPE2, theta0) if thermal else None
    trace = second_moment_trace(orc, kind, theta0 if thermal else 1.0)
    # Taylor-Green: omega = u0 (s_x + s_y) sin X sin Y
    g = globals_of_state(kind, state(orc, kind, rho, tgv_in_plane(SHAPE2, 0, 1, u0), th))
    ke = c * u0 ** 2 * V / 4
    assert g["mass"] == pytest.approx(c * V, rel=1e-13)
    assert g["ke"] == pytest.approx(ke, rel=1e-12)
    assert g["enstrophy"] == pytest.approx(0.5 * u0 ** 2 * V / 4 * (s[0] + s[1]) ** 2, rel=1e-12)
    assert g["energy"] == pytest.approx(ke + 0.5 * c * V * trace, rel=1e-12)
    # u_x = a sin Y, u_y = b sin X: omega = b s_x cos X - a s_y cos Y
    a, b = 0.02, 0.035
    u = np.stack([a * np.sin(X[1]), b * np.sin(X[0])])
    g = globals_of_state(kind, state(orc, kind, rho, u, th))
    assert g["enstrophy"] == pytest.approx(0.25 * V * (b * b * s[0] ** 2 + a * a * s[1] ** 2), rel=1e-12)
    assert g["ke"] == pytest.approx(0.5 * c * V * (a * a + b * b) / 2, rel=1e-12)


def test_nonfinite_count(orc):
    S = state(orc, "D3Q27", np.ones(SHAPE3), tgv_in_plane(SHAPE3, 0, 1, 0.02))
    S[3, 1, 2, 3] = np.nan
    S[20, 0, 0, 0] = np.inf
    S[26, 5, 9, 13] = -np.inf
    assert globals_of_state("D3Q27", S)["nonfinite"] == 3
