"""FP64 CPU oracle for the central-moment MRT lattice Boltzmann update.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product library.  It shares
no code with the HIP path.  The arithmetic lives in ``cmlb_oracle.c`` (plain C,
double precision); this module only marshals numpy arrays through ctypes, plus
plain-definition analysis helpers (mode amplitudes, decay fits, closed-form
dispersion relations, global diagnostics) in :mod:`oracle.analysis`.

Lattice kinds: ``"D2Q9"``, ``"D3Q27"``, ``"D2Q37"`` (also ``"E9A"``), and
the other minimal 2D rules of Fig. 2: ``"E9B"``-``"E9D"`` (37 velocities,
degree 9, N = M = 4) and ``"E7A"``-``"E7D"`` (17 velocities, degree 7,
N = M = 3).  Velocities crossing
this API are in lattice units (cells per step); theta is the paper's
dimensionless temperature (reference value 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cmlb_oracle.c")
_LIB = os.path.join(_HERE, "libcmlb_oracle.so")

KINDS = {"D2Q9": 0, "D3Q27": 1, "D2Q37": 2, "E9B": 3, "E9C": 4, "E9D": 5,
         "E7A": 6, "E7B": 7, "E7C": 8, "E7D": 9}
# the ninth-degree 37-velocity rule on |e|^2 <= 10 is also called E9A
KINDS["E9A"] = KINDS["D2Q37"]
MODELS = {"cm": 0, "raw_mrt": 1, "reg_bgk": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        d, i, l = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_long
        L.orc_lattice_info.argtypes = [ctypes.c_int, i, i, i, d, d, d]
        L.orc_hermite.argtypes = [ctypes.c_int, ctypes.c_int, d, d]
        L.orc_symprod.argtypes = [ctypes.c_int, ctypes.c_int, d, ctypes.c_int, d, d]
        L.orc_maxwell_coeffs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, d, ctypes.c_double, d]
        L.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, d, ctypes.c_double, d]
        L.orc_collide.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, d, d]
        L.orc_collide_definitional.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, d, d]
        L.orc_run.argtypes = [ctypes.POINTER(_Cfg), l, l, l, d, l, ctypes.c_int]
        L.orc_step_nodes.argtypes = [ctypes.POINTER(_Cfg), l, l, l, d, l,
                                     ctypes.POINTER(ctypes.c_int64), d, ctypes.c_int]
        L.orc_init_equilibrium.argtypes = [ctypes.POINTER(_Cfg), l, l, l, d, d, d, d, ctypes.c_int]
        L.orc_moments.argtypes = [ctypes.c_int, l, d, d, d, d]
        L.orc_mlp_forward.argtypes = [d, ctypes.c_int, d, d]
        L.orc_closure_inputs.argtypes = [ctypes.c_int, d, d, d]
        L.orc_collide_closure.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, d, d, d, ctypes.c_int, d, d]
        L.orc_closure_loss_grad.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, d, d, d, d, ctypes.c_int, d, d]
        L.orc_closure_loss_offsets.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, d, d, d, d, ctypes.c_int, d, d]
        L.orc_closure_eval_rounded.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, d, d, d, d, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_double, d, d, d, d, d, d, d, d, d]
        L.orc_round_sig.argtypes = [ctypes.c_int, d, ctypes.c_int, d]
        L.orc_gather_nodes.argtypes = [ctypes.c_int, l, l, l, d, l, ctypes.POINTER(ctypes.c_int64), d]
        _lib = L
    return _lib


class _Cfg(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("model", ctypes.c_int), ("thermal", ctypes.c_int),
                ("pad", ctypes.c_int), ("theta0", ctypes.c_double),
                ("omega", ctypes.c_double * 8), ("delta_coef", ctypes.c_double)]


@dataclass
class Cfg:
    """Collision configuration.

    ``tau[n]`` is the relaxation time of central-moment order n (the paper's
    omega_n = 1/tau_n, eq:omega); orders missing from the dict use ``tau_hi``.
    ``delta_coef`` is the coefficient of the delta term of the fourth-order
    relaxation (eq:mrt): 6 follows from eq:omega, 72 is as printed.
    """
    lattice: str = "D3Q27"
    tau: dict = field(default_factory=lambda: {2: 0.8})
    tau_hi: float = 1.0
    model: str = "cm"
    thermal: bool = False
    theta0: float = 1.0
    delta_coef: float = 6.0

    def omega(self):
        return [0.0, 0.0] + [1.0 / self.tau.get(n, self.tau_hi) for n in range(2, 8)]

    def c(self):
        c = _Cfg()
        c.lattice = KINDS[self.lattice]
        c.model = MODELS[self.model]
        c.thermal = 1 if self.thermal else 0
        c.theta0 = self.theta0
        for n, w in enumerate(self.omega()):
            c.omega[n] = w
        c.delta_coef = self.delta_coef
        return c


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice(kind: str):
    """Quadrature table: dict(D, Q, e (Q,3) int, w (Q,), r, resid, N) with N
    the Hermite truncation N = M the oracle uses on the lattice (0: the
    complete tensor-product basis of D2Q9/D3Q27)."""
    D, Q = ctypes.c_int(), ctypes.c_int()
    e = np.zeros(37 * 3, np.int32)
    w = np.zeros(37)
    r, resid = ctypes.c_double(), ctypes.c_double()
    rc = lib().orc_lattice_info(KINDS[kind], ctypes.byref(D), ctypes.byref(Q),
                                e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(w),
                                ctypes.byref(r), ctypes.byref(resid))
    if rc:
        raise RuntimeError("oracle lattice failed")
    q = Q.value
    return dict(D=D.value, Q=q, e=e[:3 * q].reshape(q, 3).astype(np.int64), w=w[:q].copy(),
                r=r.value, resid=resid.value, N={37: 4, 17: 3}.get(q, 0))


def hermite(D: int, nmax: int, xi) -> list:
    """Tensor Hermite polynomials H^(0..nmax)(xi) as full index arrays."""
    xi = np.ascontiguousarray(xi, np.float64)
    n_tot = sum(D ** k for k in range(nmax + 1))
    H = np.zeros(n_tot)
    if lib().orc_hermite(D, nmax, _p(xi), _p(H)):
        raise ValueError("bad hermite request")
    out, o = [], 0
    for k in range(nmax + 1):
        out.append(H[o:o + D ** k].reshape((D,) * k) if k else H[o:o + 1].reshape(()))
        o += D ** k
    return out


def symprod(A, B):
    """Symmetric product Sym(A (x) B) of two full-index tensors."""
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    D = (A.shape + B.shape)[0]
    out = np.zeros((D,) * (A.ndim + B.ndim))
    if lib().orc_symprod(D, A.ndim, _p(A.reshape(-1)), B.ndim, _p(B.reshape(-1)), _p(out)):
        raise ValueError("rank too high")
    return out


def maxwell_coeffs(D: int, nmax: int, rho: float, u_xi, theta: float) -> list:
    """Hermite coefficients a^(0..nmax) of the Maxwellian (u in xi-units)."""
    u = np.zeros(3)
    u[:D] = u_xi
    n_tot = sum(D ** k for k in range(nmax + 1))
    a = np.zeros(n_tot)
    if lib().orc_maxwell_coeffs(D, nmax, rho, _p(u), theta, _p(a)):
        raise ValueError("nmax > 4")
    out, o = [], 0
    for k in range(nmax + 1):
        out.append(a[o:o + D ** k].reshape((D,) * k) if k else a[o:o + 1].reshape(()))
        o += D ** k
    return out


def equilibrium(kind: str, rho: float, u_lat, theta: float = 1.0) -> np.ndarray:
    u = np.zeros(3)
    u[:len(u_lat)] = u_lat
    f0 = np.zeros(37)
    lib().orc_equilibrium(KINDS[kind], rho, _p(u), theta, _p(f0))
    return f0[:lattice(kind)["Q"]].copy()


def collide(cfg: Cfg, f: np.ndarray) -> np.ndarray:
    """Post-collision populations for a batch of nodes f[n, Q] (paper's route)."""
    f = np.ascontiguousarray(np.atleast_2d(f), np.float64)
    out = np.zeros_like(f)
    c = cfg.c()
    if lib().orc_collide(ctypes.byref(c), f.shape[0], _p(f), _p(out)):
        raise RuntimeError("collide failed")
    return out


def collide_definitional(cfg: Cfg, f: np.ndarray) -> np.ndarray:
    """Post-collision populations from the defining moment conditions (dense solve)."""
    f = np.ascontiguousarray(np.atleast_2d(f), np.float64)
    out = np.zeros_like(f)
    c = cfg.c()
    if lib().orc_collide_definitional(ctypes.byref(c), f.shape[0], _p(f), _p(out)):
        raise RuntimeError("singular moment system")
    return out


def _dims(S):
    Q = S.shape[0]
    if S.ndim == 3:
        return Q, 1, S.shape[1], S.shape[2]
    return Q, S.shape[1], S.shape[2], S.shape[3]


def run(cfg: Cfg, S: np.ndarray, nsteps: int, threads: int | None = None) -> np.ndarray:
    """Advance the state S[Q, (nz,) ny, nx] by nsteps pull-stream + collide steps (in place)."""
    assert S.dtype == np.float64 and S.flags.c_contiguous
    Q, nz, ny, nx = _dims(S)
    threads = threads or os.cpu_count() or 1
    if lib().orc_run(ctypes.byref(cfg.c()), nx, ny, nz, _p(S), nsteps, threads):
        raise RuntimeError("run failed")
    return S


def step_nodes(cfg: Cfg, S: np.ndarray, nodes, threads: int | None = None) -> np.ndarray:
    """One step of state S evaluated at flat node indices; returns [n, Q]."""
    S = np.ascontiguousarray(S, np.float64)
    Q, nz, ny, nx = _dims(S)
    nodes = np.ascontiguousarray(nodes, np.int64)
    out = np.zeros((len(nodes), Q))
    threads = threads or os.cpu_count() or 1
    lib().orc_step_nodes(ctypes.byref(cfg.c()), nx, ny, nz, _p(S), len(nodes),
                         nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out), threads)
    return out


def init_equilibrium(cfg: Cfg, rho: np.ndarray, u: np.ndarray, theta=None,
                     threads: int | None = None) -> np.ndarray:
    """S_0 = f0(rho, u, theta) on a grid; rho[(nz,)ny,nx], u[D, ...]."""
    L = lattice(cfg.lattice)
    rho = np.ascontiguousarray(rho, np.float64)
    shape = rho.shape
    nz, ny, nx = (1,) + shape if rho.ndim == 2 else shape
    u = np.ascontiguousarray(u, np.float64)
    th = None if theta is None else np.ascontiguousarray(theta, np.float64)
    S = np.zeros((L["Q"],) + shape)
    threads = threads or os.cpu_count() or 1
    lib().orc_init_equilibrium(ctypes.byref(cfg.c()), nx, ny, nz, _p(rho), _p(u),
                               None if th is None else _p(th), _p(S), threads)
    return S


def moments(kind: str, S: np.ndarray):
    """rho, u (lattice units, [D, ...]) and theta of a state."""
    L = lattice(kind)
    S = np.ascontiguousarray(S, np.float64)
    shape = S.shape[1:]
    n = int(np.prod(shape))
    rho = np.zeros(shape)
    u = np.zeros((L["D"],) + shape)
    th = np.zeros(shape)
    lib().orc_moments(KINDS[kind], n, _p(S), _p(rho), _p(u), _p(th))
    return rho, u, th


# ---------------------------------------------------------------------------
# Learned closure (D3Q27): a per-node MLP sets the rates of orders 3..6
# ---------------------------------------------------------------------------
MLP_NPARAM = 2084


def mlp_rates(params, x):
    """omega_3..omega_6 = 0.5 + 1.45 sigmoid(MLP(x)) for inputs x[n, 27]."""
    params = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
    out = np.zeros((x.shape[0], 4))
    lib().orc_mlp_forward(_p(params), x.shape[0], _p(x), _p(out))
    return out


def closure_inputs(f, norm):
    """Network inputs (kappa_p - kappa_eq,p) / (rho sigma_p) of D3Q27 states f[n, 27]."""
    f = np.ascontiguousarray(np.atleast_2d(f), np.float64)
    norm = np.ascontiguousarray(norm, np.float64)
    x = np.zeros_like(f)
    lib().orc_closure_inputs(f.shape[0], _p(f), _p(norm), _p(x))
    return x


def collide_closure(cfg: Cfg, f, params, norm, tie_even=False):
    """D3Q27 collision with network rates; returns (f*[n, 27], omega[n, 4]).
    tie_even: orders 4 and 6 relax at omega_2 instead of the network's rate."""
    f = np.ascontiguousarray(np.atleast_2d(f), np.float64)
    out = np.zeros_like(f)
    om = np.zeros((f.shape[0], 4))
    rc = lib().orc_collide_closure(ctypes.byref(cfg.c()), f.shape[0], _p(f),
                                   _p(np.ascontiguousarray(params, np.float64)),
                                   _p(np.ascontiguousarray(norm, np.float64)), 1 if tie_even else 0,
                                   _p(out), _p(om))
    if rc:
        raise RuntimeError("closure collision needs a D3Q27 CM configuration")
    return out, om


def closure_loss_grad(cfg: Cfg, f, fbar, params, norm, tie_even=False):
    """Mean over nodes of sum_i (f*_i - fbar_i)^2 / w_i and its gradient."""
    f = np.ascontiguousarray(np.atleast_2d(f), np.float64)
    fbar = np.ascontiguousarray(np.atleast_2d(fbar), np.float64)
    loss = ctypes.c_double()
    grad = np.zeros(MLP_NPARAM)
    rc = lib().orc_closure_loss_grad(ctypes.byref(cfg.c()), f.shape[0], _p(f), _p(fbar),
                                     _p(np.ascontiguousarray(params, np.float64)),
                                     _p(np.ascontiguousarray(norm, np.float64)), 1 if tie_even else 0,
                                     ctypes.byref(loss), _p(grad))
    if rc:
        raise RuntimeError("closure loss needs a D3Q27 CM configuration")
    return loss.value, grad


def _momentum_mismatch(S1, target, pairs_nodes):
    """Momentum after the next streaming, sum_i e_i S1_i(x - e_i), minus the
    target's momentum sum_i e_i target_i(x); [N, 3]."""
    e = lattice("D3Q27")["e"].astype(np.float64)
    N = pairs_nodes
    j2 = gather_nodes("D3Q27", S1, np.arange(N)) @ e
    jbar = np.ascontiguousarray(target, np.float64).reshape(27, N).T @ e
    return j2 - jbar


def closure_momentum_objective(cfg: Cfg, S, target, params, norm, tie_even=False):
    """Closure objective on the momentum two coarse steps ahead (not in the
    paper): S [27, nz, ny, nx] post-collision populations, target [27, nz,
    ny, nx] populations two steps later.  One closure step (pull, collide
    with network rates) gives S1; the second step's collision conserves
    momentum, so the momentum after two steps is that of S1 pulled once
    more.  Objective (1/N) sum_x |j2(x) - jbar(x)|^2; its gradient is
    sum_y sum_i lam_i(y) d S1_i(y) / d params with the adjoint
    lam_i(y) = (2/N) e_i . (j2 - jbar)(y + e_i), evaluated as the gradient
    of the one-step objective for the target S1 - lam w N / 2, whose
    residual 2 (S1 - target) / (w N) is lam.  Returns (objective, gradient,
    adjoint field D = (2/N)(j2 - jbar) [3, nz, ny, nx])."""
    S = np.ascontiguousarray(S, np.float64)
    shape = S.shape[1:]
    N = int(np.prod(shape))
    fin = gather_nodes("D3Q27", S, np.arange(N))
    f1, _ = collide_closure(cfg, fin, params, norm, tie_even)
    S1 = np.ascontiguousarray(f1.T.reshape((27,) + shape))
    dj = _momentum_mismatch(S1, target, N)
    loss = float(np.mean(np.sum(dj * dj, axis=1)))
    D = (2.0 / N) * dj.T.reshape((3,) + shape)
    lam = momentum_adjoint(D)
    w = lattice("D3Q27")["w"]
    _, grad = closure_loss_grad(cfg, fin, f1 - lam * w[None, :] * (N / 2.0), params, norm, tie_even)
    return loss, grad, D


def momentum_adjoint(D):
    """lam_i(y) = sum_d e_{i,d} D_d(y + e_i) for a field D [3, nz, ny, nx];
    returns [N, 27]."""
    e = lattice("D3Q27")["e"]
    shape = D.shape[1:]
    lam = np.zeros((int(np.prod(shape)), 27))
    for i in range(27):
        ex, ey, ez = (int(v) for v in e[i])
        # value at y + e_i: roll by -e_i along (z, y, x)
        sh = np.roll(D, shift=(-ez, -ey, -ex), axis=(1, 2, 3))
        lam[:, i] = (ex * sh[0] + ey * sh[1] + ez * sh[2]).reshape(-1)
    return lam


MLP_NQ = 27 + 2 * 32   # rounded quantities per node: inputs x, activations h1, h2


def round_sig(v, bits=8):
    """Nearest values with `bits` significant bits, ties to even (8 = BF16)."""
    v = np.ascontiguousarray(np.atleast_1d(v), np.float64)
    out = np.zeros_like(v)
    lib().orc_round_sig(v.size, _p(v), int(bits), _p(out))
    return out


def closure_eval_rounded(cfg: Cfg, f, fbar, params, norm, tie_even=False, bits=8, rho0=1.0,
                         err=(0.0, 0.0, 0.0, 0.0)):
    """The closure network with its weights, inputs and hidden activations
    rounded to `bits` significant bits (the library's BF16 operands), in FP64
    otherwise.  fbar=None evaluates the collision only.  err = (ex, eh_rel,
    eh_sum, egelu') models the errors of another evaluation of the same
    network before each rounding (see orc_closure_eval_rounded); returns a
    dict with f* [n, 27], omega [n, 4], ``bound_fs`` [n, 27] and the rounding
    ``offsets`` [n, MLP_NQ], and with fbar the objective, its gradient,
    per-entry bounds ``bound_grad`` (2084 entries, then the objective) and
    ``abs_grad`` (sum over nodes of |node share|)."""
    f = np.ascontiguousarray(np.atleast_2d(f), np.float64)
    n = f.shape[0]
    fb = None if fbar is None else np.ascontiguousarray(np.atleast_2d(fbar), np.float64)
    r = dict(fs=np.zeros((n, 27)), omega=np.zeros((n, 4)), bound_fs=np.zeros((n, 27)),
             offsets=np.zeros((n, MLP_NQ)))
    loss = ctypes.c_double()
    grad, bg, ag = np.zeros(MLP_NPARAM), np.zeros(MLP_NPARAM + 1), np.zeros(MLP_NPARAM + 1)
    errv = np.ascontiguousarray(err, np.float64)
    rc = lib().orc_closure_eval_rounded(ctypes.byref(cfg.c()), n, _p(f), None if fb is None else _p(fb),
                                        _p(np.ascontiguousarray(params, np.float64)),
                                        _p(np.ascontiguousarray(norm, np.float64)), 1 if tie_even else 0,
                                        int(bits), float(rho0), _p(errv), _p(r["fs"]), _p(r["omega"]),
                                        ctypes.byref(loss), _p(grad), _p(r["bound_fs"]), _p(bg), _p(ag),
                                        _p(r["offsets"]))
    if rc:
        raise RuntimeError("rounded closure evaluation needs a D3Q27 CM configuration")
    if fb is not None:
        r.update(loss=loss.value, grad=grad, bound_grad=bg, abs_grad=ag)
    return r


def closure_loss_offsets(cfg: Cfg, f, fbar, params, norm, offsets, tie_even=False):
    """Objective of the network whose rounded operands are replaced by the
    exact values plus constant offsets [n, MLP_NQ] (weights as given)."""
    f = np.ascontiguousarray(np.atleast_2d(f), np.float64)
    fbar = np.ascontiguousarray(np.atleast_2d(fbar), np.float64)
    loss = ctypes.c_double()
    rc = lib().orc_closure_loss_offsets(ctypes.byref(cfg.c()), f.shape[0], _p(f), _p(fbar),
                                        _p(np.ascontiguousarray(params, np.float64)),
                                        _p(np.ascontiguousarray(norm, np.float64)), 1 if tie_even else 0,
                                        _p(np.ascontiguousarray(offsets, np.float64)), ctypes.byref(loss))
    if rc:
        raise RuntimeError("closure loss needs a D3Q27 CM configuration")
    return loss.value


def gather_nodes(kind: str, S: np.ndarray, nodes) -> np.ndarray:
    """Pulled populations S_i(x - e_i) at flat node indices; returns [n, Q]."""
    S = np.ascontiguousarray(S, np.float64)
    Q, nz, ny, nx = _dims(S)
    nodes = np.ascontiguousarray(nodes, np.int64)
    out = np.zeros((len(nodes), Q))
    lib().orc_gather_nodes(KINDS[kind], nx, ny, nz, _p(S), len(nodes),
                           nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out))
    return out
