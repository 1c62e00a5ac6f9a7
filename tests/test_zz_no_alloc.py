"""cmlb_reduce_noalloc (scratch in a fixed device array) against cmlb_reduce.

Both run the same kernels in the same launch shapes, so the diagnostics
must agree to the bar of the FP64 reductions (1e-13 relative; in practice
bitwise).  Two calls in a row, the second on a smaller grid, then the first
grid again: nothing may depend on what an earlier call left in the shared
array.  A grid beyond the stated maximum is refused before any launch.
"""
import numpy as np
import pytest

from paper_1808_04406_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("mass", "energy", "ke", "enstrophy", "rho_min", "rho_max", "u_max")


def perturbed(orc, kind, shape, seed, thermal=False):
    cfg = orc.Cfg(lattice=kind, thermal=thermal)
    rho, u, th = inputs.random_fields(shape, seed, drho=0.03, umax=0.05, dtheta=0.03 if thermal else 0.0)
    S = orc.init_equilibrium(cfg, rho, u, th if thermal else None)
    return S * inputs.perturbation(S.shape, seed + 1, 0.02)


def make(cm, orc, kind, shape, storage, seed, thermal=False):
    ctx = cm.Context(kind, shape, storage=storage, thermal=thermal, tau={2: 0.7})
    ctx.set_populations(perturbed(orc, kind, shape, seed, thermal))
    ctx.step(3)
    return ctx


def same(a, b):
    for k in KEYS:
        assert a[k] == pytest.approx(b[k], rel=1e-13, abs=1e-300), k
    assert np.allclose(a["momentum"], b["momentum"], rtol=1e-13, atol=1e-13 * abs(a["mass"]))
    assert a["nonfinite"] == b["nonfinite"]


def test_noalloc_equals_reduce_two_calls(cm, orc):
    print("noalloc: D3Q27 48x40x56 f32, then D2Q37 30x40 thermal f64, then the first again", flush=True)
    big = make(cm, orc, "D3Q27", (48, 40, 56), "f32", 300)
    small = make(cm, orc, "D2Q37", (30, 40), "f64", 302, thermal=True)
    try:
        first = big.reduce(noalloc=True)
        same(first, big.reduce())
        second = small.reduce(noalloc=True)
        same(second, small.reduce())
        same(big.reduce(noalloc=True), first)
        exact = all(first[k] == big.reduce()[k] for k in KEYS)
        print(f"bitwise equal to cmlb_reduce: {exact}", flush=True)
    finally:
        big.destroy()
        small.destroy()


def test_noalloc_allocates_nothing(cm, orc):
    """After the first call (which resolves the array's device address), a
    call on a context that never reduced leaves the device's free memory
    unchanged; cmlb_reduce on the same context allocates its scratch."""
    import torch
    print("noalloc: free-memory check on D3Q27 64^3 f32", flush=True)
    warm = make(cm, orc, "D3Q27", (8, 8, 8), "f32", 304)
    warm.reduce(noalloc=True)
    warm.destroy()
    ctx = make(cm, orc, "D3Q27", (64, 64, 64), "f32", 306)
    try:
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        g = ctx.reduce(noalloc=True)
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0
        same(g, ctx.reduce())
        free2, _ = torch.cuda.mem_get_info()
        assert free2 < free1   # the allocating entry point's scratch (6.3 MB) shows
    finally:
        ctx.destroy()


def test_noalloc_refuses_grids_beyond_the_array(cm, orc):
    print("noalloc: D2Q9 2048x2048 (4.2M nodes) must be refused", flush=True)
    n = 2048
    rho = np.ones((n, n))
    u = np.zeros((2, n, n))
    ctx = cm.Context("D2Q9", (n, n), storage="f32", tau={2: 0.7})
    try:
        ctx.init_fields(rho, u)
        with pytest.raises(cm.CmlbError) as ei:
            ctx.reduce(noalloc=True)
        assert ei.value.code == cm.EINVAL and "2621440" in str(ei.value)
        assert ctx.reduce()["mass"] == pytest.approx(n * n, rel=1e-12)   # the context is still usable
    finally:
        ctx.destroy()


def test_noalloc_reports_divergence(cm, orc):
    print("noalloc: non-finite population reported", flush=True)
    shape = (6, 8, 16)
    S = perturbed(orc, "D3Q27", shape, 308)
    S[5, 2, 3, 4] = np.nan
    ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.7})
    try:
        ctx.set_populations(S)
        a = ctx.reduce(allow_unstable=True, noalloc=True)
        b = ctx.reduce(allow_unstable=True)
        assert a["nonfinite"] == b["nonfinite"] == 1
        with pytest.raises(cm.CmlbError) as ei:
            ctx.reduce(noalloc=True)
        assert ei.value.code == cm.EUNSTABLE
    finally:
        ctx.destroy()
