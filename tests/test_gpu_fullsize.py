"""Parity at the full sizes of the paper-shaped workloads, on sampled outputs.

* D3Q27 512^3 Taylor-Green vortex at Re = 1e5 (u0 = 0.05), the precision
  form: BF16 and FP16 deviation storage (FP32 arithmetic), FP32 and FP64
  storage, two steps.  Population byte offsets reach 14 GB (29 GB in
  FP64), so 64-bit addressing of the population planes is exercised; the
  FP32 and FP64 pairs of steps run in one launch of the two-step kernel.  The oracle computes the two steps at each
  sampled node from the equilibrium of the initial fields on its 5^3
  neighbourhood, rounding the intermediate state through the storage codec
  as the stored state is rounded.
* D2Q37 1024^2 thermal shear and temperature waves (Pr = 7, background
  velocity 0.1 normal to k): two steps, every node.
* D3Q27 128^3 learned closure on a perturbed Taylor-Green state: one step
  at sampled nodes.

Tolerances as in the small parity tests (per storage, relative to the
largest deviation |f_i - w_i rho0|), doubled for two steps.
"""
import math

import numpy as np
import pytest

from paper_1808_04406_amd import inputs

from test_gpu_parity import TOL, f16_scales, quantise
from test_gpu_closure import ERR_MODEL, params

pytestmark = pytest.mark.gpu

TORCH_DTYPE = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16"}


@pytest.fixture(scope="module")
def tgv512():
    n, u0, re = 512, 0.05, 1.0e5
    rho, u = inputs.tgv3d(n, u0)
    nu = u0 * (n / (2 * math.pi)) / re
    t2 = 0.5 + 3.0 * nu
    return n, rho, u, {2: t2, 3: 1.0, 4: t2, 5: 1.0, 6: t2}


def cm_layout(ctx, storage):
    """(pitch, plane) of a D3Q27 context's state (cmlb_state_layout)."""
    from paper_1808_04406_amd import cmlb
    return cmlb.state_layout("D3Q27", ctx.shape, storage)


def sampled_state(ctx, storage, nodes, scale, w):
    """Stored populations of the given nodes, decoded (f = g / s + w rho0) on the host.
    The state's x-rows and planes are padded (header: layout of the state)."""
    import torch
    _, nbytes, _ = ctx.state()
    nz, ny, nx = ctx.shape
    pitch, plane = cm_layout(ctx, storage)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ctx.store_state_device(buf)
    ctx.sync()
    g = buf.view(getattr(torch, TORCH_DTYPE[storage])).view(27, -1)
    assert g.shape[1] == plane
    offs = (nodes // nx) * pitch + nodes % nx
    sel = g[:, torch.from_numpy(offs).cuda()].double().cpu().numpy()
    del buf, g
    torch.cuda.empty_cache()
    return (sel / scale[:, None] + w[:, None]).T


@pytest.mark.parametrize("storage", ["bf16", "f16", "f32", "f64"])
def test_precision_form_512_two_steps_sampled(cm, orc, tgv512, storage):
    import torch
    n, rho, u, tau = tgv512
    L = orc.lattice("D3Q27")
    e, w = L["e"][:, :3], L["w"]
    scale = f16_scales(w) if storage == "f16" else np.ones(27)
    ctx = cm.Context("D3Q27", (n, n, n), storage=storage, tau=tau,
                     scale=scale if storage == "f16" else None)
    try:
        d_rho = torch.from_numpy(rho.reshape(-1)).cuda()
        d_u = torch.from_numpy(u.reshape(-1)).cuda()
        ctx.init_fields_device(d_rho, d_u)
        del d_rho, d_u
        ctx.step(2)
        rng = np.random.default_rng(17)
        nodes = np.concatenate([rng.choice(n ** 3, 40, replace=False),
                                [0, n - 1, n * n - 1, n ** 3 - n * n, n ** 3 - 1]]).astype(np.int64)
        got = sampled_state(ctx, storage, nodes, scale, w)
        g = ctx.reduce()
    finally:
        ctx.destroy()
        torch.cuda.empty_cache()

    def stored(f):   # FP64 populations -> what the storage codec keeps
        return quantise((f - w) * scale, storage) / scale + w

    cfg = orc.Cfg(lattice="D3Q27", tau=tau)
    pos = np.stack([nodes % n, (nodes // n) % n, nodes // (n * n)], 1)
    nb = pos[:, None, :] - e[None, :, :]                                   # [node, j, 3]

    def f0(p):
        p = p % n
        return stored(np.stack([orc.equilibrium("D3Q27", rho[z, y, x], u[:, z, y, x], 1.0)
                                for x, y, z in p.reshape(-1, 3)]))

    pulled = np.stack([f0(nb - e[i][None, None, :])[:, i] for i in range(27)], 1)
    f1 = stored(orc.collide(cfg, pulled)).reshape(len(nodes), 27, 27)      # [node, j, i]
    ref = orc.collide(cfg, np.stack([f1[:, i, i] for i in range(27)], 1))
    if storage != "f32":
        ref = stored(ref)
    err = np.abs(got - ref).max()
    dev = np.abs(ref - w).max()
    print(f"512^3 {storage} two steps, sampled: max|df| = {err:.3e} (deviation scale {dev:.3e})")
    assert err <= 2 * TOL[storage] * dev
    mass0 = rho.sum()
    assert abs(g["mass"] - mass0) / mass0 < (1e-6 if storage == "f32" else 1e-3)
    assert g["nonfinite"] == 0


@pytest.mark.parametrize("fuse", [0, 3])   # automatic (the bitwise two-step kernel), row-accumulating kernel
def test_thermal_waves_1024_two_steps(cm, orc, fuse):
    n, kx, amp, pr, tau2 = 1024, 4, 0.01, 7.0, 0.6
    r = cm.lattice_info("D2Q37")["r"]
    tau = {2: tau2, 3: 0.5 + (tau2 - 0.5) / pr, 4: tau2}
    rho, u, th = inputs.waves2d(n, n, shear_amp=amp / r, thermal_amp=amp, k=(kx, 0), background=(0.0, 0.1))
    cfg = orc.Cfg(lattice="D2Q37", tau=tau, thermal=True)
    S = orc.init_equilibrium(cfg, rho, u, th)
    w = orc.lattice("D2Q37")["w"][:, None, None]
    ctx = cm.Context("D2Q37", (n, n), storage="f32", thermal=True, tau=tau)
    try:
        ctx.set_step_fusion(fuse)
        ctx.set_populations(S)
        ctx.step(2)
        got = ctx.get_populations()
    finally:
        ctx.destroy()
    ref = quantise(S - w, "f32") + w
    for k in range(2):
        orc.run(cfg, ref, 1)
        if k == 0:
            ref = quantise(ref - w, "f32") + w
    err = np.abs(got - ref).max()
    dev = np.abs(ref - w).max()
    print(f"D2Q37 1024^2 thermal waves, two steps (mode {fuse}): max|df| = {err:.3e} (deviation scale {dev:.3e})")
    assert err <= 2 * TOL["f32"] * dev


@pytest.mark.parametrize("nz", [151, 152])
def test_two_step_addressing_at_4gib(cm, nz):
    """D3Q27 512 x 512 x nz FP32: with nz = 151 the 27 planes take 4.275 GB,
    just below 2^32 bytes, and the two-step kernel pulls through one buffer
    resource whose offsets reach the top of the 32-bit range (out-of-range
    buffer reads return zero, so an offset error would show as wrong values,
    not as a fault); with nz = 152 (4.303 GB) it takes its global-load form.
    Either way two steps in one launch equal two single-step launches
    bitwise, compared on the device."""
    import torch
    shape = (nz, 512, 512)
    nbytes = cm.state_bytes("D3Q27", shape, "f32")
    assert (nbytes < 2 ** 32) == (nz == 151)
    rho, u, _ = inputs.random_fields(shape, 11, drho=0.02, umax=0.04)
    out = []
    for fuse in (1, 2):
        ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.52, 3: 1.0, 4: 0.52, 5: 1.0, 6: 0.52})
        try:
            ctx.set_step_fusion(fuse)
            ctx.init_fields(rho, u)
            ctx.step(2)
            buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            ctx.store_state_device(buf)
            ctx.sync()
            out.append(buf)
        finally:
            ctx.destroy()
    del rho, u
    same = torch.equal(out[0], out[1])
    top = out[1].view(torch.float32)[-512 * 512:]   # the last population's top plane
    nonzero = int((top != 0).sum().item())
    del out, top, buf
    torch.cuda.empty_cache()
    assert same
    assert nonzero > 0.99 * 512 * 512


def test_thermal_two_step_past_2gib(cm, orc):
    """D2Q37 4096^2 FP32 (a 2.48 GB state, so population offsets pass 2^31
    in the two-step kernels' 32-bit buffer addressing): two steps in one
    launch equal two single-step launches bitwise, compared on the device,
    and the row-accumulating kernel equals them to FP32 rounding; a few
    nodes are also checked against the oracle's step."""
    import torch
    n, amp = 4096, 0.01
    r = cm.lattice_info("D2Q37")["r"]
    tau = {2: 0.6, 3: 0.55, 4: 0.6}
    rho, u, th = inputs.waves2d(n, n, shear_amp=amp / r, thermal_amp=amp, k=(3, 1), background=(0.0, 0.1))
    nbytes = cm.state_bytes("D2Q37", (n, n), "f32")
    assert nbytes >= 2 ** 31
    out = []
    for fuse in (1, 2, 3):
        ctx = cm.Context("D2Q37", (n, n), storage="f32", thermal=True, tau=tau)
        try:
            ctx.set_step_fusion(fuse)
            ctx.init_fields(rho, u, th)
            ctx.step(2)
            buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            ctx.store_state_device(buf)
            ctx.sync()
            out.append(buf)
        finally:
            ctx.destroy()
    assert torch.equal(out[0], out[1])
    # the row-accumulating kernel (plane offsets past 2^31 in its scalar
    # offsets) within FP32 rounding of two single steps, every node
    s1 = out[0].view(torch.float32).view(37, -1)
    s3 = out[2].view(torch.float32).view(37, -1)
    d13 = (s3 - s1).abs().max().item()
    dev1 = s1.abs().max().item()   # the stored values are deviations from w rho0
    print(f"D2Q37 4096^2 row-accumulating kernel vs single steps: {d13:.3e} (deviation scale {dev1:.3e})")
    assert d13 <= 2 * TOL["f32"] * dev1
    del s1, s3
    # the last population planes (offsets past 2^31) against the oracle at sampled nodes
    g = out[1].view(torch.float32).view(37, -1)
    nodes = np.array([0, n - 1, n * n // 2 + 17, n * n - 1, 12345678], dtype=np.int64)
    got = g[:, torch.from_numpy(nodes).cuda()].double().cpu().numpy().T
    del out, g, buf
    torch.cuda.empty_cache()
    cfg = orc.Cfg(lattice="D2Q37", tau=tau, thermal=True)
    w = orc.lattice("D2Q37")["w"]
    e = orc.lattice("D2Q37")["e"][:, :2]
    # FP32-stored state after one step at the 7 x 7 neighbourhoods, then the second step
    pos = np.stack([nodes % n, nodes // n], 1)
    ref = []
    for x, y in pos:
        xs = (x + np.arange(-6, 7)) % n
        ys = (y + np.arange(-6, 7)) % n
        S0 = orc.init_equilibrium(cfg, rho[np.ix_(ys, xs)], u[:, ys][:, :, xs], th[np.ix_(ys, xs)])
        S0 = quantise(S0 - w[:, None, None], "f32") + w[:, None, None]
        S1 = S0.copy()
        orc.run(cfg, S1, 1)
        S1 = quantise(S1 - w[:, None, None], "f32") + w[:, None, None]
        orc.run(cfg, S1, 1)
        ref.append(S1[:, 6, 6])
    ref = np.array(ref)
    err = np.abs(got + w[None, :] - ref).max()
    dev = np.abs(ref - w[None, :]).max()
    print(f"D2Q37 4096^2 two steps, sampled: max|df| = {err:.3e} (deviation scale {dev:.3e})")
    assert err <= 2 * TOL["f32"] * dev


def test_thermal_two_step_falls_back_past_4gib(cm):
    """D2Q37 5800^2 FP32: the 37 planes take 4.98 GB, beyond the 32-bit
    buffer offsets of both two-step kernels, so steps-per-launch modes 2
    and 3 run single steps instead and give bitwise the populations of mode
    1 (compared on the device)."""
    import torch
    n = 5800
    nbytes = cm.state_bytes("D2Q37", (n, n), "f32")
    assert nbytes >= 2 ** 32
    r = cm.lattice_info("D2Q37")["r"]
    rho, u, th = inputs.waves2d(n, n, shear_amp=0.01 / r, thermal_amp=0.01, k=(2, 1), background=(0.0, 0.1))
    tau = {2: 0.6, 3: 0.55, 4: 0.6}
    out = []
    for fuse in (1, 2, 3):
        ctx = cm.Context("D2Q37", (n, n), storage="f32", thermal=True, tau=tau)
        try:
            ctx.set_step_fusion(fuse)
            ctx.init_fields(rho, u, th)
            ctx.step(3)
            assert ctx.step_count() == 3
            buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            ctx.store_state_device(buf)
            ctx.sync()
            out.append(buf)
        finally:
            ctx.destroy()
    assert torch.equal(out[0], out[1]) and torch.equal(out[0], out[2])
    g = out[0].view(torch.float32)
    assert torch.isfinite(g).all().item()
    del out, g, buf
    torch.cuda.empty_cache()


def test_closure_128_sampled(cm, orc):
    n, u0, re = 128, 0.05, 1.0e5
    rho, u = inputs.tgv3d(n, u0)
    t2 = 0.5 + 3.0 * u0 * (n / (2 * math.pi)) / re
    w = orc.lattice("D3Q27")["w"][:, None, None, None]
    S = orc.init_equilibrium(orc.Cfg(lattice="D3Q27"), rho, u) * inputs.perturbation((27, n, n, n), 90, 0.02)
    S = quantise(S - w, "f32") + w
    P = params(91)
    sigma = np.random.default_rng(92).uniform(0.005, 0.03, 27).astype(np.float32).astype(np.float64)
    ctx = cm.Context("D3Q27", (n, n, n), storage="f32", tau={2: t2})
    try:
        ctx.closure_load(P, sigma)
        ctx.closure_enable(True)
        ctx.set_populations(S)
        ctx.step(1)
        got = ctx.get_populations().reshape(27, -1)
    finally:
        ctx.destroy()
    rng = np.random.default_rng(93)
    nodes = np.concatenate([rng.choice(n ** 3, 3000, replace=False), [0, n - 1, n ** 3 - 1]])
    fin = orc.gather_nodes("D3Q27", S, nodes)
    cfg = orc.Cfg(lattice="D3Q27", tau={2: t2})
    # the network as the library defines it (BF16 operands), with the
    # per-element bound of the closure parity tests
    r = orc.closure_eval_rounded(cfg, fin, None, P, sigma, err=ERR_MODEL)
    ref = r["fs"]
    assert r["omega"].std() > 0.05
    bound = r["bound_fs"] + 2e-6 * np.abs(ref - w[:, 0, 0, 0]).max()
    err = np.abs(got[:, nodes].T - ref)
    print(f"closure 128^3 sampled: max|df| = {err.max():.3e}, max err/bound = {(err / bound).max():.3f}")
    assert (err <= bound).all()
