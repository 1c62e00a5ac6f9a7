"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Inputs are seeded and synthetic; both sides receive the same FP64 fields or
populations.  For 16-bit storage the test quantises the FP64 input itself
(numpy round-to-nearest-even through FP32, as the documented codec does), so
that the oracle sees exactly the stored state; the remaining difference is
FP32 arithmetic plus the rounding of the output.

Tolerances (absolute, on populations f_i, relative to the largest deviation
|f_i - w_i rho0| of the state, written per storage in TOL):
  f64: 1e-13 (a few FP64 rounding steps of O(1) quantities, x10 margin);
  f32: 2e-6  (about 30 FP32 roundings of the deviation scale);
  f16: 2^-10 (one output ulp of an 11-bit significand, x2) plus f32 term;
  bf16: 2^-7 (one output ulp of an 8-bit significand, x2) plus f32 term.
"""
import math

import numpy as np
import pytest

from paper_1808_04406_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 2e-6, "f16": 2.0 ** -10 + 2e-6, "bf16": 2.0 ** -7 + 2e-6}


def quantise(x, storage):
    """Round FP64 values the way the storage codec does: FP64 -> FP32 -> 16-bit RNE."""
    if storage == "f64":
        return x.copy()
    f = x.astype(np.float32)
    if storage == "f32":
        return f.astype(np.float64)
    if storage == "f16":
        return f.astype(np.float16).astype(np.float64)
    b = f.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) & 0xFFFF
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def f16_scales(w, rho0=1.0):
    """Power-of-two scales for FP16 storage: largest s with 16 w rho0 s <= 32752."""
    return np.exp2(np.floor(np.log2(32752.0 / (16.0 * w * rho0))))


def random_state(orc, kind, shape, seed, thermal=False, eps=0.03):
    cfg = orc.Cfg(lattice=kind, thermal=thermal)
    rho, u, th = inputs.random_fields(shape, seed, drho=0.05, umax=0.06, dtheta=0.05 if thermal else 0.0)
    S = orc.init_equilibrium(cfg, rho, u, th if thermal else None)
    return S * inputs.perturbation(S.shape, seed + 1, eps)


def taus(kind, seed):
    rng = np.random.default_rng(seed)
    hi = 5 if kind == "D2Q37" else 7
    return {n: float(rng.uniform(0.52, 1.6)) for n in range(2, hi)}


def one_step_case(cm, orc, kind, storage, shape, seed, thermal=False, model="cm"):
    L = orc.lattice(kind)
    w = L["w"]
    S = random_state(orc, kind, shape, seed, thermal)
    tau = taus(kind, seed + 7)
    scale = f16_scales(w) if storage == "f16" else np.ones(L["Q"])
    bshape = (L["Q"],) + (1,) * len(shape)
    dev = (S - w.reshape(bshape)) * scale.reshape(bshape)
    Sq = quantise(dev, storage) / scale.reshape(bshape) + w.reshape(bshape)
    ctx = cm.Context(kind, shape, storage=storage, model=model, thermal=thermal, tau=tau,
                     scale=scale if storage == "f16" else None)
    try:
        ctx.set_populations(S)
        ctx.step(1)
        got = ctx.get_populations()
    finally:
        ctx.destroy()
    ref = Sq.copy()
    orc.run(orc.Cfg(lattice=kind, tau=tau, thermal=thermal, model=model), ref, 1)
    dev_scale = np.abs(ref - w.reshape(bshape)).max()
    err = np.abs(got - ref).max()
    return err, dev_scale


CASES = [
    ("D3Q27", (5, 7, 37)),      # ragged x inside one 64-lane block
    ("D3Q27", (3, 4, 300)),     # two x chunks of 256 with a tail
    ("D3Q27", (2, 3, 1)),       # nx = 1: x neighbours are the node itself
    ("D2Q9", (19, 70)),
    ("D2Q37", (13, 41)),
    ("D2Q37", (5, 260)),
]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("kind,shape", CASES)
def test_one_step_parity(cm, orc, kind, shape, storage):
    err, scale = one_step_case(cm, orc, kind, storage, shape, seed=100 + len(shape) * 7 + shape[-1])
    print(f"{kind} {shape} {storage}: max|df| = {err:.3e} (deviation scale {scale:.3e})")
    assert err <= TOL[storage] * scale


@pytest.mark.parametrize("model", ["cm", "raw_mrt", "reg_bgk"])
@pytest.mark.parametrize("thermal", [True, False])
def test_one_step_parity_d2q37_models(cm, orc, model, thermal):
    for storage in ("f64", "f32"):
        err, scale = one_step_case(cm, orc, "D2Q37", storage, (11, 67), seed=300, thermal=thermal, model=model)
        print(f"D2Q37 {model} thermal={thermal} {storage}: {err:.3e} / {scale:.3e}")
        assert err <= TOL[storage] * scale


# The other minimal 2D rules of Fig. 2 (FP64 and FP32 storage, central moments)
RULES = ["E9B", "E9C", "E9D", "E7A", "E7B", "E7C", "E7D"]


@pytest.mark.parametrize("thermal", [True, False])
@pytest.mark.parametrize("kind", RULES)
def test_one_step_parity_rules(cm, orc, kind, thermal):
    for storage in ("f64", "f32"):
        for shape in ((13, 41), (4, 130), (3, 700)):   # ragged rows; padded rows of 130; two x-chunks of a row
            err, scale = one_step_case(cm, orc, kind, storage, shape, seed=400 + len(kind) + shape[1],
                                       thermal=thermal)
            print(f"{kind} {shape} {storage} thermal={thermal}: {err:.3e} / {scale:.3e}")
            assert err <= TOL[storage] * scale


@pytest.mark.parametrize("kind", ["E9C", "E7A", "E7D"])
def test_rules_thermal_waves_multistep(cm, orc, kind):
    """Shear + thermal waves with a background flow, 40 steps, on 2D rules of
    both degrees: moments against the oracle (FP64 1e-12, FP32 2e-6), and
    mass, momentum and energy of the FP64 run conserved."""
    shape, steps = (24, 30), 40
    tau = {2: 0.6, 3: 0.64, 4: 1.0}
    rho, u, th = inputs.waves2d(30, 24, shear_amp=0.01, thermal_amp=0.01, background=(0.0, 0.1))
    cfg = orc.Cfg(lattice=kind, tau=tau, thermal=True)
    S = orc.init_equilibrium(cfg, rho, u, th)
    orc.run(cfg, S, steps)
    o_rho, o_u, o_th = orc.moments(kind, S)
    for storage, tol in (("f64", 1e-12), ("f32", 2e-6)):
        ctx = cm.Context(kind, shape, storage=storage, thermal=True, tau=tau)
        ctx.init_fields(rho, u, th)
        g0 = ctx.reduce()
        ctx.step(steps)
        g1 = ctx.reduce()
        g_rho, g_u, g_th = ctx.get_moments()
        ctx.destroy()
        err = max(np.abs(g_u - o_u).max(), np.abs(g_th - o_th).max(), np.abs(g_rho - o_rho).max())
        print(f"{kind} waves {storage}: max err {err:.3e}")
        assert err <= tol
        if storage == "f64":
            assert g1["mass"] == pytest.approx(g0["mass"], rel=1e-13)
            assert np.abs(g1["momentum"] - g0["momentum"]).max() <= 1e-12 * g0["mass"]
            assert g1["energy"] == pytest.approx(g0["energy"], rel=1e-12)


def test_tgv_fp64_multistep(cm, orc):
    """D3Q27 TGV 24^3, tau = 0.6, 60 steps in FP64: max|du| <= 1e-12."""
    n, steps = 24, 60
    tau = {2: 0.6}
    rho, u = inputs.tgv3d(n, 0.05)
    ctx = cm.Context("D3Q27", (n, n, n), storage="f64", tau=tau)
    ctx.init_fields(rho, u)
    ctx.step(steps)
    g_rho, g_u, _ = ctx.get_moments()
    ctx.destroy()
    cfg = orc.Cfg(lattice="D3Q27", tau=tau)
    S = orc.init_equilibrium(cfg, rho, u)
    orc.run(cfg, S, steps)
    o_rho, o_u, _ = orc.moments("D3Q27", S)
    du = np.abs(g_u - o_u).max()
    print(f"FP64 TGV 24^3 x {steps}: max|du| = {du:.3e}, max|drho| = {np.abs(g_rho - o_rho).max():.3e}")
    assert du <= 1e-12
    assert np.abs(g_rho - o_rho).max() <= 1e-12


@pytest.mark.parametrize("storage,tol_u", [("f32", 2e-6), ("f16", 2e-4), ("bf16", 3e-3)])
def test_tgv_reduced_precision_multistep(cm, orc, storage, tol_u):
    """D3Q27 TGV 32^3, tau = 0.55, 200 steps: error of u against the FP64
    oracle stays within the stated bound for each storage type."""
    n, steps = 32, 200
    tau = {2: 0.55}
    rho, u = inputs.tgv3d(n, 0.05)
    ctx = cm.Context("D3Q27", (n, n, n), storage=storage, tau=tau)
    ctx.init_fields(rho, u)
    ctx.step(steps)
    _, g_u, _ = ctx.get_moments()
    ctx.destroy()
    cfg = orc.Cfg(lattice="D3Q27", tau=tau)
    S = orc.init_equilibrium(cfg, rho, u)
    orc.run(cfg, S, steps)
    _, o_u, _ = orc.moments("D3Q27", S)
    du = np.abs(g_u - o_u).max()
    print(f"{storage} TGV 32^3 x {steps}: max|du| = {du:.3e} (u0 = 0.05)")
    assert du <= tol_u


def test_d2q37_thermal_waves_multistep(cm, orc):
    """D2Q37 thermal, shear + thermal waves with a background flow, FP64 and FP32."""
    shape, steps = (24, 30), 40
    L = orc.lattice("D2Q37")
    tau = {2: 0.6, 3: 0.64, 4: 1.0}
    rho, u, th = inputs.waves2d(30, 24, shear_amp=0.01, thermal_amp=0.01, background=(0.0, 0.1))
    cfg = orc.Cfg(lattice="D2Q37", tau=tau, thermal=True)
    S = orc.init_equilibrium(cfg, rho, u, th)
    orc.run(cfg, S, steps)
    o_rho, o_u, o_th = orc.moments("D2Q37", S)
    for storage, tol in (("f64", 1e-12), ("f32", 2e-6)):
        ctx = cm.Context("D2Q37", shape, storage=storage, thermal=True, tau=tau)
        ctx.init_fields(rho, u, th)
        ctx.step(steps)
        g_rho, g_u, g_th = ctx.get_moments()
        ctx.destroy()
        err = max(np.abs(g_u - o_u).max(), np.abs(g_th - o_th).max(), np.abs(g_rho - o_rho).max())
        print(f"D2Q37 waves {storage}: max err {err:.3e}")
        assert err <= tol


def test_full_size_sampled_d3q27_256(cm, orc):
    """The benchmark workload (D3Q27 256^3 FP32 TGV, Re = 1600): one step in the
    benchmark's launch configuration, checked at sampled nodes against the
    oracle's pull + collide of the same initial fields."""
    n, u0 = 256, 0.05
    nu = u0 * (n / (2 * math.pi)) / 1600.0
    tau = {2: 0.5 + 3.0 * nu}
    rho, u = inputs.tgv3d(n, u0)
    ctx = cm.Context("D3Q27", (n, n, n), storage="f32", tau=tau)
    ctx.init_fields(rho, u)
    ctx.step(1)
    got = ctx.get_populations()
    g = ctx.reduce()
    ctx.destroy()
    rng = np.random.default_rng(5)
    nodes = np.concatenate([rng.choice(n ** 3, 300, replace=False),
                            [0, n - 1, n * n - 1, n ** 3 - 1, n ** 3 - n]])  # faces and corners
    L = orc.lattice("D3Q27")
    cfg = orc.Cfg(lattice="D3Q27", tau=tau)
    fin = np.zeros((len(nodes), 27))
    for k, idx in enumerate(nodes):
        x, y, z = idx % n, (idx // n) % n, idx // (n * n)
        for i, e in enumerate(L["e"]):
            xs, ys, zs = (x - e[0]) % n, (y - e[1]) % n, (z - e[2]) % n
            fin[k, i] = orc.equilibrium("D3Q27", rho[zs, ys, xs], u[:, zs, ys, xs], 1.0)[i]
    # the GPU state was encoded to FP32 at initialisation
    fin = quantise(fin - L["w"], "f32") + L["w"]
    ref = orc.collide(cfg, fin)
    gs = got.reshape(27, -1)[:, nodes].T
    err = np.abs(gs - ref).max()
    scale = np.abs(ref - L["w"]).max()
    print(f"256^3 sampled: max|df| = {err:.3e} (deviation scale {scale:.3e})")
    assert err <= TOL["f32"] * scale
    mass0 = rho.sum()
    assert abs(g["mass"] - mass0) / mass0 < 1e-7


def test_full_size_sampled_two_step_launch(cm, orc):
    """The benchmark's own configuration: D3Q27 256^3 FP32 TGV (Re = 1600)
    with its rate set, two steps in one launch of the two-step kernel,
    checked at sampled nodes against two oracle steps computed from the
    5^3 neighbourhood of each node (the intermediate state rounded to FP32,
    as the stored state would be)."""
    n, u0 = 256, 0.05
    nu = u0 * (n / (2 * math.pi)) / 1600.0
    t2 = 0.5 + 3.0 * nu
    tau = {2: t2, 3: 1.0, 4: t2, 5: 1.0, 6: t2}
    rho, u = inputs.tgv3d(n, u0)
    ctx = cm.Context("D3Q27", (n, n, n), storage="f32", tau=tau)
    ctx.init_fields(rho, u)
    ctx.step(2)
    got = ctx.get_populations().reshape(27, -1)
    ctx.destroy()
    L = orc.lattice("D3Q27")
    e, w = L["e"][:, :3], L["w"]
    cfg = orc.Cfg(lattice="D3Q27", tau=tau)
    rng = np.random.default_rng(11)
    nodes = np.concatenate([rng.choice(n ** 3, 60, replace=False), [0, n ** 3 - 1, n - 1, n * n - n]])
    pos = np.stack([nodes % n, (nodes // n) % n, nodes // (n * n)], 1)            # x, y, z

    def f0(p):   # stored initial state at positions p[..., 3] (FP32 deviation storage)
        p = p % n
        feq = np.stack([orc.equilibrium("D3Q27", rho[z, y, x], u[:, z, y, x], 1.0)
                        for x, y, z in p.reshape(-1, 3)])
        return quantise(feq - w, "f32") + w

    # first step at the 27 neighbours x - e_j of every sampled node
    nb = pos[:, None, :] - e[None, :, :]                                            # [node, j, 3]
    pulled = np.stack([f0(nb - e[i][None, None, :])[:, i] for i in range(27)], 1)  # [node*j, i]
    f1 = orc.collide(cfg, pulled)
    f1 = quantise(f1 - w, "f32") + w
    f1 = f1.reshape(len(nodes), 27, 27)                                             # [node, j, i]
    # second step at the node pulls population i from neighbour j = i
    fin = np.stack([f1[:, i, i] for i in range(27)], 1)
    ref = orc.collide(cfg, fin)
    gs = got[:, nodes].T
    err = np.abs(gs - ref).max()
    scale = np.abs(ref - w).max()
    print(f"256^3 two-step launch, sampled: max|df| = {err:.3e} (deviation scale {scale:.3e})")
    assert err <= 2 * TOL["f32"] * scale


def test_determinism(cm):
    n = 32
    rho, u = inputs.tgv3d(n, 0.05)
    outs = []
    for _ in range(2):
        ctx = cm.Context("D3Q27", (n, n, n), storage="f32", tau={2: 0.52})
        ctx.init_fields(rho, u)
        ctx.step(25)
        outs.append(ctx.get_populations())
        outs.append(ctx.reduce())
        ctx.destroy()
    assert np.array_equal(outs[0], outs[2])
    assert outs[1]["enstrophy"] == outs[3]["enstrophy"] and outs[1]["ke"] == outs[3]["ke"]


@pytest.mark.parametrize("kind,shape,thermal", [("D3Q27", (9, 10, 11), False), ("D2Q37", (12, 13), True),
                                                ("D2Q9", (20, 17), False),
                                                ("D3Q27", (3, 4, 300), False)])   # padded rows
def test_moments_and_reductions(cm, orc, kind, shape, thermal):
    from oracle.analysis import globals_of_state
    S = random_state(orc, kind, shape, 44, thermal)
    ctx = cm.Context(kind, shape, storage="f64", thermal=thermal)
    ctx.set_populations(S)
    g_rho, g_u, g_th = ctx.get_moments()
    g = ctx.reduce()
    ctx.destroy()
    o_rho, o_u, o_th = orc.moments(kind, S)
    assert np.abs(g_rho - o_rho).max() < 1e-14
    assert np.abs(g_u - o_u).max() < 1e-14
    assert np.abs(g_th - o_th).max() < 1e-13
    ref = globals_of_state(kind, S)
    for key in ("mass", "energy", "ke", "enstrophy"):
        assert g[key] == pytest.approx(ref[key], rel=1e-12, abs=1e-15), key
    assert np.allclose(g["momentum"][:len(ref["momentum"])], ref["momentum"], rtol=1e-12, atol=1e-13)
    assert g["nonfinite"] == 0
    # range diagnostics: same node arithmetic as the moment readout
    assert g["rho_min"] == g_rho.min() and g["rho_max"] == g_rho.max()
    assert abs(g["rho_min"] - o_rho.min()) < 1e-14 and abs(g["rho_max"] - o_rho.max()) < 1e-14
    assert g["u_max"] == pytest.approx(np.sqrt((o_u ** 2).sum(0)).max(), rel=1e-13)


def test_nonfinite_detected(cm, orc):
    S = random_state(orc, "D3Q27", (4, 5, 6), 45)
    S[3, 1, 2, 3] = np.nan
    ctx = cm.Context("D3Q27", (4, 5, 6), storage="f32")
    ctx.set_populations(S)
    with pytest.raises(cm.CmlbError) as ei:
        ctx.reduce()
    assert ei.value.code == cm.EUNSTABLE
    g = ctx.reduce(allow_unstable=True)
    assert g["nonfinite"] == 1
    assert np.isfinite(g["rho_min"]) and np.isfinite(g["u_max"])   # ranges over the finite nodes
    ctx.destroy()


def test_error_paths(cm):
    ctx = cm.Context("D3Q27", (4, 4, 4))
    with pytest.raises(cm.CmlbError) as ei:
        ctx.step(1)
    assert ei.value.code == cm.ESTATE
    with pytest.raises(cm.CmlbError) as ei:
        ctx.get_moments()
    assert ei.value.code == cm.ESTATE
    with pytest.raises(cm.CmlbError) as ei:
        ctx.set_tau([-1.0])
    assert ei.value.code == cm.EINVAL
    with pytest.raises(cm.CmlbError):
        ctx.init_fields(np.zeros((4, 4, 4)), np.zeros((3, 4, 4, 4)))   # rho must be positive
    ctx.init_fields(np.ones((4, 4, 4)), np.zeros((3, 4, 4, 4)))
    ctx.step(0)
    assert ctx.step_count() == 0
    ctx.destroy()


@pytest.mark.parametrize("shape", [(16, 16, 16), (4, 6, 250)])   # the second has padded rows
def test_external_buffers_match_internal(cm, shape):
    import torch
    rho, u = inputs.random_fields(shape, 3, drho=0.02, umax=0.04)[:2]
    nbytes = cm.state_bytes("D3Q27", shape, "f32")
    assert nbytes >= 27 * int(np.prod(shape)) * 4
    bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    a = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.7}, external=bufs, stream=stream)
    b = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.7})
    for c in (a, b):
        c.init_fields(rho, u)
        c.step(7)
    assert np.array_equal(a.get_populations(), b.get_populations())
    ptr, size, s = a.state()
    assert ptr in (bufs[0].data_ptr(), bufs[1].data_ptr()) and size == nbytes
    assert s == stream.cuda_stream
    with pytest.raises(ValueError):
        cm.Context("D3Q27", shape, stream=torch.cuda.default_stream())
    a.destroy()
    b.destroy()


def test_device_tensor_checks(cm):
    """Device tensors handed to the binding are checked for placement, dtype
    and size before any kernel sees their address."""
    import torch
    shape = (4, 4, 8)
    n = 4 * 4 * 8
    f64 = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")
    ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.7})
    try:
        with pytest.raises(ValueError, match="elements"):
            ctx.init_fields_device(f64(n), f64(3 * n - 1))
        with pytest.raises(ValueError, match="float64"):
            ctx.init_fields_device(f64(n).float(), f64(3 * n))
        with pytest.raises(ValueError, match="CUDA"):
            ctx.init_fields_device(torch.zeros(n, dtype=torch.float64), f64(3 * n))
        with pytest.raises(ValueError, match="contiguous"):
            ctx.init_fields_device(f64(2 * n)[::2], f64(3 * n))
        ctx.init_fields_device(torch.ones(n, dtype=torch.float64, device="cuda"), f64(3 * n))
        nbytes = ctx.state()[1]
        with pytest.raises(ValueError, match="bytes"):
            ctx.store_state_device(torch.empty(nbytes - 1, dtype=torch.uint8, device="cuda"))
        with pytest.raises(ValueError, match="bytes"):
            ctx.load_state_device(torch.empty(nbytes // 4 - 1, dtype=torch.float32, device="cuda"))
        with pytest.raises(ValueError, match="elements"):
            ctx.box_filter(2, torch.empty(27 * n // 8 + 1, dtype=torch.float32, device="cuda"))
        with pytest.raises(ValueError, match="divide"):
            ctx.box_filter(3, torch.empty(27, dtype=torch.float32, device="cuda"))
        st = torch.zeros(27 * n, dtype=torch.float32, device="cuda")
        ctx.closure_load(np.zeros(cm.CLOSURE_NPARAM), np.full(27, 0.01))
        with pytest.raises(ValueError, match="elements"):
            ctx.closure_objective(st, st, n_pairs=2)
        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        ctx.store_state_device(buf)       # the right sizes pass
        ctx.load_state_device(buf)
        ctx.sync()
    finally:
        ctx.destroy()
    with pytest.raises(ValueError, match="bytes"):
        short = [torch.empty(cm.state_bytes("D3Q27", shape, "f32") - 4, dtype=torch.uint8, device="cuda")
                 for _ in range(2)]
        cm.Context("D3Q27", shape, storage="f32", external=short)


def test_device_fields_on_torch_stream(cm, orc):
    """Fields handed over as device tensors on the caller's stream."""
    import torch
    n = 12
    rho, u = inputs.tgv3d(n, 0.05)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        d_rho = torch.from_numpy(rho.reshape(-1)).to("cuda")
        d_u = torch.from_numpy(u.reshape(-1)).to("cuda")
        ctx = cm.Context("D3Q27", (n, n, n), storage="f64", tau={2: 0.8}, stream=stream)
        ctx.init_fields_device(d_rho, d_u)
        ctx.step(3)
        _, g_u, _ = ctx.get_moments()
        ctx.destroy()
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.8})
    S = orc.init_equilibrium(cfg, rho, u)
    orc.run(cfg, S, 3)
    _, o_u, _ = orc.moments("D3Q27", S)
    assert np.abs(g_u - o_u).max() < 1e-13


@pytest.mark.parametrize("shape,storage", [((64, 64, 64), "f32"), ((4, 6, 250), "bf16"), ((3, 5, 300), "f64"),
                                           ((128, 128, 128), "f16")])
def test_load_deviations_device(cm, orc, shape, storage):
    """cmlb_load_deviations_device: unpadded FP32 deviations land in the
    state's own storage and layout (128^3 FP16 has padded planes, the 250-
    and 300-wide grids padded rows), read back through cmlb_get_populations:
    exact for FP32 and FP64 storage, one rounding of dev * s for the 16-bit
    forms."""
    import torch
    w = orc.lattice("D3Q27")["w"][:, None, None, None]
    dev = (0.01 * np.random.default_rng(5).standard_normal((27,) + shape)).astype(np.float32)
    scale = f16_scales(w[:, 0, 0, 0]) if storage == "f16" else np.ones(27)
    ctx = cm.Context("D3Q27", shape, storage=storage, scale=scale if storage == "f16" else None)
    try:
        ctx.load_deviations_device(torch.from_numpy(dev).cuda())
        assert ctx.step_count() == 0
        f = ctx.get_populations()
    finally:
        ctx.destroy()
    s = scale[:, None, None, None]
    ref = quantise(dev.astype(np.float64) * s, storage) / s + w
    assert np.array_equal(f, ref)


@pytest.mark.parametrize("kind,shape,storage,thermal", [("D3Q27", (2, 3, 300), "f32", False),
                                                        ("D2Q37", (4, 260), "f64", True)])
def test_init_fields_on_padded_rows(cm, orc, kind, shape, storage, thermal):
    """Equilibrium initialisation, moments and one step on a state whose
    x-rows are padded to the pitch (header: layout of the state)."""
    rho, u, th = inputs.random_fields(shape, 47, drho=0.03, umax=0.05, dtheta=0.03 if thermal else 0.0)
    elem = {"f64": 8, "f32": 4}[storage]
    assert cm.state_bytes(kind, shape, storage) > orc.lattice(kind)["Q"] * int(np.prod(shape)) * elem
    ctx = cm.Context(kind, shape, storage=storage, thermal=thermal, tau={2: 0.7, 3: 0.9, 4: 0.8})
    try:
        ctx.init_fields(rho, u, th if thermal else None)
        S0 = ctx.get_populations()
        g_rho, g_u, g_th = ctx.get_moments()
        ctx.step(1)
        S1 = ctx.get_populations()
    finally:
        ctx.destroy()
    cfg = orc.Cfg(lattice=kind, tau={2: 0.7, 3: 0.9, 4: 0.8}, thermal=thermal)
    ref = orc.init_equilibrium(cfg, rho, u, th if thermal else None)
    w = orc.lattice(kind)["w"].reshape((-1,) + (1,) * len(shape))
    dev = np.abs(ref - w).max()
    assert np.abs(S0 - ref).max() <= TOL[storage] * dev
    o_rho, o_u, o_th = orc.moments(kind, S0)
    assert np.abs(g_rho - o_rho).max() < 1e-13 and np.abs(g_u - o_u).max() < 1e-13
    if thermal:
        assert np.abs(g_th - o_th).max() < 1e-12
    orc.run(cfg, S0, 1)
    assert np.abs(S1 - S0).max() <= TOL[storage] * dev


def test_set_tau_changes_rates(cm, orc):
    S = random_state(orc, "D3Q27", (4, 5, 6), 46)
    ctx = cm.Context("D3Q27", (4, 5, 6), storage="f64", tau={2: 0.9})
    ctx.set_tau([0.7, 0.8, 0.9, 1.1, 1.3])
    ctx.set_populations(S)
    ctx.step(1)
    got = ctx.get_populations()
    ctx.destroy()
    ref = S.copy()
    orc.run(orc.Cfg(lattice="D3Q27", tau={2: 0.7, 3: 0.8, 4: 0.9, 5: 1.1, 6: 1.3}), ref, 1)
    assert np.abs(got - ref).max() < 1e-14


def test_tgv_long_run_stable_rates(cm):
    """64^3 Taylor-Green vortex at tau_2 = 0.50095 (Re = 1600 at this size) with
    the benchmark's rate set (odd orders at 1, even orders at omega_2) stays
    finite for 600 steps and loses kinetic energy monotonically."""
    n = 64
    tau = 0.5 + 3.0 * 0.05 * (n / (2 * math.pi)) / 1600.0
    rho, u = inputs.tgv3d(n, 0.05)
    ctx = cm.Context("D3Q27", (n, n, n), storage="f32", tau={2: tau, 3: 1.0, 4: tau, 5: 1.0, 6: tau})
    ctx.init_fields(rho, u)
    ke = [ctx.reduce()["ke"]]
    for _ in range(6):
        ctx.step(100)
        g = ctx.reduce()
        assert g["nonfinite"] == 0
        ke.append(g["ke"])
    ctx.destroy()
    assert all(b < a for a, b in zip(ke, ke[1:]))


FUSION_SHAPES = [
    (5, 7, 37),      # one tile, ragged in x and y
    (3, 4, 300),     # five x tiles with a tail
    (2, 3, 1),       # nx = 1
    (1, 1, 1),       # every neighbour is the node itself
    (12, 17, 70),    # several tiles in x and y, nz not a multiple of the z chunk
    (40, 24, 128),   # 240 one-plane z chunks
]


def test_two_step_launch_ragged_z_chunks(cm, orc):
    """256 workgroups of 128 x-y tiles in two z chunks of 16 and 15 planes."""
    test_two_step_launch_equals_single_steps(cm, orc, (31, 128, 512), "f32")


@pytest.mark.parametrize("storage", ["f32", "f64", "bf16", "f16"])
@pytest.mark.parametrize("shape", FUSION_SHAPES)
def test_two_step_launch_equals_single_steps(cm, orc, shape, storage):
    """Pairs of D3Q27 FP32 or FP64 steps in one launch (intermediate state on
    chip) give bitwise the same populations as one launch per step; odd
    counts end with a single step.  16-bit storage keeps one step per launch
    either way."""
    L = orc.lattice("D3Q27")
    S = random_state(orc, "D3Q27", shape, seed=sum(shape) + 3)
    tau = taus("D3Q27", seed=len(shape) + shape[-1])
    scale = f16_scales(L["w"]) if storage == "f16" else None
    out = {}
    for fuse in (1, 2, 0):
        ctx = cm.Context("D3Q27", shape, storage=storage, tau=tau, scale=scale)
        try:
            ctx.set_step_fusion(fuse)
            ctx.set_populations(S)
            ctx.step(2)
            a = ctx.get_populations()
            ctx.step(5)
            out[fuse] = (a, ctx.get_populations(), ctx.step_count())
        finally:
            ctx.destroy()
    assert out[1][2] == out[2][2] == out[0][2] == 7
    for k in (0, 2):
        assert np.array_equal(out[1][0], out[k][0])
        assert np.array_equal(out[1][1], out[k][1])


D37_FUSION_CASES = [
    ((13, 41), "cm", True),          # one segment, ragged; rows fewer than a chunk's lead-in
    ((5, 260), "cm", True),          # three segments, padded rows
    ((3, 3), "cm", True),            # smallest grid: every shift wraps more than once
    ((130, 250), "raw_mrt", True),   # several segments, one-row chunks
    ((301, 250), "cm", True),        # two-row chunks, the last one ragged
    ((61, 122), "reg_bgk", False),   # one full segment, isothermal
    ((24, 7), "cm", False),
    ((2000, 130), "cm", True),       # tall: two segments, many short row chunks
    ((130, 2000), "raw_mrt", True),  # wide: 17 segments
]


@pytest.mark.parametrize("shape,model,thermal", D37_FUSION_CASES)
def test_two_step_launch_equals_single_steps_d37(cm, orc, shape, model, thermal):
    """Pairs of D2Q37 FP32 steps in one launch (first-step rows kept in LDS)
    give bitwise the same populations as one launch per step, for each
    collision model; odd counts end with a single step."""
    S = random_state(orc, "D2Q37", shape, seed=sum(shape) + 5, thermal=thermal)
    tau = taus("D2Q37", seed=shape[-1] + 1)
    out = {}
    for fuse in (1, 2, 0):
        ctx = cm.Context("D2Q37", shape, storage="f32", model=model, thermal=thermal, tau=tau)
        try:
            ctx.set_step_fusion(fuse)
            ctx.set_populations(S)
            ctx.step(2)
            a = ctx.get_populations()
            ctx.step(5)
            out[fuse] = (a, ctx.get_populations(), ctx.step_count())
        finally:
            ctx.destroy()
    assert out[1][2] == out[2][2] == out[0][2] == 7
    for k in (0, 2):
        assert np.array_equal(out[1][0], out[k][0])
        assert np.array_equal(out[1][1], out[k][1])


@pytest.mark.parametrize("shape,model,thermal", D37_FUSION_CASES)
def test_two_step_accumulating_kernel_d37(cm, orc, shape, model, thermal):
    """The D2Q37 two-step kernel that folds each first-step row into the
    moments of the rows it feeds (steps-per-launch mode 3): two steps against
    the oracle's two steps from the same FP32 state (the intermediate state
    rounded to FP32 as the kernel keeps it), element by element within the
    FP32 bound of two steps; then 7 steps (three launches and a single step)
    against 7 single-step launches.  The moment sums run in another order
    than the single-step kernel's, so each step may differ by FP32 rounding:
    the bound is 7 times the one-step FP32 bound."""
    S = random_state(orc, "D2Q37", shape, seed=sum(shape) + 5, thermal=thermal)
    w = orc.lattice("D2Q37")["w"][:, None, None]
    S = quantise(S - w, "f32") + w
    tau = taus("D2Q37", seed=shape[-1] + 1)
    out = {}
    for fuse in (1, 3):
        ctx = cm.Context("D2Q37", shape, storage="f32", model=model, thermal=thermal, tau=tau)
        try:
            ctx.set_step_fusion(fuse)
            ctx.set_populations(S)
            ctx.step(2)
            a = ctx.get_populations()
            ctx.step(5)
            out[fuse] = (a, ctx.get_populations(), ctx.step_count())
        finally:
            ctx.destroy()
    assert out[1][2] == out[3][2] == 7
    cfg = orc.Cfg(lattice="D2Q37", tau=tau, thermal=thermal, model=model)
    ref = S.copy()
    orc.run(cfg, ref, 1)
    ref = quantise(ref - w, "f32") + w
    orc.run(cfg, ref, 1)
    dev = np.abs(ref - w).max()
    err2 = np.abs(out[3][0] - ref).max()
    err7 = np.abs(out[3][1] - out[1][1]).max()
    dev7 = np.abs(out[1][1] - w).max()
    print(f"D2Q37 {shape} {model} thermal={thermal}: two steps vs oracle {err2:.3e} / {dev:.3e}, "
          f"7 steps vs single steps {err7:.3e} / {dev7:.3e}")
    assert err2 <= 2 * TOL["f32"] * dev
    assert err7 <= 7 * TOL["f32"] * dev7


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_two_step_launch_options(cm, storage):
    ctx = cm.Context("D3Q27", (4, 4, 4), storage=storage, tau={2: 0.6})
    try:
        for bad in (4, -1):
            with pytest.raises(cm.CmlbError):
                ctx.set_step_fusion(bad)
        for v in (0, 2, 3):      # 16-bit storage: one step per launch, silently
            ctx.set_step_fusion(v)
        ctx.init_fields(np.ones((4, 4, 4)), np.zeros((3, 4, 4, 4)))
        ctx.step(3)
        assert ctx.step_count() == 3
    finally:
        ctx.destroy()


def test_device_moments_and_energy_spectrum(cm):
    import torch
    from paper_1808_04406_amd import diagnostics
    n, u0 = 32, 0.05
    rho, u = inputs.tgv3d(n, u0)
    stream = torch.cuda.Stream()
    ctx = cm.Context("D3Q27", (n, n, n), storage="f32", tau={2: 0.6}, stream=stream)
    try:
        ctx.init_fields(rho, u)
        ctx.step(3)
        r_h, u_h, th_h = ctx.get_moments()
        r_d = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
        u_d = torch.empty(3 * n ** 3, dtype=torch.float64, device="cuda")
        ctx.get_moments_device(rho=r_d, u=u_d)
        ctx.sync()
        assert np.array_equal(r_d.cpu().numpy().reshape(r_h.shape), r_h)
        assert np.array_equal(u_d.cpu().numpy().reshape(u_h.shape), u_h)
        E = diagnostics.energy_spectrum(ctx)
        assert E.sum() == pytest.approx(0.5 * (u_h ** 2).sum(0).mean(), rel=1e-12)
        assert E[2] / E.sum() > 0.999          # the Taylor-Green modes, |m| = sqrt(3)
    finally:
        ctx.destroy()


@pytest.mark.parametrize("kind,shape,storage,thermal,closure", [
    ("D3Q27", (6, 10, 70), "f32", False, False),
    ("D3Q27", (6, 10, 70), "f16", False, False),
    ("D2Q37", (24, 40), "bf16", True, False),
    ("E7B", (12, 30), "f64", True, False),     # a 2D rule of Fig. 2: its name round-trips
    ("D3Q27", (4, 8, 64), "f32", False, True),
])
def test_checkpoint_resume_is_bitwise(cm, orc, tmp_path, kind, shape, storage, thermal, closure):
    """Save after 9 steps, continue 7; a context loaded from the file and
    stepped 7 times holds bitwise the same populations and step count."""
    from paper_1808_04406_amd import checkpoint
    L = orc.lattice(kind)
    S = random_state(orc, kind, shape, seed=41, thermal=thermal)
    tau = taus(kind, 5)
    ctx = cm.Context(kind, shape, storage=storage, thermal=thermal, tau=tau,
                     scale=f16_scales(L["w"]) if storage == "f16" else None)
    try:
        ctx.set_populations(S)
        if closure:
            P = 0.3 * np.random.default_rng(3).normal(size=cm.CLOSURE_NPARAM)
            ctx.closure_load(P, np.full(27, 0.01))
            ctx.closure_tie_even(True)
            ctx.closure_enable(True)
        ctx.step(9)
        ctx.set_tau([tau[2] * 1.01])
        path = str(tmp_path / "state.cmlb")
        checkpoint.save(ctx, path)
        ctx.step(7)
        want, n_want = ctx.get_populations(), ctx.step_count()
    finally:
        ctx.destroy()
    ctx = checkpoint.load(path)
    try:
        assert ctx.step_count() == 9
        ctx.step(7)
        assert ctx.step_count() == n_want == 16
        assert np.array_equal(ctx.get_populations(), want)
    finally:
        ctx.destroy()


@pytest.mark.parametrize("kind,shape,thermal,closure", [
    ("D3Q27", (12, 10, 70), False, False),   # two steps per launch
    ("D2Q37", (24, 40), True, False),        # two steps per launch
    ("D3Q27", (4, 8, 64), False, True),      # learned closure, one step per launch
])
def test_graph_replay_equals_direct_launches(cm, orc, kind, shape, thermal, closure):
    """Steps replayed from a HIP graph give bitwise the direct launches' state:
    several replays, with the program's own work (moments, reductions,
    synchronisation) between them, a rate change (recapture) and step counts
    that leave remainders and flip the buffer parity."""
    S = random_state(orc, kind, shape, seed=23, thermal=thermal)
    tau = taus(kind, 9)
    ctxs = [cm.Context(kind, shape, storage="f32", thermal=thermal, tau=tau) for _ in range(2)]
    try:
        for c in ctxs:
            c.set_step_fusion(2)   # two-step launches where supported (FP32, closure off)
        ctxs[1].set_graph_steps(8)
        P = 0.3 * np.random.default_rng(4).normal(size=cm.CLOSURE_NPARAM)
        for c in ctxs:
            c.set_populations(S)
            if closure:
                c.closure_load(P, np.full(27, 0.01))
                c.closure_tie_even(True)
                c.closure_enable(True)
        for k, n in enumerate((8, 17, 3, 24, 9, 16)):
            if k == 3:
                for c in ctxs:
                    c.set_tau([tau[2] * 1.02])
            for c in ctxs:
                c.step(n)
            ctxs[1].get_moments()
            ctxs[1].reduce()
            ctxs[1].sync()
            a, b = ctxs[0].get_populations(), ctxs[1].get_populations()
            assert ctxs[0].step_count() == ctxs[1].step_count()
            assert np.array_equal(a, b), (k, n)
    finally:
        for c in ctxs:
            c.destroy()


def test_graph_steps_validation(cm):
    ctx = cm.Context("D3Q27", (4, 4, 4), storage="f32", tau={2: 0.6})
    try:
        for bad in (-4, 6, 1):
            with pytest.raises(cm.CmlbError):
                ctx.set_graph_steps(bad)
        ctx.set_graph_steps(0)
        ctx.set_graph_steps(4)
    finally:
        ctx.destroy()


BATCH_CASES = [
    ("D2Q37", (24, 40), "f32", "cm", True),
    ("D2Q37", (13, 41), "f32", "raw_mrt", False),
    ("D2Q37", (16, 16), "f64", "cm", True),
    ("D3Q27", (6, 10, 70), "f32", "cm", False),
    ("D3Q27", (5, 7, 37), "bf16", "cm", False),
    ("D2Q9", (19, 70), "f32", "cm", False),
    ("D3Q27", (3, 4, 300), "f32", "cm", False),    # padded rows
    ("D2Q37", (5, 260), "f32", "cm", True),        # padded rows
]


@pytest.mark.parametrize("kind,shape,storage,model,thermal", BATCH_CASES)
def test_step_batch_equals_individual(cm, orc, kind, shape, storage, model, thermal):
    """Several lattices with different relaxation times and buffer parities
    stepped in one launch per step end bitwise where cmlb_step leaves them."""
    count = 5
    states = [random_state(orc, kind, shape, seed=400 + k, thermal=thermal) for k in range(count)]
    taus_k = [taus(kind, seed=410 + k) for k in range(count)]
    mk = lambda k: cm.Context(kind, shape, storage=storage, model=model, thermal=thermal, tau=taus_k[k])
    solo, batch = [mk(k) for k in range(count)], [mk(k) for k in range(count)]
    try:
        for k in range(count):
            for c in (solo[k], batch[k]):
                c.set_populations(states[k])
                c.step(k % 2)          # different buffer parities
        for n in (7, 4):
            for c in solo:
                c.step(n)
            cm.step_batch(batch, n)
            for a, b in zip(solo, batch):
                assert a.step_count() == b.step_count()
                assert np.array_equal(a.get_populations(), b.get_populations())
    finally:
        for c in solo + batch:
            c.destroy()


def test_step_batch_validation(cm):
    mk = lambda shape=(4, 4, 4), **kw: cm.Context("D3Q27", shape, storage=kw.pop("storage", "f32"), tau={2: 0.6}, **kw)
    a, b, c, d = mk(), mk(), mk((4, 4, 5)), mk(storage="f64")
    try:
        for x in (a, b, c, d):
            x.init_fields(np.ones(x.shape), np.zeros((3,) + x.shape))
        for bad in ([a, c], [a, d], [a, a]):
            with pytest.raises(cm.CmlbError):
                cm.step_batch(bad, 1)
        many = [mk() for _ in range(cm.MAX_BATCH + 1)]
        try:
            for x in many:
                x.init_fields(np.ones(x.shape), np.zeros((3,) + x.shape))
            with pytest.raises(cm.CmlbError):
                cm.step_batch(many, 1)
            cm.step_batch(many[:cm.MAX_BATCH], 2)
            assert all(x.step_count() == 2 for x in many[:cm.MAX_BATCH])
        finally:
            for x in many:
                x.destroy()
        a.closure_load(np.zeros(cm.CLOSURE_NPARAM), np.ones(27))
        a.closure_enable(True)
        with pytest.raises(cm.CmlbError):
            cm.step_batch([a, b], 1)
        assert a.step_count() == b.step_count() == 0   # nothing ran
    finally:
        for x in (a, b, c, d):
            x.destroy()
