"""Learned closure on the GPU against the FP64 oracle.

The library evaluates the network with BF16 weights, inputs and hidden
activations on the matrix cores (FP32 accumulation) and trains it with the
derivative passing through each rounding unchanged.  The oracle's rounded
evaluation (oracle.closure_eval_rounded) rounds the same quantities in FP64
arithmetic, so both compute the same network.  Every output is compared
element by element within a bound the oracle derives per element from an
error model of the library's arithmetic before each rounding (ERR_MODEL):

* inputs x_p: the non-equilibrium central moments are FP32 sums over the 27
  deviations: three per-axis sweeps (2 roundings each), the binomial shift
  to central moments (3 per axis) and the deviation equilibrium and
  division (3), each below 2^-24 of sum_i |f_i - w_i rho0| (1 + |u|)^6 <
  1.4 sum |f_i - w_i|: 32 * 2^-24 * sum |f_i - w_i rho0| / (rho sigma_p);
* activations: GELU as max(a, 0) - |a| P(|a|) with a degree-11 polynomial
  P of Phi(-x) (paper_1808_04406_amd/gelu_poly.py), at most 4.6e-6 |a|
  from GELU(a) in FP32, taken as 5e-6 |a|; the FP32 accumulation of at
  most 33 terms times |GELU'| <= 1.13, plus a few roundings inside GELU:
  48 * 2^-24 * (|b| + sum |W h|); the logits carry the same accumulation term;
* GELU' in the backward pass: Abramowitz and Stegun 7.1.26 (erf error
  1.5e-7, so 7.5e-8 in Phi), the a phi(a) term and the FP32 sum: 3e-7.

Where a quantity's error interval rounds to other BF16 values than the
oracle's, the library may use any of them.  The oracle enumerates those of
the inputs (one step of x moves every layer-1 pre-activation) and carries
the distances of the others forward through the network and its backward
pass as deviation bounds (products, sums and smooth maps to first order,
with the second-order terms of GELU and the sigmoid written out).  That
gives bound_fs and bound_grad.  What remains is FP32 arithmetic outside the
roundings:
* the collision: 2e-6 of the largest deviation (about 30 FP32 roundings, as
  for the plain kernel);
* the gradient: each node's share carries the relative FP32 error of its
  residuals f* - fbar (about 30 roundings of the deviation scale, which is
  below 5 |f* - fbar| on these states) and of the chain through the
  reconstruction and the two layers, a few hundred roundings of 2^-24 in
  all: ETA = 2e-5 of the sum over nodes of |node share|.
"""
import numpy as np
import pytest

from paper_1808_04406_amd import inputs

pytestmark = pytest.mark.gpu

ERR_MODEL = (32 * 2.0 ** -24, 5e-6, 48 * 2.0 ** -24, 3e-7)
ETA = 2e-5


def bf16_round(x):
    f = np.asarray(x, np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) & 0xFFFF
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def params(seed, scale=0.4):
    return bf16_round(scale * np.random.default_rng(seed).normal(size=2084))


def near_eq_state(orc, shape, seed, eps=0.03):
    cfg = orc.Cfg(lattice="D3Q27")
    rho, u, _ = inputs.random_fields(shape, seed, drho=0.03, umax=0.05)
    S = orc.init_equilibrium(cfg, rho, u)
    return S * inputs.perturbation(S.shape, seed + 1, eps)


@pytest.mark.parametrize("tie,shape", [(False, (3, 5, 128)), (True, (3, 5, 128)),
                                       (False, (2, 3, 300))])   # the last has padded rows
def test_closure_step_matches_oracle(cm, orc, tie, shape):
    w = orc.lattice("D3Q27")["w"]
    S = near_eq_state(orc, shape, 50)
    S = (S - w[:, None, None, None]).astype(np.float32).astype(np.float64) + w[:, None, None, None]
    P = params(51)
    sigma = np.random.default_rng(52).uniform(0.005, 0.03, 27).astype(np.float32).astype(np.float64)
    ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6})
    ctx.closure_load(P, sigma)
    ctx.closure_tie_even(tie)
    ctx.closure_enable(True)
    ctx.set_populations(S)
    ctx.step(1)
    got = ctx.get_populations().reshape(27, -1).T
    ctx.destroy()
    nodes = np.arange(int(np.prod(shape)))
    fin = orc.gather_nodes("D3Q27", S, nodes)
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    r = orc.closure_eval_rounded(cfg, fin, None, P, sigma, tie_even=tie, err=ERR_MODEL)
    ref = r["fs"]
    assert r["omega"].std() > 0.05   # the network really varies the rates
    bound = r["bound_fs"] + 2e-6 * np.abs(ref - w).max()
    err = np.abs(got - ref)
    print(f"closure step: max|df| = {err.max():.3e}, max err/bound = {(err / bound).max():.3f}, "
          f"nodes where a rounding may differ {(r['bound_fs'].max(1) > 0).mean():.3f}")
    assert (err <= bound).all()


def test_constant_network_equals_plain_kernel(cm, orc):
    shape = (4, 6, 64)
    S = near_eq_state(orc, shape, 53)
    rates = np.array([0.9, 1.3, 0.7, 1.8])
    P = params(54)
    P[1952:2080] = 0.0
    P[2080:] = np.log((rates - 0.5) / 1.45 / (1 - (rates - 0.5) / 1.45))
    tau = {2: 0.6, 3: 1 / rates[0], 4: 1 / rates[1], 5: 1 / rates[2], 6: 1 / rates[3]}
    a = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6})
    a.closure_load(P, np.ones(27))
    a.closure_enable(True)
    b = cm.Context("D3Q27", shape, storage="f32", tau=tau)
    for c in (a, b):
        c.set_populations(S)
        c.step(3)
    fa, fb = a.get_populations(), b.get_populations()
    a.destroy()
    b.destroy()
    scale = np.abs(fb - orc.lattice("D3Q27")["w"][:, None, None, None]).max()
    assert np.abs(fa - fb).max() <= 1e-6 * scale + 1e-7


@pytest.mark.parametrize("tie", [False, True])
def test_closure_gradient_matches_oracle(cm, orc, tie):
    """Every one of the 2084 gradient entries (W1, b1, W2, b2, W3, b3) and the
    objective, against the oracle's rounded network, within its per-entry
    bound."""
    import torch
    shape = (3, 4, 64)
    n = int(np.prod(shape))
    w = orc.lattice("D3Q27")["w"]
    pairs = [(near_eq_state(orc, shape, 60 + 2 * k), near_eq_state(orc, shape, 61 + 2 * k)) for k in range(2)]
    dev = lambda S: (S - w[:, None, None, None]).reshape(27, -1)
    st = torch.from_numpy(np.stack([dev(a) for a, _ in pairs]).astype(np.float32)).cuda()
    tg = torch.from_numpy(np.stack([dev(b) for _, b in pairs]).astype(np.float32)).cuda()
    P = params(62, scale=0.3)
    sigma = np.random.default_rng(63).uniform(0.005, 0.03, 27).astype(np.float32).astype(np.float64)
    ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6})
    ctx.closure_load(P, sigma)
    ctx.closure_tie_even(tie)
    obj, g = ctx.closure_objective(st, tg, n_pairs=2)
    ctx.destroy()
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    fin = np.concatenate([orc.gather_nodes("D3Q27", (st[k].double().cpu().numpy().reshape((27,) + shape)
                                                     + w[:, None, None, None]), np.arange(n)) for k in range(2)])
    tgt = np.concatenate([(tg[k].double().cpu().numpy() + w[:, None]).T for k in range(2)])
    r = orc.closure_eval_rounded(cfg, fin, tgt, P, sigma, tie_even=tie, err=ERR_MODEL)
    o_g = r["grad"]
    bound = r["bound_grad"] + ETA * r["abs_grad"]
    err = np.abs(np.append(g, obj) - np.append(o_g, r["loss"]))
    ratio = err / np.where(bound > 0, bound, np.inf)
    worst = int(np.argmax(ratio))
    print(f"objective {obj:.6e} vs {r['loss']:.6e}; gradient max err/bound {ratio.max():.3f} (entry {worst}), "
          f"median {np.median(ratio):.3f}; median bound / |entry| "
          f"{np.median(bound[:-1] / np.maximum(np.abs(o_g), 1e-30)):.3e}")
    exact_zero = bound == 0   # tied outputs: both sides give exactly 0
    assert (err[exact_zero] == 0).all()
    assert (err <= bound).all(), np.nonzero(err > bound)[0][:20]
    for name, sl in (("b1", slice(864, 896)), ("b2", slice(1920, 1952)), ("b3", slice(2080, 2084))):
        assert np.abs(o_g[sl]).max() > 0, name


def test_training_learns_the_rates(cm, orc):
    """Targets are the oracle's one-step result with known rates for orders
    3..6; Adam on the GPU objective moves the network towards them."""
    import torch
    shape = (2, 4, 64)
    w = orc.lattice("D3Q27")["w"]
    a = near_eq_state(orc, shape, 70)
    true_tau = {2: 0.6, 3: 1 / 1.4, 4: 1 / 0.8, 5: 1 / 1.6, 6: 1 / 0.9}
    b = a.copy()
    orc.run(orc.Cfg(lattice="D3Q27", tau=true_tau), b, 1)
    st = torch.from_numpy((a - w[:, None, None, None]).reshape(1, 27, -1).astype(np.float32)).cuda()
    tg = torch.from_numpy((b - w[:, None, None, None]).reshape(1, 27, -1).astype(np.float32)).cuda()
    ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6})
    ctx.closure_load(params(72, 0.2), np.full(27, 0.02))
    first = ctx.closure_train_step(st, tg, lr=2e-2)
    for _ in range(80):
        last = ctx.closure_train_step(st, tg, lr=2e-2)
    P = ctx.closure_get()
    ctx.destroy()
    print(f"objective {first:.3e} -> {last:.3e}")
    assert np.isfinite(P).all()
    assert last < 0.2 * first


@pytest.mark.parametrize("tie,frozen", [(False, ()), (True, (5,))])
def test_adam_steps_follow_their_definition(cm, orc, tie, frozen):
    """Three Adam steps with non-default constants (cmlb_closure_set_adam):
    each step's master weights equal P - lr mhat / (sqrt(vhat) + eps), with
    the moments carried in FP64 from the library's own gradients, within the
    FP32 roundings of the update; entries with no gradient (tied outputs)
    and the weights of frozen outputs (cmlb_closure_freeze) stay exactly
    unchanged.  Invalid constants are rejected."""
    import torch
    shape = (2, 4, 64)
    w = orc.lattice("D3Q27")["w"]
    a = near_eq_state(orc, shape, 90)
    b = near_eq_state(orc, shape, 91)
    st = torch.from_numpy((a - w[:, None, None, None]).reshape(1, 27, -1).astype(np.float32)).cuda()
    tg = torch.from_numpy((b - w[:, None, None, None]).reshape(1, 27, -1).astype(np.float32)).cuda()
    ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6})
    ctx.closure_load(params(92, 0.3), np.full(27, 0.02))
    ctx.closure_tie_even(tie)
    for bad in ((1.0, 0.999, 1e-8), (0.9, -0.1, 1e-8), (0.9, 0.999, 0.0), (0.9, 0.999, float("nan"))):
        with pytest.raises(cm.CmlbError) as ei:
            ctx.closure_set_adam(*bad)
        assert ei.value.code == cm.EINVAL
    with pytest.raises(ValueError):
        ctx.closure_freeze((2,))
    b1, b2, eps, lr = 0.8, 0.99, 1e-10, 0.01
    ctx.closure_set_adam(b1, b2, eps)
    ctx.closure_freeze(frozen)
    keep = np.zeros(2084, bool)
    for n in frozen:
        keep[1952 + 32 * (n - 3):1952 + 32 * (n - 2)] = True
        keep[2080 + n - 3] = True
    P = ctx.closure_get().astype(np.float64)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    for t in range(1, 4):
        _, g = ctx.closure_objective(st, tg)
        g = g.astype(np.float64)
        if frozen:
            assert (g[keep] != 0).any()      # frozen although the objective depends on them
        g[keep] = 0.0
        ctx.closure_train_step(st, tg, lr)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        step = lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        ref = P - step
        P = ctx.closure_get().astype(np.float64)
        err = np.abs(P - ref)
        bound = 2.0 ** -23 * np.abs(ref) + 1e-5 * np.abs(step)
        print(f"step {t}: max |step| {np.abs(step).max():.3e}, max err/bound {(err / np.maximum(bound, 1e-300)).max():.3f}")
        assert (err <= bound).all(), np.nonzero(err > bound)[0][:20]
        assert (P[m == 0] == ref[m == 0]).all()
        assert np.abs(step).max() > 0.5 * lr
    ctx.destroy()
    # biases of outputs 1 and 3 (orders 4 and 6) get a gradient only when untied
    assert (m[[2081, 2083]] == 0).all() == tie


@pytest.mark.parametrize("shape", [(8, 8, 16), (4, 2, 300)])   # the second has padded rows
def test_box_filter(cm, orc, shape):
    import torch
    nz, ny, nx = shape
    S = near_eq_state(orc, shape, 80)
    w = orc.lattice("D3Q27")["w"]
    ctx = cm.Context("D3Q27", shape, storage="f64")
    ctx.set_populations(S)
    out = torch.empty(27 * (nz // 2) * (ny // 2) * (nx // 2), dtype=torch.float32, device="cuda")
    ctx.box_filter(2, out)
    torch.cuda.synchronize()
    ctx.destroy()
    ref = (S - w[:, None, None, None]).reshape(27, nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(2, 4, 6))
    assert np.abs(out.cpu().numpy().reshape(ref.shape) - ref).max() < 1e-8


def test_trained_closure_against_fixed_rates(cm):
    """What training gains over the method without the network: 128^3
    random multi-mode runs at Re = 1e5, box-filtered 2^3 -> 64^3 (one coarse
    step = 2 fine steps).  The baseline is the plain method at the rates it
    runs stably here: odd orders at 1, even orders at omega_2 (any other
    even-order rate makes the linearised update grow as tau_2 -> 1/2, so the
    network's even outputs are tied to omega_2).  The network starts at that
    fixed set, trains 300 Adam steps on seeds 0 and 1 and is evaluated on
    held-out seed 2.

    Measured: it matches the fixed set to 0.1 % and does not beat it by a
    useful margin: constant omega_3 or omega_5 anywhere in [0.6, 1.94] moves
    the held-out objective by less than 1 % (the odd orders have almost no
    leverage on this objective), so the rate 1 the plain method uses is
    already near the best.  Against every order >= 3 at rate 1 (the unstable
    set) the held-out objective is 1.5x lower."""
    import math
    import torch
    from paper_1808_04406_amd import studies
    n_fine, factor, u0, re = 128, 2, 0.05, 1.0e5
    tau_f = 0.5 + 3.0 * u0 * (n_fine / (2 * math.pi)) / re
    tau_c = 0.5 + (tau_f - 0.5) / factor
    nc = n_fine // factor
    data = {}
    for seed in (0, 1, 2):
        rho, u = inputs.random_multimode(n_fine, seed, kmax=4, umax=u0)
        fine = cm.Context("D3Q27", (n_fine,) * 3, storage="f32", tau=studies._tgv_rates(tau_f))
        try:
            fine.init_fields(rho, u)
            fine.step(100)
            pairs = []
            for _ in range(3):
                a = torch.empty(27 * nc ** 3, dtype=torch.float32, device="cuda")
                b = torch.empty_like(a)
                fine.box_filter(factor, a)
                fine.step(factor)
                fine.box_filter(factor, b)
                pairs.append((a, b))
                fine.step(40 - factor)
            fine.sync()
        finally:
            fine.destroy()
        data[seed] = pairs
    train, test = data[0] + data[1], data[2]
    sigma = studies._input_scales(train[0][0].cpu().numpy(), nc)
    rate1 = studies._constant_net([1.0] * 4)
    stable = studies._constant_net([1.0] * 4, seed=1, scale=0.1)
    ctx = cm.Context("D3Q27", (nc,) * 3, storage="f32", tau={2: tau_c})
    try:
        def objective(params, pairs, tie):
            ctx.closure_load(params, sigma)
            ctx.closure_tie_even(tie)
            return float(np.mean([ctx.closure_objective(a, b, grad=False) for a, b in pairs]))

        unstable = objective(rate1, test, False)
        fixed = objective(stable, test, True)
        sweep = [objective(studies._constant_net([w, 1.0, w, 1.0], seed=1, scale=0.1), test, True)
                 for w in (0.6, 1.4, 1.94)]
        ctx.closure_load(stable, sigma)
        ctx.closure_tie_even(True)
        for it in range(300):
            a, b = train[it % len(train)]
            ctx.closure_train_step(a, b, 2e-3 * (1.0 - it / 300))
        learned = objective(ctx.closure_get().astype(np.float64), test, True)
    finally:
        ctx.destroy()
    print(f"held-out objective: every order >= 3 at 1 {unstable:.4e}, fixed odd 1 / even omega_2 {fixed:.4e}, "
          f"trained network {learned:.4e} (ratio to the fixed set {learned / fixed:.5f}); constant odd rates "
          f"0.6 / 1.4 / 1.94: {', '.join(f'{v / fixed:.4f}' for v in sweep)}")
    assert learned <= 1.001 * fixed             # training keeps at least the fixed set's quality
    assert unstable / learned > 1.3             # and gains over the unstable all-ones set
    assert all(0.99 < v / fixed < 1.03 for v in sweep)   # the odd orders barely move the objective


@pytest.mark.parametrize("tie", [False, True])
def test_momentum_objective_matches_oracle(cm, orc, tie):
    """The momentum objective (two coarse steps ahead) and every gradient
    entry against the oracle.  The library's closure step f1 of each pair is
    taken from a context stepped once with the same network (the same kernel
    and inputs, so the same values); the oracle computes the momentum
    mismatch from it in FP64, and the gradient of its rounded network for
    the resulting adjoint lam_i(y) = e_i . D(y + e_i), within the per-entry
    bound of that evaluation plus ETA of the absolute node shares."""
    import torch
    shape = (3, 4, 64)
    n = int(np.prod(shape))
    w = orc.lattice("D3Q27")["w"]
    e = orc.lattice("D3Q27")["e"].astype(np.float64)
    wb = w[:, None, None, None]
    q32 = lambda S: (S - wb).astype(np.float32).astype(np.float64) + wb
    pairs = [(q32(near_eq_state(orc, shape, 80 + 2 * k)), q32(near_eq_state(orc, shape, 81 + 2 * k)))
             for k in range(2)]
    dev = lambda S: (S - wb).reshape(27, -1)
    st = torch.from_numpy(np.stack([dev(a) for a, _ in pairs]).astype(np.float32)).cuda()
    tg = torch.from_numpy(np.stack([dev(b) for _, b in pairs]).astype(np.float32)).cuda()
    P = params(82, scale=0.3)
    sigma = np.random.default_rng(83).uniform(0.005, 0.03, 27).astype(np.float32).astype(np.float64)
    ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6})
    ctx.closure_load(P, sigma)
    ctx.closure_tie_even(tie)
    ctx.closure_set_objective("momentum")
    obj, g = ctx.closure_objective(st, tg, n_pairs=2)
    ctx.destroy()
    # the library's closure step of each state
    f1 = []
    for a, _ in pairs:
        c = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6})
        c.closure_load(P, sigma)
        c.closure_tie_even(tie)
        c.closure_enable(True)
        c.set_populations(a)
        c.step(1)
        f1.append(c.get_populations())
        c.destroy()
    ntot = 2 * n
    fin, fbar, loss_o = [], [], 0.0
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    rs = [orc.closure_eval_rounded(cfg, orc.gather_nodes("D3Q27", a, np.arange(n)), None, P, sigma,
                                   tie_even=tie, err=ERR_MODEL) for a, _ in pairs]
    for k, (a, b) in enumerate(pairs):
        dj = orc.gather_nodes("D3Q27", f1[k], np.arange(n)) @ e - b.reshape(27, n).T @ e
        loss_o += float(np.sum(dj * dj)) / ntot
        lam = orc.momentum_adjoint((2.0 / ntot) * dj.T.reshape((3,) + shape))
        fin.append(orc.gather_nodes("D3Q27", a, np.arange(n)))
        fbar.append(rs[k]["fs"] - lam * w[None, :] * (ntot / 2.0))   # residual of the rounded network = lam
    r = orc.closure_eval_rounded(cfg, np.concatenate(fin), np.concatenate(fbar), P, sigma, tie_even=tie,
                                 err=ERR_MODEL)
    print(f"momentum objective {obj:.6e} vs {loss_o:.6e}")
    assert obj == pytest.approx(loss_o, rel=1e-5)
    bound = r["bound_grad"][:-1] + ETA * r["abs_grad"][:-1]
    err = np.abs(g - r["grad"])
    ratio = err / np.where(bound > 0, bound, np.inf)
    print(f"momentum gradient max err/bound {ratio.max():.3f}, median bound / |entry| "
          f"{np.median(bound / np.maximum(np.abs(r['grad']), 1e-30)):.3e}")
    assert (err[bound == 0] == 0).all()
    assert (err <= bound).all(), np.nonzero(err > bound)[0][:20]
    assert np.abs(r["grad"][2080:2084]).max() > 0


def test_momentum_objective_equals_two_plain_steps(cm, orc):
    """On 64^3, at constant rates (W3 = 0), the momentum objective of an
    unpadded batch equals the mismatch of two plain steps of the same state,
    run by a plain context with those rates (in its own layout) and read
    through cmlb_get_moments."""
    import torch
    from paper_1808_04406_amd import studies
    shape = (64, 64, 64)
    w = orc.lattice("D3Q27")["w"][:, None, None, None]
    e = orc.lattice("D3Q27")["e"][:, :3].astype(np.float64)
    S = (near_eq_state(orc, shape, 95) - w).astype(np.float32)
    T = (near_eq_state(orc, shape, 97) - w).astype(np.float32)
    st = torch.from_numpy(S.reshape(1, 27, -1)).cuda()
    tg = torch.from_numpy(T.reshape(1, 27, -1)).cuda()
    ctx = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6})
    plain = cm.Context("D3Q27", shape, storage="f32", tau={2: 0.6, 3: 1.0, 4: 0.6, 5: 1.0, 6: 0.6})
    try:
        ctx.closure_load(studies._constant_net([1.0] * 4, seed=1, scale=0.1), np.ones(27))
        ctx.closure_tie_even(True)
        ctx.closure_set_objective("momentum")
        obj = ctx.closure_objective(st, tg, grad=False)
        plain.set_populations(S.astype(np.float64) + w)
        plain.step(2)
        rho, u, _ = plain.get_moments()
    finally:
        ctx.destroy()
        plain.destroy()
    j2 = rho[None] * u
    jbar = np.einsum("id,i...->d...", e, T.astype(np.float64) + w)
    ref = float(np.mean(np.sum((j2 - jbar) ** 2, axis=0)))
    print(f"momentum objective {obj:.6e}, two plain steps {ref:.6e}")
    assert abs(obj - ref) <= 1e-4 * ref


def test_momentum_trained_closure_beats_fixed_rates(cm):
    """What training on the momentum objective (cmlb_closure_set_objective:
    the momentum two coarse steps ahead) gains over the method without the
    network.  128^3 random multi-mode runs at Re = 1e5 filtered to 64^3;
    seeds 0 and 1 train, seed 2 is held out; the baseline is the stable
    fixed rates (odd orders at 1, even orders at omega_2), which the network
    starts from.  The network sets omega_3 (omega_5 frozen at 1: learned
    too, it makes the rollout diverge), with Adam's eps scaled to the
    gradient.  Margins: the held-out objective at most 0.6 of the
    baseline's (measured 0.31 in the study with more data), and in the
    64^3 Taylor-Green rollout against the filtered 128^3 run, KE and
    enstrophy errors no larger than the baseline's and the enstrophy error
    at least 3 % smaller (measured 7 % in the study)."""
    import math
    import torch
    from paper_1808_04406_amd import studies
    n_fine, factor, u0, re = 128, 2, 0.05, 1.0e5
    tau_f = 0.5 + 3.0 * u0 * (n_fine / (2 * math.pi)) / re
    tau_c = 0.5 + (tau_f - 0.5) / factor
    nc = n_fine // factor
    data = {}
    for seed in (0, 1, 2):
        rho, u = inputs.random_multimode(n_fine, seed, kmax=4, umax=u0)
        fine = cm.Context("D3Q27", (n_fine,) * 3, storage="f32", tau=studies._tgv_rates(tau_f))
        try:
            fine.init_fields(rho, u)
            fine.step(200)
            pairs = []
            for _ in range(3):
                a = torch.empty(27 * nc ** 3, dtype=torch.float32, device="cuda")
                b = torch.empty_like(a)
                fine.box_filter(factor, a)
                fine.step(2 * factor)
                fine.box_filter(factor, b)
                pairs.append((a, b))
                fine.step(80 - 2 * factor)
            fine.sync()
        finally:
            fine.destroy()
        data[seed] = pairs
    train, test = data[0] + data[1], data[2]
    sigma = studies._input_scales(train[0][0].cpu().numpy(), nc)
    stable = studies._constant_net([1.0] * 4, seed=1, scale=0.1)
    ctx = cm.Context("D3Q27", (nc,) * 3, storage="f32", tau={2: tau_c})
    try:
        def objective(params, pairs):
            ctx.closure_load(params, sigma)
            ctx.closure_tie_even(True)
            ctx.closure_set_objective("momentum")
            return float(np.mean([ctx.closure_objective(a, b, grad=False) for a, b in pairs]))

        fixed = objective(stable, test)
        ctx.closure_load(stable, sigma)
        ctx.closure_tie_even(True)
        ctx.closure_set_objective("momentum")
        g0 = np.concatenate([ctx.closure_objective(a, b)[1] for a, b in train]).astype(np.float64)
        ctx.closure_set_adam(0.9, 0.999, 1e-6 * float(np.sqrt(np.mean(g0 ** 2))))
        ctx.closure_freeze((5,))
        steps = 3000
        for it in range(steps):
            a, b = train[it % len(train)]
            ctx.closure_train_step(a, b, 0.1 * (1.0 - it / steps))
        P = ctx.closure_get().astype(np.float64)
        learned = objective(P, test)
    finally:
        ctx.destroy()
    print(f"held-out momentum objective: stable fixed {fixed:.4e}, trained {learned:.4e} ({learned / fixed:.3f})")
    assert learned <= 0.6 * fixed
    # rollout: 64^3 Taylor-Green from the filtered 128^3 state, 400 coarse steps
    rho, u = inputs.tgv3d(n_fine, u0)
    fine = cm.Context("D3Q27", (n_fine,) * 3, storage="f32", tau=studies._tgv_rates(tau_f))
    runs = {"fixed": stable, "trained": P}
    ctxs = {}
    buf = torch.empty(27 * nc ** 3, dtype=torch.float32, device="cuda")
    try:
        fine.init_fields(rho, u)
        fine.box_filter(factor, buf)
        fine.sync()
        for k, params in runs.items():
            c = cm.Context("D3Q27", (nc,) * 3, storage="f32", tau={2: tau_c})
            ctxs[k] = c
            c.closure_load(params, sigma)
            c.closure_tie_even(True)
            c.closure_enable(True)
            c.load_deviations_device(buf)
            c.sync()
        probe = cm.Context("D3Q27", (nc,) * 3, storage="f32", tau={2: tau_c})
        ctxs["probe"] = probe
        err = {k: [0.0, 0.0] for k in runs}
        for t in range(50, 401, 50):
            fine.step(50 * factor)
            fine.box_filter(factor, buf)
            fine.sync()
            probe.load_deviations_device(buf)
            ref = probe.reduce()
            for k in runs:
                ctxs[k].step(50)
                g = ctxs[k].reduce()
                err[k][0] = max(err[k][0], abs(g["ke"] - ref["ke"]) / ref["ke"])
                err[k][1] = max(err[k][1], abs(g["enstrophy"] - ref["enstrophy"]) / ref["enstrophy"])
    finally:
        for c in ctxs.values():
            c.destroy()
        fine.destroy()
    print(f"rollout max relative errors (KE, enstrophy): fixed {err['fixed']}, trained {err['trained']}")
    assert err["trained"][0] <= err["fixed"][0]
    assert err["trained"][1] <= 0.97 * err["fixed"][1]
