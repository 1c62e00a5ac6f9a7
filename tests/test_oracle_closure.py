"""Pins of the oracle's learned-closure pieces (not in the paper: the network
only chooses the rates omega_3..omega_6 of eq:omega).

* forward pass against an independent FP64 torch implementation (exact-erf
  GELU, sigmoid);
* inputs vanish at equilibrium and for orders 0 and 1;
* a network with W3 = 0 and constant logits reproduces the plain collision;
* the analytic gradient of the training objective against central finite
  differences;
* the momentum objective (two coarse steps ahead): its adjoint node by
  node, its value at constant rates against two plain oracle steps, and its
  gradient against central finite differences.
"""
import numpy as np
import pytest

from paper_1808_04406_amd import inputs


def unpack(P):
    o, parts = 0, []
    for shape in [(32, 27), (32,), (32, 32), (32,), (4, 32), (4,)]:
        n = int(np.prod(shape))
        parts.append(P[o:o + n].reshape(shape))
        o += n
    assert o == 2084
    return parts


def random_params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return scale * rng.normal(size=2084)


def states(orc, n, seed):
    rng = np.random.default_rng(seed)
    f = []
    for _ in range(n):
        f0 = orc.equilibrium("D3Q27", 1 + 0.05 * rng.normal(), 0.05 * rng.normal(size=3), 1.0)
        f.append(f0 * inputs.perturbation(27, int(rng.integers(1 << 30)), 0.05))
    return np.array(f)


def test_forward_matches_torch(orc):
    import torch
    P = random_params(1)
    x = np.random.default_rng(2).normal(size=(7, 27))
    W1, b1, W2, b2, W3, b3 = (torch.from_numpy(a) for a in unpack(P))
    t = torch.from_numpy(x)
    h1 = torch.nn.functional.gelu(t @ W1.T + b1)
    h2 = torch.nn.functional.gelu(h1 @ W2.T + b2)
    ref = 0.5 + 1.45 * torch.sigmoid(h2 @ W3.T + b3)
    assert np.abs(orc.mlp_rates(P, x) - ref.numpy()).max() < 1e-14


def test_inputs_vanish_at_equilibrium(orc):
    norm = np.random.default_rng(3).uniform(0.5, 2.0, 27)
    f0 = np.array([orc.equilibrium("D3Q27", 1.02, [0.03, -0.04, 0.01], 1.0)])
    assert np.abs(orc.closure_inputs(f0, norm)).max() < 1e-15
    x = orc.closure_inputs(states(orc, 5, 4), norm)
    for p in (0, 1, 3, 9):  # orders 0 and 1: mass and momentum
        assert np.abs(x[:, p]).max() < 1e-15
    assert np.abs(x).max() > 1e-4


def test_constant_rates_fall_back_to_plain_collision(orc):
    f = states(orc, 6, 5)
    norm = np.ones(27)
    P = random_params(6)
    W1, b1, W2, b2, W3, b3 = unpack(P)
    W3[:] = 0.0
    rates = np.array([0.9, 1.3, 0.7, 1.8])
    b3[:] = np.log((rates - 0.5) / 1.45 / (1 - (rates - 0.5) / 1.45))
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    got, om = orc.collide_closure(cfg, f, P, norm)
    assert np.allclose(om, rates, atol=1e-14)
    ref = orc.collide(orc.Cfg(lattice="D3Q27", tau={2: 0.6, **{n + 3: 1 / rates[n] for n in range(4)}}), f)
    assert np.abs(got - ref).max() < 1e-15


def test_gradient_matches_finite_differences(orc):
    f = states(orc, 9, 7)
    fbar = states(orc, 9, 8)
    norm = np.random.default_rng(9).uniform(0.002, 0.02, 27)
    P = random_params(10, scale=0.3)
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.55})
    L0, g = orc.closure_loss_grad(cfg, f, fbar, P, norm)
    assert L0 > 0 and np.abs(g).max() > 0
    rng = np.random.default_rng(11)
    idx = np.concatenate([rng.choice(864, 6, replace=False),                # W1
                          864 + rng.choice(32, 2, replace=False),           # b1
                          896 + rng.choice(1024, 6, replace=False),         # W2
                          1920 + rng.choice(32, 2, replace=False),          # b2
                          1952 + rng.choice(128, 4, replace=False),         # W3
                          2080 + np.arange(4)])                             # b3
    h = 1e-4  # the objective is O(0.05): smaller steps are dominated by rounding
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (orc.closure_loss_grad(cfg, f, fbar, Pp, norm)[0] - orc.closure_loss_grad(cfg, f, fbar, Pm, norm)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-12), k


def test_tie_even(orc):
    """With orders 4 and 6 tied to omega_2 the network's outputs 1 and 3 are
    unused: a constant network gives the plain collision with the tied rates,
    and the gradient of those outputs' weights vanishes (finite differences
    agree on the others)."""
    f = states(orc, 6, 12)
    norm = np.ones(27)
    P = random_params(13)
    W1, b1, W2, b2, W3, b3 = unpack(P)
    W3[:] = 0.0
    rates = np.array([0.9, 1.3, 0.7, 1.8])
    b3[:] = np.log((rates - 0.5) / 1.45 / (1 - (rates - 0.5) / 1.45))
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    got, om = orc.collide_closure(cfg, f, P, norm, tie_even=True)
    ref = orc.collide(orc.Cfg(lattice="D3Q27", tau={2: 0.6, 3: 1 / 0.9, 4: 0.6, 5: 1 / 0.7, 6: 0.6}), f)
    assert np.abs(got - ref).max() < 1e-15
    fbar = states(orc, 6, 14)
    P = random_params(15, scale=0.3)
    norm = np.random.default_rng(16).uniform(0.002, 0.02, 27)
    L0, g = orc.closure_loss_grad(cfg, f, fbar, P, norm, tie_even=True)
    W3g = g[1952:2080].reshape(4, 32)
    assert np.abs(W3g[1]).max() == 0.0 and np.abs(W3g[3]).max() == 0.0
    assert g[2081] == 0.0 and g[2083] == 0.0 and abs(g[2080]) > 0
    h = 1e-4
    for k in (5, 900, 1960, 2080, 2082):
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (orc.closure_loss_grad(cfg, f, fbar, Pp, norm, True)[0]
              - orc.closure_loss_grad(cfg, f, fbar, Pm, norm, True)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-12), k


# ---------------------------------------------------------------------------
# The rounded evaluation (BF16 weights, inputs and activations, as the
# library evaluates the network)
# ---------------------------------------------------------------------------
def bf16_bits(x32):
    """BF16 round-to-nearest-even of FP32 values by bit manipulation."""
    b = np.asarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) & 0xFFFF
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_params(seed, scale=0.3):
    return bf16_bits(random_params(seed, scale).astype(np.float32))


def test_round_sig_is_bf16(orc):
    """round_sig(., 8) is BF16 rounding: random FP32 values, and exact ties
    (low 16 bits 0x8000) in both parities of the kept bit."""
    rng = np.random.default_rng(20)
    v = (rng.normal(size=4000) * np.exp(rng.uniform(-20, 20, 4000))).astype(np.float32)
    mant = rng.integers(0, 1 << 7, 200, dtype=np.uint32) << 16      # the 7 kept fraction bits
    expo = rng.integers(100, 150, 200, dtype=np.uint32) << 23
    ties = (expo | mant | np.uint32(0x8000)).view(np.float32)
    ties = np.concatenate([ties, -ties])
    for arr in (v, ties):
        assert np.array_equal(orc.round_sig(arr.astype(np.float64), 8), bf16_bits(arr))


def unpack_r(orc, P):
    return [orc.round_sig(a, 8).reshape(a.shape) if a.ndim == 2 else a for a in unpack(P)]


def test_rounded_forward_matches_independent(orc):
    """Independent forward pass of the rounded network (torch exact GELU,
    rounding by round_sig): x, h1 and h2 rounded, weights rounded, biases
    exact; rates and f* agree with the oracle's rounded evaluation."""
    import torch
    f = states(orc, 12, 21)
    norm = np.random.default_rng(22).uniform(0.002, 0.02, 27)
    P = random_params(23, 0.3)          # not BF16-exact: the weights must be rounded too
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    r = orc.closure_eval_rounded(cfg, f, None, P, norm)
    W1, b1, W2, b2, W3, b3 = unpack_r(orc, P)
    gelu = lambda a: torch.nn.functional.gelu(torch.from_numpy(a)).numpy()
    x = orc.round_sig(orc.closure_inputs(f, norm), 8).reshape(-1, 27)
    h1 = orc.round_sig(gelu(x @ W1.T + b1), 8).reshape(-1, 32)
    h2 = orc.round_sig(gelu(h1 @ W2.T + b2), 8).reshape(-1, 32)
    om = 0.5 + 1.45 / (1.0 + np.exp(-(h2 @ W3.T + b3)))
    assert np.abs(r["omega"] - om).max() < 1e-13
    ref = np.concatenate([orc.collide(orc.Cfg(lattice="D3Q27", tau={2: 0.6, **{n + 3: 1 / om[k, n] for n in range(4)}}),
                                      f[k:k + 1]) for k in range(len(f))])
    assert np.abs(r["fs"] - ref).max() < 1e-14
    plain, _ = orc.collide_closure(cfg, f, P, norm)
    assert np.abs(r["fs"] - plain).max() > 1e-7   # the rounding is really applied


@pytest.mark.parametrize("tie", [False, True])
def test_rounded_gradient_is_exact_gradient_of_offset_network(orc, tie):
    """The rounded evaluation's gradient (with respect to the master weights,
    the rounding passing derivatives unchanged) is the exact gradient of the
    network that uses the rounded weights and whose rounded operands are the
    exact values plus the (constant) rounding errors: equal objectives, and
    central finite differences of the latter match every bias entry and a
    sample of weights."""
    f = states(orc, 9, 24)
    fbar = states(orc, 9, 25)
    norm = np.random.default_rng(26).uniform(0.002, 0.02, 27)
    Pm = random_params(27, 0.3)        # master weights, not BF16 values
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.55})
    r = orc.closure_eval_rounded(cfg, f, fbar, Pm, norm, tie_even=tie)
    off = r["offsets"]
    assert np.abs(off).max() > 0
    # the weights the rounded network uses; biases stay as given
    P = np.concatenate([a.reshape(-1) for a in unpack_r(orc, Pm)])
    assert np.abs(P - Pm).max() > 0
    L0 = orc.closure_loss_offsets(cfg, f, fbar, P, norm, off, tie_even=tie)
    assert L0 == pytest.approx(r["loss"], rel=1e-14)
    rng = np.random.default_rng(28)
    idx = np.concatenate([rng.choice(864, 8, replace=False), 864 + np.arange(32),
                          896 + rng.choice(1024, 8, replace=False), 1920 + np.arange(32),
                          1952 + rng.choice(128, 8, replace=False), 2080 + np.arange(4)])
    h = 1e-4
    for k in idx:
        Pp, Pn = P.copy(), P.copy()
        Pp[k] += h
        Pn[k] -= h
        fd = (orc.closure_loss_offsets(cfg, f, fbar, Pp, norm, off, tie)
              - orc.closure_loss_offsets(cfg, f, fbar, Pn, norm, off, tie)) / (2 * h)
        assert r["grad"][k] == pytest.approx(fd, rel=1e-6, abs=1e-12), k


def test_rounding_to_many_bits_is_the_fp64_network(orc):
    """With 52 significant bits every rounding is the identity on these
    values: f*, objective and gradient equal the unrounded oracle's."""
    f = states(orc, 7, 29)
    fbar = states(orc, 7, 30)
    norm = np.random.default_rng(31).uniform(0.002, 0.02, 27)
    P = random_params(32, 0.3)
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    r = orc.closure_eval_rounded(cfg, f, fbar, P, norm, bits=53)
    L0, g = orc.closure_loss_grad(cfg, f, fbar, P, norm)
    fs, om = orc.collide_closure(cfg, f, P, norm)
    assert np.abs(r["fs"] - fs).max() < 1e-15 and np.abs(r["omega"] - om).max() < 1e-15
    assert r["loss"] == pytest.approx(L0, rel=1e-13)
    assert np.abs(r["grad"] - g).max() <= 1e-12 * np.abs(g).max()


def test_bounds_follow_the_error_model(orc):
    """With no error model every rounding is certain and the bounds vanish;
    with one they are positive, leave the values unchanged, and grow with
    the modelled errors."""
    f = states(orc, 6, 33)
    fbar = states(orc, 6, 34)
    norm = np.random.default_rng(35).uniform(0.002, 0.02, 27)
    P = bf16_params(36)
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    r0 = orc.closure_eval_rounded(cfg, f, fbar, P, norm)
    assert not r0["bound_fs"].any() and not r0["bound_grad"].any()
    r1 = orc.closure_eval_rounded(cfg, f, fbar, P, norm, err=(1e-4, 1e-4, 1e-4, 1e-4))
    r2 = orc.closure_eval_rounded(cfg, f, fbar, P, norm, err=(1e-3, 1e-3, 1e-3, 1e-3))
    assert r1["bound_fs"].max() > 0 and r1["bound_grad"].max() > 0
    assert np.array_equal(r1["grad"], r0["grad"]) and np.array_equal(r1["fs"], r0["fs"])
    assert (r2["bound_fs"] >= r1["bound_fs"]).all() and (r2["bound_grad"] >= r1["bound_grad"]).all()


def test_bounds_cover_a_perturbed_evaluation(orc):
    """The bound of the rounded network covers the same network evaluated
    with its pre-rounding quantities actually perturbed within the model:
    here every GELU is replaced by GELU * (1 + 1e-3), inside a model of
    eh_rel = 1.2e-3 (|GELU(a)| <= |a|), and every rate, f* and objective
    then stays within the bounds."""
    f = states(orc, 40, 37)
    norm = np.random.default_rng(38).uniform(0.002, 0.02, 27)
    P = bf16_params(39)
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.6})
    r = orc.closure_eval_rounded(cfg, f, None, P, norm, err=(0.0, 1.2e-3, 0.0, 0.0))
    W1, b1, W2, b2, W3, b3 = unpack(P)
    import torch
    gelu = lambda a: torch.nn.functional.gelu(torch.from_numpy(a)).numpy() * (1 + 1e-3)
    x = orc.round_sig(orc.closure_inputs(f, norm), 8).reshape(-1, 27)
    h1 = orc.round_sig(gelu(x @ W1.T + b1), 8).reshape(-1, 32)
    h2 = orc.round_sig(gelu(h1 @ W2.T + b2), 8).reshape(-1, 32)
    om = 0.5 + 1.45 / (1.0 + np.exp(-(h2 @ W3.T + b3)))
    fs = np.concatenate([orc.collide(orc.Cfg(lattice="D3Q27", tau={2: 0.6, **{n + 3: 1 / om[k, n] for n in range(4)}}),
                                     f[k:k + 1]) for k in range(len(f))])
    assert np.abs(fs - r["fs"]).max() > 0          # the perturbation changes some roundings
    assert (np.abs(fs - r["fs"]) <= r["bound_fs"] * (1 + 1e-9) + 1e-15).all()


# --- the momentum objective (two coarse steps ahead) ------------------------

def grid_state(orc, shape, seed, eps=0.03):
    cfg = orc.Cfg(lattice="D3Q27")
    rho, u, _ = inputs.random_fields(shape, seed, drho=0.03, umax=0.05)
    S = orc.init_equilibrium(cfg, rho, u)
    return S * inputs.perturbation(S.shape, seed + 1, eps)


def test_momentum_adjoint_by_brute_force(orc):
    """lam_i(y) = sum_d e_{i,d} D_d(y + e_i), periodic, node by node."""
    shape = (3, 4, 5)
    D = np.random.default_rng(20).normal(size=(3,) + shape)
    lam = orc.momentum_adjoint(D)
    e = orc.lattice("D3Q27")["e"]
    nz, ny, nx = shape
    for node in range(nz * ny * nx):
        z, y, x = node // (ny * nx), (node // nx) % ny, node % nx
        for i in range(27):
            ex, ey, ez = e[i]
            zz, yy, xx = (z + ez) % nz, (y + ey) % ny, (x + ex) % nx
            want = ex * D[0, zz, yy, xx] + ey * D[1, zz, yy, xx] + ez * D[2, zz, yy, xx]
            assert lam[node, i] == pytest.approx(want, abs=1e-15)


@pytest.mark.parametrize("tie", [False, True])
def test_momentum_objective_at_constant_rates_is_two_plain_steps(orc, tie):
    """A constant network: the objective equals the momentum mismatch after
    two steps of the plain collision (orc.run), computed from the momentum
    moments of the stepped state."""
    shape = (4, 5, 6)
    S = grid_state(orc, shape, 21)
    target = grid_state(orc, shape, 23)
    P = random_params(24)
    W1, b1, W2, b2, W3, b3 = unpack(P)
    W3[:] = 0.0
    rates = np.array([0.9, 1.3, 0.7, 1.8])
    b3[:] = np.log((rates - 0.5) / 1.45 / (1 - (rates - 0.5) / 1.45))
    tau2 = 0.55
    cfg = orc.Cfg(lattice="D3Q27", tau={2: tau2})
    loss, g, D = orc.closure_momentum_objective(cfg, S, target, P, np.ones(27), tie_even=tie)
    om = {3: rates[0], 4: rates[1], 5: rates[2], 6: rates[3]}
    if tie:
        om[4] = om[6] = 1.0 / tau2
    S2 = S.copy()
    orc.run(orc.Cfg(lattice="D3Q27", tau={2: tau2, **{n: 1.0 / om[n] for n in om}}), S2, 2)
    rho2, u2, _ = orc.moments("D3Q27", S2)
    rhot, ut, _ = orc.moments("D3Q27", target)
    dj = rho2[None] * u2 - rhot[None] * ut
    assert loss == pytest.approx(float(np.mean(np.sum(dj * dj, axis=0))), rel=1e-12)
    assert np.allclose(D, 2.0 / rho2.size * dj, rtol=1e-10, atol=1e-18)


@pytest.mark.parametrize("tie", [False, True])
def test_momentum_objective_gradient_matches_finite_differences(orc, tie):
    shape = (3, 4, 5)
    S = grid_state(orc, shape, 31)
    target = grid_state(orc, shape, 33)
    norm = np.random.default_rng(34).uniform(0.002, 0.02, 27)
    P = random_params(35, scale=0.3)
    cfg = orc.Cfg(lattice="D3Q27", tau={2: 0.55})
    L0, g, _ = orc.closure_momentum_objective(cfg, S, target, P, norm, tie_even=tie)
    assert L0 > 0 and np.abs(g).max() > 0
    rng = np.random.default_rng(36)
    idx = np.concatenate([rng.choice(864, 4, replace=False), 864 + rng.choice(32, 2, replace=False),
                          896 + rng.choice(1024, 4, replace=False), 1920 + rng.choice(32, 2, replace=False),
                          1952 + rng.choice(128, 4, replace=False), 2080 + np.arange(4)])
    h = 1e-4
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (orc.closure_momentum_objective(cfg, S, target, Pp, norm, tie_even=tie)[0]
              - orc.closure_momentum_objective(cfg, S, target, Pm, norm, tie_even=tie)[0]) / (2 * h)
        if tie and 2080 <= k and (k - 2080) % 2 == 1:
            assert g[k] == 0.0 and abs(fd) < 1e-13   # tied outputs do not act
        else:
            assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-13), k
