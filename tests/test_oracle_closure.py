"""Pins of the oracle's learned-closure pieces (not in the paper: the network
only chooses the rates omega_3..omega_6 of eq:omega).

* forward pass against an independent FP64 torch implementation (exact-erf
  GELU, sigmoid);
* inputs vanish at equilibrium and for orders 0 and 1;
* a network with W3 = 0 and constant logits reproduces the plain collision;
* the analytic gradient of the training objective against central finite
  differences.
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
