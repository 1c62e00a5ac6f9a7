"""Linear (von Neumann) stability of the collision operators near tau_2 = 1/2.

Relaxing central *monomial* moments (eq:omega) couples Hermite orders: a
monomial of order 4 carries order-2 Hermite content (eq:hermite-r), which
is the delta term of eq:mrt.  When omega_4 differs from omega_2 the
linearised update is non-normal and, as omega_2 -> 2, has growing modes even
at rest; relaxing the same orders in the orthogonal Hermite basis (raw MRT,
eq:regnmrt) does not.  On D3Q27 the same holds for order 6.  Setting the even
orders >= 4 to omega_2 removes the coupling.  These pins fix the rate sets
used by the benchmark and the long runs.
"""
import pytest

TAU2 = 0.50382  # D3Q27 256^3 Taylor-Green vortex at Re = 1600, L = N / (2 pi)


def test_d3q27_higher_orders_at_one_are_unstable(orc):
    from oracle.analysis import spectral_radius
    cfg = orc.Cfg(lattice="D3Q27", tau={2: TAU2}, tau_hi=1.0)
    r, k = spectral_radius(cfg, (0.0, 0.0, 0.0), nk=6)
    assert r > 1.05
    raw = orc.Cfg(lattice="D3Q27", tau={2: TAU2}, tau_hi=1.0, model="raw_mrt")
    assert spectral_radius(raw, (0.0, 0.0, 0.0), nk=6)[0] < 1.0 + 1e-6


@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.05, 0.0, 0.0), (0.05, 0.05, 0.05), (0.1, 0.0, 0.0)])
def test_d3q27_even_orders_at_omega2_are_stable(orc, u):
    from oracle.analysis import spectral_radius
    cfg = orc.Cfg(lattice="D3Q27", tau={2: TAU2, 3: 1.0, 4: TAU2, 5: 1.0, 6: TAU2})
    assert spectral_radius(cfg, u, nk=6)[0] < 1.0 + 1e-6


def test_d2q37_fourth_order_rate(orc):
    from oracle.analysis import spectral_radius
    unstable = orc.Cfg(lattice="D2Q37", tau={2: TAU2, 3: 1.0, 4: 1.0}, thermal=True)
    stable = orc.Cfg(lattice="D2Q37", tau={2: TAU2, 3: 1.0, 4: TAU2}, thermal=True)
    assert spectral_radius(unstable, (0.0, 0.0), nk=12)[0] > 1.1
    for u in [(0.0, 0.0), (0.1, 0.05)]:
        assert spectral_radius(stable, u, nk=12)[0] < 1.0 + 1e-6
