"""Host-side checks of the C ABI library that need no GPU: it loads, exports
every symbol the header declares, derives the same lattice tables as the
oracle (independently), and rejects invalid parameters before touching a
device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "cmlb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmlb_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported(cm):
    syms = header_symbols()
    assert len(syms) >= 17
    lib = ctypes.CDLL(cm.LIB_PATH)
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.parametrize("kind", ["D2Q9", "D3Q27", "D2Q37"])
def test_lattice_tables_match_oracle(cm, orc, kind):
    a = cm.lattice_info(kind)
    b = orc.lattice(kind)
    assert a["D"] == b["D"] and a["Q"] == b["Q"]
    assert np.array_equal(a["e"], b["e"])
    assert a["r"] == pytest.approx(b["r"], rel=1e-14)
    assert np.allclose(a["w"], b["w"], rtol=1e-13, atol=0)


@pytest.mark.parametrize("bad", [
    dict(lattice="D2Q9", shape=(2, 8, 8)),          # 2D lattice with nz > 1
    dict(lattice="D3Q27", shape=(0, 8, 8)),         # empty grid
    dict(lattice="D3Q27", shape=(8, 8, 8), tau={2: -0.5}),
    dict(lattice="D3Q27", shape=(8, 8, 8), rho0=0.0),
    dict(lattice="D3Q27", shape=(8, 8, 8), thermal=True),
    dict(lattice="D3Q27", shape=(8, 8, 8), model="raw_mrt"),
    dict(lattice="D2Q37", shape=(8, 8), scale=[-1.0] * 37),
    dict(lattice="D3Q27", shape=(4096, 4096, 4096)),
    dict(lattice="D2Q37", shape=(2, 8)),            # D2Q37 shifts reach 3 cells
])
def test_create_rejects_invalid_params(cm, bad):
    with pytest.raises(cm.CmlbError) as ei:
        cm.Context(**bad)
    assert ei.value.code == cm.EINVAL


def test_null_context_is_rejected(cm):
    L = cm.lib()
    assert L.cmlb_step(None, 1) == cm.EINVAL
    assert L.cmlb_set_step_fusion(None, 2) == cm.EINVAL
    assert L.cmlb_set_step_count(None, 3) == cm.EINVAL
    assert L.cmlb_set_graph_steps(None, 64) == cm.EINVAL
    assert L.cmlb_step_batch(None, 1, 1) == cm.EINVAL
    assert L.cmlb_step_batch((ctypes.c_void_p * 1)(None), 1, 1) == cm.EINVAL
    assert L.cmlb_step_batch((ctypes.c_void_p * 1)(None), 0, 1) == cm.EINVAL
    assert L.cmlb_sync(None) == cm.EINVAL
    assert L.cmlb_step_count(None) == -1
    L.cmlb_destroy(None)


def test_max_stable_bisection():
    """Host logic of the stability-boundary search (Sec. III.B)."""
    from paper_1808_04406_amd.studies import max_stable
    for edge in (0.05, 0.2688, 0.7, 1.19):
        m, calls = max_stable(lambda x: x <= edge, 0.05, 1.2, 0.005)
        assert m <= edge < m + 0.005 + 1e-12
        assert len(calls) <= 2 + math.ceil(math.log2(1.15 / 0.005))
        assert all(ok == (x <= edge) for x, ok in calls)
    m, calls = max_stable(lambda x: False, 0.05, 1.2, 0.005)
    assert m == 0.05 and calls == [(0.05, False)]
    m, calls = max_stable(lambda x: True, 0.05, 1.2, 0.005)
    assert m == 1.2 and len(calls) == 2


def test_double_shear_layer_fields():
    """Sec. III.B initial fields: shear layers at y = 1/4 and 3/4, perturbation delta u0."""
    from paper_1808_04406_amd import inputs
    rho, u, th = inputs.double_shear_layer(128, 0.2)
    assert u.shape == (2, 128, 128)
    assert np.allclose(u[0][32], 0.0) and np.allclose(u[0][96], 0.0)      # y = 1/4, 3/4
    assert u[0][64].min() == pytest.approx(0.2 * math.tanh(20.0))           # y = 1/2
    assert u[0][0].max() == pytest.approx(-0.2 * math.tanh(20.0))
    assert abs(u[1]).max() == pytest.approx(0.05 * 0.2, rel=1e-12)
    assert u[1][:, 0] == pytest.approx(np.full(128, 0.01))                 # sin(pi/2) at x = 0
    assert (rho == 1.0).all() and (th == 1.0).all()


def test_energy_spectrum_closed_forms():
    """E(k) of fields with known spectra (CPU tensors; the GPU path runs the
    same function on device moments)."""
    import torch
    from paper_1808_04406_amd import diagnostics, inputs
    u0 = 0.05
    _, u = inputs.tgv3d(32, u0)
    E = diagnostics.spectrum_of(torch.from_numpy(u)).numpy()
    assert E[2] == pytest.approx(u0 ** 2 / 8, rel=1e-12)           # all modes at |m| = sqrt(3)
    assert abs(E.sum() - E[2]) < 1e-15
    n, A = 24, 0.01
    x = np.arange(n)
    v = np.zeros((2, n, n))
    v[1] = A * np.sin(2 * np.pi * 5 * x / n)[None, :]                 # shear wave, mode 5 along x
    E = diagnostics.spectrum_of(torch.from_numpy(v)).numpy()
    assert E[5] == pytest.approx(A ** 2 / 4, rel=1e-12)
    w = np.random.default_rng(1).normal(size=(3, 16, 16, 16))
    E = diagnostics.spectrum_of(torch.from_numpy(w)).numpy()
    assert E.sum() == pytest.approx(0.5 * (w ** 2).sum(0).mean(), rel=1e-12)   # Parseval
    with pytest.raises(ValueError):
        diagnostics.spectrum_of(torch.zeros((3, 4, 4, 8), dtype=torch.float64))


def test_checkpoint_header_errors(tmp_path):
    from paper_1808_04406_amd import checkpoint
    bad = tmp_path / "x.bin"
    bad.write_bytes(b"NOTACKPT" + b"\0" * 32)
    with pytest.raises(ValueError):
        checkpoint.read_header(str(bad))
    import json
    import struct
    hb = json.dumps({"lattice": "D3Q27"}).encode()
    ok = tmp_path / "y.bin"
    ok.write_bytes(checkpoint.MAGIC + struct.pack("<IQ", checkpoint.VERSION, len(hb)) + hb)
    h, off = checkpoint.read_header(str(ok))
    assert h["lattice"] == "D3Q27" and off == 20 + len(hb)
    old = tmp_path / "z.bin"
    old.write_bytes(checkpoint.MAGIC + struct.pack("<IQ", 99, len(hb)) + hb)
    with pytest.raises(ValueError):
        checkpoint.read_header(str(old))
