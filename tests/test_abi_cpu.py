"""Host-side checks of the C ABI library that need no GPU: it loads, exports
every symbol the header declares, derives the same lattice tables as the
oracle (independently), and rejects invalid parameters before touching a
device."""
import ctypes
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
    assert L.cmlb_sync(None) == cm.EINVAL
    assert L.cmlb_step_count(None) == -1
    L.cmlb_destroy(None)
