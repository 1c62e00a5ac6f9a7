"""The configuration runner on the GPU: records, resume and divergence."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _read(path):
    return [json.loads(line) for line in open(path)]


def test_tgv_records_and_resume(tmp_path):
    from paper_1808_04406_amd import run
    base = {"lattice": "D3Q27", "grid": [32, 32, 32], "tau": {"2": 0.56}, "init": {"kind": "tgv", "u0": 0.05},
            "every": 5}
    full = run.run(dict(base, steps=30), output=str(tmp_path / "full.jsonl"))
    assert [r["step"] for r in full] == [0, 5, 10, 15, 20, 25, 30]
    assert full == _read(tmp_path / "full.jsonl")
    assert all(r["nonfinite"] == 0 for r in full)
    mass0 = full[0]["mass"]
    assert all(abs(r["mass"] - mass0) / mass0 < 1e-6 for r in full)
    ke = [r["ke"] for r in full]
    assert ke[-1] < ke[0] and max(ke) <= ke[0] * (1 + 1e-6)   # viscous decay
    ck = str(tmp_path / "at20.ckpt")
    run.run(dict(base, steps=20, checkpoint_out=ck), output=str(tmp_path / "a.jsonl"))
    rest = run.run({"steps": 10, "every": 5, "init": {"kind": "checkpoint", "path": ck}},
                   output=str(tmp_path / "b.jsonl"))
    assert [r["step"] for r in rest] == [20, 25, 30]
    for a, b in zip(full[4:], rest):                       # bitwise resume
        assert (a["mass"], a["ke"], a["enstrophy"]) == (b["mass"], b["ke"], b["enstrophy"])


def test_thermal_waves_from_yaml(tmp_path):
    from paper_1808_04406_amd import run
    y = tmp_path / "waves.yaml"
    y.write_text("lattice: D2Q37\ngrid: [64, 48]\nthermal: true\nstorage: f32\n"
                 "tau: {2: 0.6, 3: 0.55, 4: 0.6}\nsteps: 40\nevery: 20\n"
                 "init: {kind: waves, shear_amp: 0.002, thermal_amp: 0.01, k: [1, 0], background: [0.0, 0.05]}\n")
    recs = run.run(str(y), output=str(tmp_path / "w.jsonl"))
    assert [r["step"] for r in recs] == [0, 20, 40]
    n = 64 * 48
    # thermal: mass, momentum and energy are collision invariants (FP32 storage rounds each step)
    assert abs(recs[-1]["energy"] - recs[0]["energy"]) < 1e-6 * abs(recs[0]["energy"])
    assert abs(recs[-1]["mass"] - recs[0]["mass"]) < 1e-6 * recs[0]["mass"]
    assert np.allclose(recs[-1]["momentum"], recs[0]["momentum"], rtol=1e-6, atol=1e-5 * n)


def test_divergence_stops_the_run(tmp_path):
    from paper_1808_04406_amd import run
    cfg = tmp_path / "dsl.json"
    cfg.write_text(json.dumps({"lattice": "D2Q37", "grid": [64, 64], "thermal": True,
                               "tau": {"2": 0.50002, "3": 0.50002, "4": 0.50002}, "steps": 4000, "every": 50,
                               "init": {"kind": "double_shear_layer", "u0": 1.0},
                               "output": str(tmp_path / "dsl.jsonl")}))
    assert run.main([str(cfg)]) == 1
    recs = _read(tmp_path / "dsl.jsonl")
    assert recs[-1].get("diverged") and recs[-1]["nonfinite"] > 0
    assert recs[-1]["step"] < 4000
