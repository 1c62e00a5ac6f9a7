"""Run a simulation from a JSON or YAML configuration and write FP64
diagnostic histories as JSON lines.

    python -m paper_1808_04406_amd.run CONFIG [--out FILE]

Configuration keys (x first in ``grid``; defaults in brackets):

    lattice      "D2Q9" | "D3Q27" | "D2Q37" (also "E9A") | "E9B" | "E9C" | "E9D"
                 | "E7A" | "E7B" | "E7C" | "E7D" (the 2D rules of Fig. 2)  (required)
    grid         [nx, ny] or [nx, ny, nz]                         (required)
    storage      "f64" | "f32" | "bf16" | "f16"                   ["f32"]
    model        "cm" | "raw_mrt" | "reg_bgk" (the last two: D2Q37)  ["cm"]
    thermal      true | false (the 2D Hermite rules)              [false]
    rho0, theta0 reference density and temperature                [1.0, 1.0]
    tau          {order: relaxation time}, orders 2..7 (missing orders: 1.0)
    scale        storage scale per population (Q values, 0 = automatic) [automatic]
    init         {"kind": ...} with
                   "rest"                 uniform rho0, u = 0
                   "tgv"                  Taylor-Green vortex: u0 [0.05], background [0, ...]
                                          (3D: a cubic grid)
                   "waves"                shear and thermal waves (2D): shear_amp, thermal_amp,
                                          k [[1, 0]], kt, background
                   "double_shear_layer"   (square 2D): u0 (lattice units), sharpness [80],
                                          delta [0.05]
                   "random_multimode"     (cubic 3D or square 2D): seed [0], kmax [4], umax [0.05]
                   "checkpoint"           path: resume from a checkpoint file (the other
                                          context keys are then taken from the file)
    steps        steps to run                                     (required)
    every        steps between diagnostics records               [steps, at most 100]
    fusion       0 automatic, 1 one step per launch, 2 two where supported,
                 3 as 2 with the row-accumulating D2Q37 kernel (FP32 rounding, not bitwise)  [0]
    graph_steps  replay steps from a HIP graph of this many steps (multiple of 4) [0]
    output       JSON-lines file for the records                 [standard output]
    checkpoint_out  write a checkpoint at the end                 [none]

Each record holds the step, wall time, MLUPS since the previous record and
the FP64 reductions of the library (mass, momentum, energy, kinetic energy,
enstrophy, smallest and largest density, largest speed, count of
non-finite populations).  A run that produces
non-finite populations stops at that record with "diverged": true.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

_KEYS = {"lattice", "grid", "storage", "model", "thermal", "rho0", "theta0", "tau", "scale", "init", "steps",
         "every", "fusion", "graph_steps", "output", "checkpoint_out"}
_INIT = {"rest": set(), "tgv": {"u0", "background"},
         "waves": {"shear_amp", "thermal_amp", "k", "kt", "background"},
         "double_shear_layer": {"u0", "sharpness", "delta"},
         "random_multimode": {"seed", "kmax", "umax"}, "checkpoint": {"path"}}
_DIMS = {"D2Q9": 2, "D3Q27": 3, "D2Q37": 2, "E9A": 2, "E9B": 2, "E9C": 2, "E9D": 2, "E7A": 2, "E7B": 2, "E7C": 2,
         "E7D": 2}


def load_config(source) -> dict:
    """Parse (path or dict) and validate a configuration; returns a normalised
    dict or raises ValueError naming the problem."""
    if isinstance(source, dict):
        cfg = dict(source)
    else:
        with open(source) as f:
            text = f.read()
        if str(source).endswith((".yaml", ".yml")):
            import yaml
            cfg = yaml.safe_load(text)
        else:
            cfg = json.loads(text)
        if not isinstance(cfg, dict):
            raise ValueError("the configuration must be a mapping")
    unknown = set(cfg) - _KEYS
    if unknown:
        raise ValueError(f"unknown keys: {sorted(unknown)}")
    init = dict(cfg.get("init") or {"kind": "rest"})
    kind = init.pop("kind", None)
    if kind not in _INIT:
        raise ValueError(f"init.kind must be one of {sorted(_INIT)}")
    bad = set(init) - _INIT[kind]
    if bad:
        raise ValueError(f"init '{kind}' does not take {sorted(bad)}")
    out = {"init": dict(init, kind=kind)}
    if "steps" not in cfg or not isinstance(cfg["steps"], int) or cfg["steps"] < 0:
        raise ValueError("steps must be a non-negative integer")
    out["steps"] = cfg["steps"]
    every = cfg.get("every", min(cfg["steps"], 100) or 1)
    if not isinstance(every, int) or every < 1:
        raise ValueError("every must be a positive integer")
    out["every"] = every
    for k, default in (("fusion", 0), ("graph_steps", 0)):
        v = cfg.get(k, default)
        if not isinstance(v, int):
            raise ValueError(f"{k} must be an integer")
        out[k] = v
    out["output"] = cfg.get("output")
    out["checkpoint_out"] = cfg.get("checkpoint_out")
    if kind == "checkpoint":
        if "path" not in init:
            raise ValueError("init 'checkpoint' needs a path")
        return out
    lattice = cfg.get("lattice")
    if lattice not in _DIMS:
        raise ValueError(f"lattice must be one of {sorted(_DIMS)}")
    grid = cfg.get("grid")
    if not isinstance(grid, (list, tuple)) or len(grid) not in (2, 3) or \
            not all(isinstance(g, int) and g >= 1 for g in grid):
        raise ValueError("grid must be [nx, ny] or [nx, ny, nz] with positive integers")
    D = _DIMS[lattice]
    grid = list(grid) + ([1] if len(grid) == 2 else [])
    if D == 2 and grid[2] != 1:
        raise ValueError(f"{lattice} is a 2D lattice: grid must be [nx, ny]")
    if D == 3 and len(cfg["grid"]) != 3:
        raise ValueError("D3Q27 needs grid [nx, ny, nz]")
    nx, ny, nz = grid
    if kind in ("tgv", "random_multimode") and D == 3 and not nx == ny == nz:
        raise ValueError(f"init '{kind}' needs a cubic grid")
    if kind in ("double_shear_layer", "random_multimode") and D == 2 and nx != ny:
        raise ValueError(f"init '{kind}' needs a square grid")
    if kind == "waves" and D != 2:
        raise ValueError("init 'waves' is two-dimensional")
    out.update(lattice=lattice, grid=grid, storage=cfg.get("storage", "f32"), model=cfg.get("model", "cm"),
               thermal=bool(cfg.get("thermal", False)), rho0=float(cfg.get("rho0", 1.0)),
               theta0=float(cfg.get("theta0", 1.0)), scale=cfg.get("scale"))
    tau = cfg.get("tau") or {}
    if not isinstance(tau, dict):
        raise ValueError("tau must map orders to relaxation times")
    try:
        out["tau"] = {int(k): float(v) for k, v in tau.items()}
    except (TypeError, ValueError):
        raise ValueError("tau must map integer orders to numbers") from None
    if any(k < 2 or k > 7 for k in out["tau"]):
        raise ValueError("tau orders are 2..7")
    return out


def _fields(cfg):
    from . import inputs
    nx, ny, nz = cfg["grid"]
    D = _DIMS[cfg["lattice"]]
    shape = (ny, nx) if D == 2 else (nz, ny, nx)
    init = dict(cfg["init"])
    kind = init.pop("kind")
    rho0, theta0 = cfg["rho0"], cfg["theta0"]
    theta = None
    if kind == "rest":
        rho, u = np.full(shape, rho0), np.zeros((D,) + shape)
    elif kind == "tgv":
        u0 = init.get("u0", 0.05)
        if D == 3:
            rho, u = inputs.tgv3d(nx, u0, rho0=rho0, background=tuple(init.get("background", (0.0,) * 3)))
        else:
            rho, u = inputs.tgv2d(nx, ny, u0, rho0=rho0)
            u = u + np.asarray(init.get("background", (0.0, 0.0)), float).reshape(2, 1, 1)
    elif kind == "waves":
        rho, u, theta = inputs.waves2d(nx, ny, init.get("shear_amp", 0.0), init.get("thermal_amp", 0.0),
                                       k=tuple(init.get("k", (1, 0))), kt=init.get("kt"),
                                       background=tuple(init.get("background", (0.0, 0.0))), rho0=rho0,
                                       theta0=theta0)
    elif kind == "double_shear_layer":
        rho, u, theta = inputs.double_shear_layer(nx, init.get("u0", 0.05), init.get("sharpness", 80.0),
                                                  init.get("delta", 0.05), rho0=rho0, theta0=theta0)
    else:   # random_multimode
        _, u = inputs.random_multimode(nx, init.get("seed", 0), init.get("kmax", 4), init.get("umax", 0.05), dim=D)
        rho = np.full(shape, rho0)
    return rho, u, theta


def make_context(cfg, stream=None):
    """The configured context with its initial state."""
    from . import checkpoint, cmlb
    if cfg["init"]["kind"] == "checkpoint":
        return checkpoint.load(cfg["init"]["path"], stream=stream)
    nx, ny, nz = cfg["grid"]
    D = _DIMS[cfg["lattice"]]
    shape = (ny, nx) if D == 2 else (nz, ny, nx)
    ctx = cmlb.Context(cfg["lattice"], shape, storage=cfg["storage"], model=cfg["model"], thermal=cfg["thermal"],
                       rho0=cfg["rho0"], theta0=cfg["theta0"], tau=cfg["tau"], scale=cfg["scale"], stream=stream)
    try:
        rho, u, theta = _fields(cfg)
        ctx.init_fields(rho, u, theta if cfg["thermal"] else None)
    except Exception:
        ctx.destroy()
        raise
    return ctx


def run(source, output=None, stream=None) -> list:
    """Run a configuration (path or dict); returns the records, which are
    also written as JSON lines to ``output`` (or the configured file, or
    standard output)."""
    cfg = load_config(source)
    output = output or cfg["output"]
    sink = open(output, "w") if output else sys.stdout
    records = []
    ctx = make_context(cfg, stream)
    try:
        ctx.set_step_fusion(cfg["fusion"])
        ctx.set_graph_steps(cfg["graph_steps"])
        nodes = ctx.nodes
        done, last = 0, time.perf_counter()
        start = last

        def record(k_steps):
            nonlocal last
            g = ctx.reduce(allow_unstable=True)
            now = time.perf_counter()
            rec = {"step": int(ctx.step_count()), "time_s": now - start,
                   "mlups": nodes * k_steps / max(now - last, 1e-12) / 1e6 if k_steps else None,
                   "mass": g["mass"], "momentum": [float(v) for v in g["momentum"]], "energy": g["energy"],
                   "ke": g["ke"], "enstrophy": g["enstrophy"], "rho_min": g["rho_min"], "rho_max": g["rho_max"],
                   "u_max": g["u_max"], "nonfinite": int(g["nonfinite"])}
            if g["nonfinite"]:
                rec["diverged"] = True
            last = now
            records.append(rec)
            sink.write(json.dumps(rec) + "\n")
            sink.flush()
            return not g["nonfinite"]

        ok = record(0)
        while ok and done < cfg["steps"]:
            k = min(cfg["every"], cfg["steps"] - done)
            ctx.step(k)
            done += k
            ok = record(k)
        if cfg["checkpoint_out"]:
            from . import checkpoint
            checkpoint.save(ctx, cfg["checkpoint_out"])
    finally:
        ctx.destroy()
        if sink is not sys.stdout:
            sink.close()
    return records


def main(argv=None):
    ap = argparse.ArgumentParser(description="Run a CM-MRT lattice Boltzmann configuration (JSON or YAML).")
    ap.add_argument("config")
    ap.add_argument("--out", default=None, help="JSON-lines output (default: the configured file or stdout)")
    args = ap.parse_args(argv)
    records = run(args.config, args.out)
    return 1 if records and records[-1].get("diverged") else 0


if __name__ == "__main__":
    sys.exit(main())
