"""Checkpoint and resume of a simulation context.

A checkpoint file holds a small JSON header and the stored populations as
they sit in device memory (deviations in the storage type, structure of
arrays), so that a resumed run continues bitwise as if it had never
stopped.  The header records what the context needs to be rebuilt: lattice,
grid, storage, collision model, thermal flag, rho0, theta0, the relaxation
times and storage scales in use, the step counter, the state's row pitch
and plane stride, and the learned closure (FP32 master weights, input
scales, switches) when one is loaded.  Version 2 pads large population
planes (cmlb.h, layout of the state); a file whose layout differs from the
rebuilt context's is refused.

Layout: b"CMLBCKPT", uint32 version, uint64 header length, header (UTF-8
JSON), population bytes.
"""
from __future__ import annotations

import json
import struct

import numpy as np

from . import cmlb

MAGIC = b"CMLBCKPT"
VERSION = 2

_NAMES = {
    "lattice": {v: k for k, v in reversed(list(cmlb.LATTICES.items()))},   # the first name of an alias
    "storage": {v: k for k, v in cmlb.STORAGES.items()},
    "model": {v: k for k, v in cmlb.MODELS.items()},
}


def save(ctx, path):
    """Write the context's current state and configuration to path (synchronises)."""
    import torch
    p = ctx.params
    _, nbytes, _ = ctx.state()
    buf = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{p.device}")
    ctx.store_state_device(buf)
    ctx.sync()
    header = {
        "lattice": _NAMES["lattice"][p.lattice],
        "shape": list(ctx.shape),
        "storage": _NAMES["storage"][p.storage],
        "model": _NAMES["model"][p.model],
        "thermal": bool(p.thermal),
        "rho0": p.rho0,
        "theta0": p.theta0,
        "tau": {str(n): float(t) for n, t in enumerate(ctx.get_tau()) if n >= 2 and t != 0.0},
        "scale": [float(s) for s in ctx.get_scale()],
        "steps": int(ctx.step_count()),
        "bytes": int(nbytes),
        "layout": list(cmlb.state_layout(_NAMES["lattice"][p.lattice], ctx.shape, _NAMES["storage"][p.storage])),
        "closure": None,
    }
    if ctx._closure is not None:
        header["closure"] = {"params": [float(v) for v in ctx.closure_get()],
                             "sigma": [float(v) for v in ctx._closure["sigma"]],
                             "enabled": ctx._closure["enabled"], "tie_even": ctx._closure["tie_even"]}
    hb = json.dumps(header).encode()
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<IQ", VERSION, len(hb)))
        f.write(hb)
        f.write(buf.cpu().numpy().tobytes())


def read_header(path):
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a checkpoint")
        version, n = struct.unpack("<IQ", f.read(12))
        if version != VERSION:
            raise ValueError(f"{path}: checkpoint version {version}, expected {VERSION}")
        return json.loads(f.read(n).decode()), 20 + n


def load(path, stream=None, device=0):
    """Rebuild a context from a checkpoint; its state, step counter, relaxation
    times and closure are those saved."""
    import torch
    h, offset = read_header(path)
    layout = list(cmlb.state_layout(h["lattice"], tuple(h["shape"]), h["storage"]))
    if h.get("layout") != layout:
        raise ValueError(f"{path}: state layout (pitch, plane) {h.get('layout')}, this library uses {layout}")
    ctx = cmlb.Context(h["lattice"], tuple(h["shape"]), storage=h["storage"], model=h["model"],
                       thermal=h["thermal"], rho0=h["rho0"], theta0=h["theta0"],
                       tau={int(k): v for k, v in h["tau"].items()}, scale=h["scale"], device=device,
                       stream=stream)
    try:
        data = np.fromfile(path, dtype=np.uint8, offset=offset)
        if data.size != h["bytes"]:
            raise ValueError(f"{path}: {data.size} population bytes, expected {h['bytes']}")
        buf = torch.from_numpy(data).to(f"cuda:{device}")
        ctx.load_state_device(buf)
        ctx.sync()
        ctx.set_step_count(h["steps"])
        if h["closure"] is not None:
            c = h["closure"]
            ctx.closure_load(np.array(c["params"], np.float32), np.array(c["sigma"], np.float32))
            ctx.closure_tie_even(c["tie_even"])
            ctx.closure_enable(c["enabled"])
    except Exception:
        ctx.destroy()
        raise
    return ctx
