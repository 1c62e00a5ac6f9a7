"""Benchmark: CM-MRT fused stream + collide, D3Q27 256^3 FP32, one MI355X.

Workload: 3D Taylor-Green vortex on a 256^3 periodic grid, u0 = 0.05,
Re = 1600 with L = N / (2 pi) (nu = u0 L / Re, tau_2 = 1/2 + 3 nu).  Odd
central-moment orders (3, 5) relax at rate 1; the even orders 4 and 6 relax
at omega_2, because with rate 1 there the linearised D3Q27 update has growing
modes at this tau_2 (spectral radius 1.12 at rest), and the run diverges.
Populations are FP32 deviations f_i - w_i rho0 in HBM (27 planes of 256^3).
A step is one launch of the fused pull-stream + collide kernel over every
node; the rates are kernel arguments, so the work per step does not depend
on them.

Prints one JSON line: MLUPS (million lattice-node updates per second, whole
job), ms per step, the kernel's HBM roofline (algorithmic bytes 2 Q s = 216 B
per node update against MI355X's 8 TB/s, and the bytes the two-step launch
actually moves against 8 TB/s and against the measured copy rate), and the
FP64 CPU oracle timed for ten steps of the same 256^3 workload on the host
cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 256
U0 = 0.05
RE = 1600.0
Q = 27
STORAGE_BYTES = 4
PEAK_HBM_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 << 20   # MI355X last-level (MALL) cache
KERNEL = "k_step2_tp<kF32>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_d3q27_256_f32.json")
KERNEL_SOURCES = ["paper_1808_04406_amd/csrc/step_tp2.hip", "paper_1808_04406_amd/csrc/collide_tp.hpp",
                  "paper_1808_04406_amd/csrc/common.hpp"]
# The learned-closure step is bound by vector-ALU issue; its instruction count
# per launch comes from a committed rocprofv3 counter summary.
VALU_FILE = os.path.join(ROOT, "profiles", "valu_k_step_closure_d3q27_128_f32.json")
CLOSURE_SOURCES = ["paper_1808_04406_amd/csrc/kernels_closure.hip", "paper_1808_04406_amd/csrc/closure.hpp",
                   "paper_1808_04406_amd/csrc/collide_tp.hpp", "paper_1808_04406_amd/csrc/common.hpp"]
# Vector-ALU issue peak in lane-instructions per second: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz (a wave64 instruction occupies a SIMD for 4 cycles;
# packed FP32 is not used).
PEAK_VALU_TLANE = 256 * 4 * 16 * 2.4e9 / 1e12
STORAGE_TAG = {"f64": "kF64", "f32": "kF32", "f16": "kF16", "bf16": "kBF16"}


def tau_shear(n=N, u0=U0, re=RE):
    nu = u0 * (n / (2.0 * math.pi)) / re
    return 0.5 + 3.0 * nu


def rates(tau):
    """tau by central-moment order: odd orders at 1, even orders at tau_2."""
    return {2: tau, 3: 1.0, 4: tau, 5: 1.0, 6: tau}


def kernel_source_hash(sources=None):
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_valu():
    """VALU wave-instructions per launch of the closure step (128^3), or None
    if the summary is missing or was taken on a different kernel source."""
    try:
        with open(VALU_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash(CLOSURE_SOURCES):
        return None
    return t.get("valu_wave_instructions_per_launch")


def measured_traffic(bytes_per_launch_alg):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if it is missing or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(tau, n=N, steps=10):
    """FP64 oracle (plain C, OpenMP) on the benchmark's own grid: the same
    256^3 Taylor-Green vortex and rates for `steps` steps after one warm-up
    step, timed on the host cores and reported in MLUPS (about 70-80 s on
    16 host cores).  A one-core figure is taken on a 64^3 sample of the same
    workload (a 256^3 step takes about 100 s on one core)."""
    import numpy as np
    import oracle
    from paper_1808_04406_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    cfg = oracle.Cfg(lattice="D3Q27", tau=rates(tau))
    rho, u = inputs.tgv3d(n, U0)
    S = oracle.init_equilibrium(cfg, rho, u, threads=threads)
    oracle.run(cfg, S, 1, threads=threads)
    t0 = time.perf_counter()
    oracle.run(cfg, S, steps, threads=threads)
    dt = time.perf_counter() - t0
    assert np.isfinite(S).all()
    o_rho, o_u, _ = oracle.moments("D3Q27", S)
    del S
    # one core, on a 64^3 sample of the same workload
    n1 = 64
    r1, u1 = inputs.tgv3d(n1, U0)
    S1 = oracle.init_equilibrium(cfg, r1, u1, threads=threads)
    oracle.run(cfg, S1, 1, threads=1)
    t0 = time.perf_counter()
    oracle.run(cfg, S1, 2, threads=1)
    one_core = n1 ** 3 * 2 / (time.perf_counter() - t0) / 1e6
    ref = {"n": n, "steps": 1 + steps, "rho0": rho, "u0": u, "rho": o_rho, "u": o_u}
    return {"value": n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"D3Q27 TGV {n}^3 (the benchmark grid, same u0 and rates), {steps} steps after 1 warm-up "
                      f"step, FP64, {dt:.1f} s", "one_core_MLUPS": round(one_core, 3),
            "one_core_sample": f"D3Q27 TGV {n1}^3, 2 steps after 1 warm-up step, 1 thread",
            "cpu_model": _cpu_model()}, ref


def error_vs_oracle(cmlb, tau, ref):
    """The benchmarked path (FP32 storage, two steps per launch) on the CPU
    baseline's grid, for as many steps as the oracle took there, against the
    oracle's final moments."""
    import numpy as np
    n, steps = ref["n"], ref["steps"]
    ctx = cmlb.Context("D3Q27", (n, n, n), storage="f32", tau=rates(tau))
    try:
        ctx.set_step_fusion(2)
        ctx.init_fields(ref["rho0"], ref["u0"])
        ctx.step(steps)
        g_rho, g_u, _ = ctx.get_moments()
    finally:
        ctx.destroy()
    return {"max_abs_du_over_u0": float(np.abs(g_u - ref["u"]).max() / U0),
            "max_abs_drho": float(np.abs(g_rho - ref["rho"]).max()),
            "steps": steps,
            "sample": f"D3Q27 TGV {n}^3 (same u0 and rates), FP32 storage, two steps per launch, {steps} steps, "
                      "against the FP64 oracle run of the CPU baseline"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def copy_bandwidth(torch, nbytes=4 << 30, reps=40):
    """Device-to-device copy bandwidth (read + write bytes / time) with torch."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--steps-per-launch", type=int, default=2, choices=[1, 2, 3],
                    help="2: pairs of steps in one launch where supported (D3Q27 FP32/FP64, D2Q37 FP32; default); "
                         "1: one launch per step; 3: as 2, with the D2Q37 kernel that accumulates the second "
                         "step's moments row by row (equal to two single steps to FP32 rounding, not bitwise)")
    ap.add_argument("--workload", default="tgv256_f32", choices=sorted(WORKLOADS),
                    help="default: the D3Q27 256^3 FP32 Taylor-Green benchmark; others report the precision "
                         "form and the thermal lattice with the same JSON fields")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "domain decomposition is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1808_04406_amd import cmlb, inputs

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # default priority; all work of the run is ordered on it
    with torch.cuda.stream(stream):
        out = run(torch, cmlb, inputs, stream, args)
    if not args.no_cpu_baseline and args.workload == "tgv256_f32":
        out["cpu_baseline"], ref = cpu_baseline(out["config"]["tau_shear"])
        out["error_vs_oracle"] = error_vs_oracle(cmlb, out["config"]["tau_shear"], ref)
    print(json.dumps(out), flush=True)


WORKLOADS = {
    # name: (lattice, grid, storage, description)
    "tgv256_f32": ("D3Q27", (256, 256, 256), "f32", "D3Q27 CM-MRT 256^3 periodic 3D Taylor-Green vortex, u0=0.05, "
                   "Re=1600, FP32 deviation storage"),
    "tgv512_f32": ("D3Q27", (512, 512, 512), "f32", "D3Q27 CM-MRT 512^3 TGV, u0=0.05, Re=1e5, FP32 storage"),
    "tgv512_f16": ("D3Q27", (512, 512, 512), "f16", "D3Q27 CM-MRT 512^3 TGV, u0=0.05, Re=1e5, FP16 scaled storage"),
    "tgv512_bf16": ("D3Q27", (512, 512, 512), "bf16", "D3Q27 CM-MRT 512^3 TGV, u0=0.05, Re=1e5, BF16 storage"),
    "tgv512_f64": ("D3Q27", (512, 512, 512), "f64", "D3Q27 CM-MRT 512^3 TGV, u0=0.05, Re=1e5, FP64 storage"),
    "tgv128_f32": ("D3Q27", (128, 128, 128), "f32", "D3Q27 CM-MRT 128^3 TGV, u0=0.05, Re=1e5, FP32 storage"),
    "tgv128_closure_f32": ("D3Q27", (128, 128, 128), "f32", "D3Q27 CM-MRT 128^3 TGV, u0=0.05, Re=1e5, FP32 "
                           "storage, learned closure (per-node 27-32-32-4 MLP on the matrix cores) setting the "
                           "rates of orders 3..6"),
    "waves1024_f32": ("D2Q37", (1024, 1024), "f32", "D2Q37 thermal CM-MRT 1024^2, shear + thermal waves "
                      "(amplitude 0.01), tau_2=0.6, Pr=0.71, background 0.1, FP32 storage"),
    "waves2048_f32": ("D2Q37", (2048, 2048), "f32", "D2Q37 thermal CM-MRT 2048^2, shear + thermal waves "
                      "(amplitude 0.01), tau_2=0.6, Pr=0.71, background 0.1, FP32 storage"),
    "waves2048_rawmrt_f32": ("D2Q37", (2048, 2048), "f32", "D2Q37 thermal raw-moment MRT 2048^2, shear + thermal "
                             "waves (amplitude 0.01), tau_2=0.6, Pr=0.71, background 0.1, FP32 storage"),
    "waves2048_regbgk_f32": ("D2Q37", (2048, 2048), "f32", "D2Q37 thermal regularised BGK 2048^2, shear + thermal "
                             "waves (amplitude 0.01), tau=0.6, background 0.1, FP32 storage"),
}
WORKLOAD_MODEL = {"waves2048_rawmrt_f32": "raw_mrt", "waves2048_regbgk_f32": "reg_bgk"}
MODEL_TAG = {"cm": "kCM", "raw_mrt": "kRawMRT", "reg_bgk": "kCM"}
QS = {"D3Q27": 27, "D2Q37": 37}
SBYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


def setup_workload(name, torch, cmlb, inputs, stream):
    """Context, external buffers and device fields of a workload."""
    lattice, shape, storage, desc = WORKLOADS[name]
    q, sb = QS[lattice], SBYTES[storage]
    nodes = 1
    for s_ in shape:
        nodes *= s_
    nbytes = cmlb.state_bytes(lattice, shape, storage)   # x-rows padded to the library's pitch
    bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
    theta = None
    if lattice == "D3Q27":
        n = shape[0]
        re = RE if n == 256 else 1.0e5
        tau = tau_shear(n, U0, re)
        taus = rates(tau)
        ctx = cmlb.Context("D3Q27", shape, storage=storage, tau=taus, external=bufs, stream=stream)
        if name.endswith("closure_f32"):
            import numpy as np
            params = 0.3 * np.random.default_rng(0).normal(size=cmlb.CLOSURE_NPARAM)
            ctx.closure_load(params, np.full(27, 0.01))
            ctx.closure_tie_even(True)   # orders 4, 6 at omega_2: stable as tau_2 -> 1/2
            ctx.closure_enable(True)
        rho, u = inputs.tgv3d(n, U0)
    else:
        n = shape[0]
        tau2, pr = 0.6, 0.71
        taus = {2: tau2, 3: 0.5 + (tau2 - 0.5) / pr, 4: tau2}
        ctx = cmlb.Context("D2Q37", shape, storage=storage, thermal=True, model=WORKLOAD_MODEL.get(name, "cm"),
                           tau=taus, external=bufs, stream=stream)
        rho, u, theta = inputs.waves2d(n, n, shear_amp=0.01, thermal_amp=0.01, k=(1, 0), background=(0.0, 0.1))
    d = [torch.from_numpy(a.reshape(-1)).to("cuda") for a in (rho, u)]
    d_th = None if theta is None else torch.from_numpy(theta.reshape(-1)).to("cuda")
    ctx.init_fields_device(d[0], d[1], d_th)
    torch.cuda.synchronize()
    return ctx, bufs, float(rho.sum()), taus, desc, nodes, q, sb


def run(torch, cmlb, inputs, stream, args):
    ctx, bufs, mass0, taus, desc, nodes, q, sb = setup_workload(args.workload, torch, cmlb, inputs, stream)
    lattice, shape, storage, _ = WORKLOADS[args.workload]
    closure = args.workload.endswith("closure_f32")
    # pairs of steps run as one launch (intermediate state on chip): D3Q27
    # FP32 and FP64, D2Q37 FP32
    fused = (storage == "f32" or (lattice == "D3Q27" and storage == "f64")) and not closure \
        and args.steps_per_launch >= 2
    ctx.set_step_fusion(args.steps_per_launch)

    # Achievable ceilings, measured before the steps: torch's device copy
    # (also the reference of the HBM counter calibration), and the library's
    # streaming copy of one 4 GiB plane and of 27 planes of 2^24 FP32 values
    # (the step's access pattern and state size; planes whose size is not a
    # multiple of 128 B copy markedly slower).  About 0.2 s of copies: a
    # device fresh from idle runs its first ~10 ms of work at lower clocks,
    # and this way the timed steps do not start there.
    torch_copy_gbs = copy_bandwidth(torch, reps=40)
    copy1_gbs = cmlb.copy_bandwidth(4 << 30, planes=1, reps=40)
    copy_gbs = cmlb.copy_bandwidth(27 * 4 * (1 << 24), planes=27, reps=40)
    torch.cuda.synchronize()

    ctx.step(args.warmup)
    torch.cuda.synchronize()

    # the K timed steps in five segments with events between them (per-launch
    # time of each segment; their median is reported beside the average)
    def n_launches(m):
        return (m // 2 + m % 2) if fused else m

    base = args.steps // 5
    if fused:
        base -= base % 2
    sizes = [base] * 4 + [args.steps - 4 * base]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k, m in enumerate(sizes):
        ctx.step(m)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ev0, ev1 = evs[0], evs[-1]
    kernel_ms = ev0.elapsed_time(ev1) / max(n_launches(args.steps), 1)
    seg_ms = [evs[k].elapsed_time(evs[k + 1]) / n_launches(m) for k, m in enumerate(sizes) if n_launches(m) > 0]
    kernel_ms_median = sorted(seg_ms)[len(seg_ms) // 2] if seg_ms else kernel_ms
    updates_per_launch = 2 if fused else 1

    g = ctx.reduce()
    assert g["nonfinite"] == 0, "simulation diverged"
    assert abs(g["mass"] - mass0) / mass0 < 1e-5, "mass not conserved"
    ctx.destroy()
    del bufs
    torch.cuda.empty_cache()


    value = nodes * args.steps / wall / 1e6
    per_node = 2 * q * sb
    # algorithmic bytes per launch: 2 Q s per node update (each population read
    # and written once) x the node updates of one launch
    alg_bytes = per_node * nodes * updates_per_launch
    achieved = per_node * nodes * args.steps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    traffic = measured_traffic(alg_bytes) if (args.workload == "tgv256_f32" and fused) else None
    if fused and lattice == "D3Q27":
        kernel = "k_step2_tp<%s>" % STORAGE_TAG[storage]
    elif fused:
        kernel = "k_step2_d37%s<%s>" % ("_acc" if args.steps_per_launch == 3 else "",
                                        MODEL_TAG[WORKLOAD_MODEL.get(args.workload, "cm")])
    elif lattice == "D3Q27":
        kernel = "k_step_tp<3, %s>" % STORAGE_TAG[storage]
    else:
        kernel = "k_step_d37<%s, %s>" % (STORAGE_TAG[storage], MODEL_TAG[WORKLOAD_MODEL.get(args.workload, "cm")])
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic}
    # both population buffers inside the 256 MB Infinity Cache: the rate may
    # then exceed what HBM alone allows
    state_bytes = cmlb.state_bytes(lattice, shape, storage)
    roof["fits_infinity_cache"] = 2 * state_bytes <= INFINITY_CACHE_BYTES
    if traffic is not None:
        # bytes the launch actually moves (rocprofv3 counters) per unit time
        moved = traffic / (kernel_ms * 1e-3) / 1e9
        roof.update(traffic_ratio=round(traffic / alg_bytes, 4), moved_GBps=round(moved, 1),
                    moved_frac=round(moved / PEAK_HBM_GBS, 4), moved_frac_of_copy=round(moved / copy_gbs, 4))
    if fused:
        roof["note"] = ("two node updates per launch with the intermediate state on chip: achieved counts "
                        "2 Q s bytes per node update, so frac can exceed 1; the bound that binds this kernel "
                        "is the HBM traffic it actually makes: moved_GBps = traffic / kernel time, against "
                        "8 TB/s (moved_frac) and against the measured 27-plane copy (moved_frac_of_copy)")
    if closure:
        kernel = "k_step_closure"
        valu = measured_valu()
        if valu is not None:
            lane_rate = valu * 64 / (kernel_ms * 1e-3) / 1e12
            roof = {"bound": "alu", "achieved": round(lane_rate, 2), "peak": PEAK_VALU_TLANE,
                    "unit": "T lane-instructions/s (VALU)", "frac": round(lane_rate / PEAK_VALU_TLANE, 4),
                    "traffic": None, "valu_wave_instructions_per_launch": valu,
                    "hbm_GBps": round(achieved, 1), "hbm_frac": round(achieved / PEAK_HBM_GBS, 4)}
    out = {
        "metric": "MLUPS of CM-MRT stream+collide, % HBM roofline; error vs FP64 oracle",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / max(args.steps, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": storage,
        "data": "synthetic",
        "config": {"workload": desc, "lattice": lattice, "grid": list(shape), "storage": storage,
                   "tau_shear": taus[2], "tau_by_order": {str(k): v for k, v in taus.items()},
                   "parallelism": "single GPU"},
        "roofline": dict(roof, kernel=kernel, kernel_ms=round(kernel_ms, 5),
                         kernel_ms_median_of_5_segments=round(kernel_ms_median, 5), steps_per_launch=updates_per_launch,
                         bytes_per_node_update=per_node, algorithmic_bytes_per_launch=alg_bytes,
                         copy_GBps=round(copy_gbs, 1), frac_of_copy=round(achieved / copy_gbs, 4),
                         copy_note="copy_GBps: streaming copy of 27 FP32 planes (the step's pattern); "
                                   "copy1_GBps: one plane; torch_copy_GBps: torch's device copy",
                         copy1_GBps=round(copy1_gbs, 1), torch_copy_GBps=round(torch_copy_gbs, 1)),
    }
    return out


if __name__ == "__main__":
    main()
