"""Long-run studies on the HIP path (the library only; no oracle).

    python -m paper_1808_04406_amd.studies precision [--n 512] [--steps 5000]
    python -m paper_1808_04406_amd.studies thermal   [--n 1024] [--steps 5000]

precision: the D3Q27 Taylor-Green vortex at Re = 1e5 run in FP64, FP32, FP16
and BF16 storage from the same initial fields; kinetic-energy and enstrophy
histories (FP64 reductions) and their deviation from the FP64 run, which the
parity tests tie to the FP64 oracle.  Also the step throughput of each.

thermal: D2Q37 thermal CM-MRT with a decaying shear wave and an isobaric
thermal wave, background velocity 0 or 0.1 normal to k, Pr = 0.71 and 7;
viscosity and thermal diffusivity from exponential fits of the mode
amplitudes (u_perp and entropy), against the Chapman-Enskog values
nu = theta (tau_2 - 1/2), kappa = theta (tau_3 - 1/2) (Sec. III.A).

Results are written as JSON (``--out``) and summarised on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import cmlb, inputs


def _tgv_rates(tau):
    return {2: tau, 3: 1.0, 4: tau, 5: 1.0, 6: tau}


def precision(n=512, steps=5000, every=100, u0=0.05, re=1.0e5, storages=("f64", "f32", "f16", "bf16"),
              stream=None):
    import torch
    nu = u0 * (n / (2 * math.pi)) / re
    tau = 0.5 + 3.0 * nu
    rho, u = inputs.tgv3d(n, u0)
    d_rho = torch.from_numpy(rho.reshape(-1)).to("cuda")
    d_u = torch.from_numpy(u.reshape(-1)).to("cuda")
    del rho, u
    res = {"n": n, "steps": steps, "every": every, "u0": u0, "re": re, "tau": tau, "runs": {}}
    for st in storages:
        ctx = cmlb.Context("D3Q27", (n, n, n), storage=st, tau=_tgv_rates(tau), stream=stream)
        ctx.init_fields_device(d_rho, d_u)
        hist = {"t": [0], "ke": [], "enstrophy": [], "mass": [], "nonfinite": []}
        g = ctx.reduce()
        for k in ("ke", "enstrophy", "mass", "nonfinite"):
            hist[k].append(g[k])
        t_step = 0.0
        diverged_at = None
        for t in range(every, steps + 1, every):
            ctx.sync()
            t0 = time.perf_counter()
            ctx.step(every)
            ctx.sync()
            t_step += time.perf_counter() - t0
            g = ctx.reduce(allow_unstable=True)
            hist["t"].append(t)
            for k in ("ke", "enstrophy", "mass", "nonfinite"):
                hist[k].append(g[k])
            if g["nonfinite"]:
                diverged_at = t
                break
        ctx.destroy()
        torch.cuda.empty_cache()
        done = hist["t"][-1]
        hist["mlups"] = n ** 3 * done / t_step / 1e6
        hist["diverged_at"] = diverged_at
        res["runs"][st] = hist
        print(f"{st}: {done} steps, {hist['mlups']:.0f} MLUPS, KE/KE0 = {hist['ke'][-1] / hist['ke'][0]:.5f}, "
              f"diverged_at = {diverged_at}", flush=True)
    ref = res["runs"].get("f64")
    if ref:
        for st, h in res["runs"].items():
            m = min(len(h["ke"]), len(ref["ke"]))
            ke = np.array(h["ke"][:m]); ke_r = np.array(ref["ke"][:m])
            en = np.array(h["enstrophy"][:m]); en_r = np.array(ref["enstrophy"][:m])
            h["max_rel_err_ke"] = float(np.max(np.abs(ke - ke_r)) / ke_r[0])
            h["max_rel_err_enstrophy"] = float(np.max(np.abs(en - en_r)) / np.max(en_r))
            h["final_rel_err_ke"] = float(abs(ke[-1] - ke_r[-1]) / ke_r[-1])
            print(f"{st}: max |dKE|/KE0 = {h['max_rel_err_ke']:.3e}, max |dZ|/max Z = "
                  f"{h['max_rel_err_enstrophy']:.3e}", flush=True)
    return res


def _mode(field, kx):
    """(2/N) sum field exp(-i k x) for mode number kx along x."""
    ny, nx = field.shape
    x = np.arange(nx)
    return 2.0 * np.sum(field * np.exp(-2j * np.pi * kx * x / nx)[None, :]) / field.size


def _decay_rate(t, a):
    t = np.asarray(t, float)
    y = np.log(np.abs(np.asarray(a)))
    return -np.polyfit(t, y, 1)[0]


def thermal(n=1024, steps=5000, every=250, kx=4, tau2=0.6, prs=(0.71, 7.0), us=(0.0, 0.1), storage="f32",
            amp=0.01, model="cm", stream=None):
    info = cmlb.lattice_info("D2Q37")
    r = info["r"]
    res = {"n": n, "steps": steps, "kx": kx, "tau2": tau2, "storage": storage, "model": model, "runs": []}
    k_xi = 2 * math.pi * kx / n / r
    for pr in prs:
        tau3 = 0.5 + (tau2 - 0.5) / pr
        for u0 in us:
            ctx = cmlb.Context("D2Q37", (n, n), storage=storage, thermal=True, model=model,
                               tau={2: tau2, 3: tau3, 4: tau2}, stream=stream)
            rho, u, th = inputs.waves2d(n, n, shear_amp=amp / r, thermal_amp=amp, k=(kx, 0),
                                        background=(0.0, u0))
            ctx.init_fields(rho, u, th)
            ts, av, at = [], [], []
            t0 = time.perf_counter()
            for t in range(0, steps + 1, every):
                if t:
                    ctx.step(every)
                g_rho, g_u, g_th = ctx.get_moments()
                s = np.log(g_th * g_rho ** (1.0 - 2.0))   # entropy, c_v = 1, gamma = 2
                ts.append(t)
                av.append(abs(_mode(g_u[1] - u0, kx)))
                at.append(abs(_mode(s, kx)))
            wall = time.perf_counter() - t0
            ctx.destroy()
            nu_th, ka_th = 1.0 * (tau2 - 0.5), 1.0 * (tau3 - 0.5)
            gam, cs = 2.0, math.sqrt(2.0)
            lam = 1.0 + (gam - 3.0) * pr
            pe = cs / (ka_th * k_xi)
            skip = max(1, len(ts) // 10)
            nu_m = _decay_rate(ts[skip:], av[skip:]) / k_xi ** 2
            ka_m = _decay_rate(ts[skip:], at[skip:]) / (k_xi ** 2 * (1 + (gam - 1) * lam / pe ** 2))
            run = {"pr": pr, "u0": u0, "tau3": tau3, "nu_theory": nu_th, "kappa_theory": ka_th,
                   "nu_measured": nu_m, "kappa_measured": ka_m, "nu_rel_err": nu_m / nu_th - 1,
                   "kappa_rel_err": ka_m / ka_th - 1, "wall_s": wall}
            res["runs"].append(run)
            print(f"Pr={pr} u0={u0}: nu err {run['nu_rel_err']:+.3e}, kappa err {run['kappa_rel_err']:+.3e}",
                  flush=True)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["precision", "thermal"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--model", default="cm")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        if a.study == "precision":
            res = precision(n=a.n or 512, steps=a.steps, every=a.every or 100, stream=stream)
        else:
            res = thermal(n=a.n or 1024, steps=a.steps, every=a.every or 250, storage=a.storage, model=a.model,
                          stream=stream)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
