"""Long-run studies on the HIP path (the library only; no oracle).

    python -m paper_1808_04406_amd.studies precision [--n 512] [--steps 5000]
    python -m paper_1808_04406_amd.studies thermal   [--n 1024] [--steps 5000]
    python -m paper_1808_04406_amd.studies closure   [--n 512]

precision: the D3Q27 Taylor-Green vortex at Re = 1e5 run in FP64, FP32, FP16
and BF16 storage from the same initial fields; kinetic-energy and enstrophy
histories (FP64 reductions) and their deviation from the FP64 run, which the
parity tests tie to the FP64 oracle.  Also the step throughput of each.

thermal: D2Q37 thermal CM-MRT with a decaying shear wave and an isobaric
thermal wave, background velocity 0 or 0.1 normal to k, Pr = 0.71 and 7;
viscosity and thermal diffusivity from exponential fits of the mode
amplitudes (u_perp and entropy), against the Chapman-Enskog values
nu = theta (tau_2 - 1/2), kappa = theta (tau_3 - 1/2) (Sec. III.A).

closure: the learned closure (rates of orders 3..6 from a per-node network),
trained on the GPU on box-filtered fine runs, its objective on held-out data
against networks with fixed rates, and a coarse Taylor-Green rollout against
the filtered fine run.

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


def _logit_rate(omega):
    """Network logit that gives the rate omega = 0.5 + 1.45 sigmoid(z)."""
    q = (np.asarray(omega, float) - 0.5) / 1.45
    return np.log(q / (1.0 - q))


def _constant_net(omegas, seed=0, scale=0.05):
    """Parameters whose output rates are the constants omegas (W3 = 0)."""
    p = scale * np.random.default_rng(seed).normal(size=cmlb.CLOSURE_NPARAM)
    p[1952:2080] = 0.0
    p[2080:] = _logit_rate(omegas)
    return p


def _input_scales(state, n, samples=20000, seed=0):
    """Standard deviation of the non-equilibrium central moments of the pulled
    coarse states (network input scales sigma_p; 1 for the conserved orders).
    Central moments follow their definition, sum_i f_i prod_d (e_{i,d} - u_d)^{p_d}."""
    info = cmlb.lattice_info("D3Q27")
    e, w = info["e"], info["w"]
    rng = np.random.default_rng(seed)
    f = state.reshape(27, n, n, n)
    idx = rng.integers(0, n, size=(samples, 3))  # x, y, z
    fin = np.stack([f[i, (idx[:, 2] - e[i, 2]) % n, (idx[:, 1] - e[i, 1]) % n, (idx[:, 0] - e[i, 0]) % n]
                    for i in range(27)], 1) + w                                     # [sample, i]
    rho = fin.sum(1)
    u = fin @ e / rho[:, None]
    x = np.zeros((samples, 27))
    m = (1.0, 0.0, 1.0 / 3.0)
    for p in range(27):
        pd = (p % 3, (p // 3) % 3, p // 9)
        c = np.prod([(e[None, :, d] - u[:, d, None]) ** pd[d] for d in range(3)], axis=0)
        kap = (fin * c).sum(1)
        keq = rho * m[pd[0]] * m[pd[1]] * m[pd[2]]
        x[:, p] = (kap - keq) / rho
    sig = x.std(0)
    orders = np.array([p % 3 + (p // 3) % 3 + p // 9 for p in range(27)])
    sig[orders < 2] = 1.0
    return np.maximum(sig, 1e-12)


def closure(n_fine=512, factor=4, seeds=tuple(range(8)), held_out=(7,), spinup=400, pairs_per_seed=3, gap=400,
            train_steps=600, lr=2e-3, tgv_coarse_steps=1250, every=50, stream=None):
    """Learned closure: data from fine random multi-mode runs at Re = 1e5
    (acoustic scaling, coarse time step = factor fine steps), box-filtered;
    training on the GPU; gain on held-out seeds against fixed rates; TGV
    rollout at the coarse size against the filtered fine run."""
    import torch
    u0, re = 0.05, 1.0e5
    tau_f = 0.5 + 3.0 * u0 * (n_fine / (2 * math.pi)) / re
    tau_c = 0.5 + (tau_f - 0.5) / factor
    nc = n_fine // factor
    nodes_c = nc ** 3
    res = {"n_fine": n_fine, "n_coarse": nc, "tau_fine": tau_f, "tau_coarse": tau_c, "seeds": list(seeds),
           "held_out": list(held_out)}
    # 1. data
    data = {}
    t0 = time.perf_counter()
    for seed in seeds:
        rho, u = inputs.random_multimode(n_fine, seed, kmax=4, umax=u0)
        fine = cmlb.Context("D3Q27", (n_fine,) * 3, storage="f32", tau=_tgv_rates(tau_f), stream=stream)
        fine.init_fields(rho, u)
        del rho, u
        fine.step(spinup)
        pairs = []
        for k in range(pairs_per_seed):
            a = torch.empty(27 * nodes_c, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            fine.box_filter(factor, a)
            fine.step(factor)
            fine.box_filter(factor, b)
            pairs.append((a, b))
            if k + 1 < pairs_per_seed:
                fine.step(gap - factor)
        g = fine.reduce()
        fine.destroy()
        data[seed] = pairs
        print(f"data seed {seed}: {pairs_per_seed} pairs, fine KE {g['ke']:.4e}, {time.perf_counter() - t0:.0f} s",
              flush=True)
    torch.cuda.synchronize()
    train = [p for s_ in seeds if s_ not in held_out for p in data[s_]]
    test = [p for s_ in held_out for p in data[s_]]
    sigma = _input_scales(train[0][0].cpu().numpy(), nc)
    res["sigma"] = sigma.tolist()
    # 2. training (orders 4 and 6 tied to omega_2, the network sets orders 3 and 5)
    ctx = cmlb.Context("D3Q27", (nc,) * 3, storage="f32", tau={2: tau_c}, stream=stream)
    fixed1 = _constant_net([1.0, 1.0, 1.0, 1.0])
    odd1 = _constant_net([1.0, 1.0, 1.0, 1.0], seed=1, scale=0.1)

    def objective(params, pairs, tie):
        ctx.closure_load(params, sigma)
        ctx.closure_tie_even(tie)
        return float(np.mean([ctx.closure_objective(a, b, grad=False) for a, b in pairs]))

    res["objective_fixed_rate1_test"] = objective(fixed1, test, False)
    res["objective_stable_fixed_test"] = objective(odd1, test, True)
    ctx.closure_load(odd1, sigma)
    ctx.closure_tie_even(True)
    hist = []
    t1 = time.perf_counter()
    for it in range(train_steps):
        a, b = train[it % len(train)]
        hist.append(ctx.closure_train_step(a, b, lr * (1.0 - it / train_steps)))
        if it % 50 == 0:
            print(f"train step {it}: objective {hist[-1]:.4e}", flush=True)
    torch.cuda.synchronize()
    res["train_seconds"] = time.perf_counter() - t1
    res["train_history"] = hist
    learned = ctx.closure_get().astype(np.float64)
    res["params"] = learned.tolist()
    res["objective_learned_train"] = objective(learned, train, True)
    res["objective_learned_test"] = objective(learned, test, True)
    res["objective_stable_fixed_train"] = objective(odd1, train, True)
    res["gain_vs_rate1"] = res["objective_fixed_rate1_test"] / res["objective_learned_test"]
    res["gain_vs_stable_fixed"] = res["objective_stable_fixed_test"] / res["objective_learned_test"]
    print(f"held-out objective: fixed rates 1 {res['objective_fixed_rate1_test']:.4e}, stable fixed "
          f"{res['objective_stable_fixed_test']:.4e}, learned {res['objective_learned_test']:.4e}", flush=True)
    del data, train, test
    torch.cuda.empty_cache()
    # 3. Taylor-Green rollout: coarse runs from the filtered fine initial state
    rho, u = inputs.tgv3d(n_fine, u0)
    fine = cmlb.Context("D3Q27", (n_fine,) * 3, storage="f32", tau=_tgv_rates(tau_f), stream=stream)
    fine.init_fields(rho, u)
    del rho, u
    buf = torch.empty(27 * nodes_c, dtype=torch.float32, device="cuda")
    probe = cmlb.Context("D3Q27", (nc,) * 3, storage="f32", tau={2: tau_c}, stream=stream)
    runs = {"learned": cmlb.Context("D3Q27", (nc,) * 3, storage="f32", tau={2: tau_c}, stream=stream),
            "fixed_odd1_even_omega2": cmlb.Context("D3Q27", (nc,) * 3, storage="f32", tau=_tgv_rates(tau_c),
                                                   stream=stream),
            "fixed_rate1": cmlb.Context("D3Q27", (nc,) * 3, storage="f32", tau={2: tau_c}, stream=stream)}
    runs["learned"].closure_load(learned, sigma)
    runs["learned"].closure_tie_even(True)
    runs["learned"].closure_enable(True)
    fine.box_filter(factor, buf)
    for c in runs.values():
        c.load_state_device(buf)
    hist = {k: {"ke": [], "enstrophy": [], "nonfinite": []} for k in list(runs) + ["filtered_fine"]}
    tt = []
    for t in range(0, tgv_coarse_steps + 1, every):
        if t:
            fine.step(every * factor)
            for c in runs.values():
                c.step(every)
        fine.box_filter(factor, buf)
        probe.load_state_device(buf)
        items = [("filtered_fine", probe)] + list(runs.items())
        for name, c in items:
            g = c.reduce(allow_unstable=True)
            for k in ("ke", "enstrophy", "nonfinite"):
                hist[name][k].append(g[k])
        tt.append(t)
    for c in list(runs.values()) + [probe, fine]:
        c.destroy()
    ref_ke = np.array(hist["filtered_fine"]["ke"])
    ref_z = np.array(hist["filtered_fine"]["enstrophy"])
    res["tgv"] = {"t_coarse": tt, "histories": hist}
    for name in runs:
        ke = np.array(hist[name]["ke"])
        z = np.array(hist[name]["enstrophy"])
        ok = np.isfinite(ke) & np.isfinite(z) & (np.array(hist[name]["nonfinite"]) == 0)
        m = ok.sum()
        res["tgv"][name] = {"stable_samples": int(m), "of": len(tt),
                            "max_rel_err_ke": float(np.max(np.abs(ke[ok] - ref_ke[ok]) / ref_ke[0])) if m else None,
                            "max_rel_err_enstrophy": float(np.max(np.abs(z[ok] - ref_z[ok]) / ref_z[ok].max()))
                            if m else None}
        print(f"TGV {name}: {res['tgv'][name]}", flush=True)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["precision", "thermal", "closure"])
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
        elif a.study == "closure":
            res = closure(n_fine=a.n or 512, stream=stream)
        else:
            res = thermal(n=a.n or 1024, steps=a.steps, every=a.every or 250, storage=a.storage, model=a.model,
                          stream=stream)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
