"""Throughput benchmark of the C-dTWA hot path on one MI355X.

Workload (the paper's 2D Bose-Hubbard quench, Sec. III, at the scale of a
production run): 32x32 periodic lattice cut into 256 clusters of 2x2 sites,
d = 3 (D = 81), unit-filling Mott state quenched to U/J = 5, RK4 with
dt = 0.01/J to T = 4/J (400 steps), observables recorded every 10 steps.
One benchmark step = one batch of trajectories through the whole path:
sample_noise -> 400 x step_rk4 -> 41 x accumulate_observables.

Prints one JSON line (metric: cluster-steps/s, one cluster-step = one
four-stage RK4 step of one 81x81 cluster matrix).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LX = LY = 32
DT = 0.01
N_STEPS = 400
RECORD_EVERY = 10
N_TRAJ_TOTAL = 4096
FLOP_PER_CLUSTER_STEP = 1.76e6          # structured operator, d = 3, 2x2 clusters
PEAK_FP64_TFLOPS = 78.6                 # MI355X FP64 vector
PEAK_FP32_TFLOPS = 157.3                # MI355X FP32 vector (packed); unpacked issue is half


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed batches")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1024, help="trajectories per batch")
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--rk-steps", type=int, default=N_STEPS, help="RK4 steps per batch (profiling runs only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-leg", action="store_true", help="skip the FP32-state leg")
    ap.add_argument("--no-cv", action="store_true", help="skip the control-variate leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32-vs-FP64 precision leg")
    ap.add_argument("--no-batching", action="store_true", help="skip the mixed-batch leg")
    ap.add_argument("--cv-epochs", type=int, default=60)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


KERNELS = {1: ("k_fused", "kernels_fused.hip"), 2: ("k_plaq", "kernels_plaq.hip")}


def kernel_source_digest(src):
    """Digest of the source of a fused kernel; a stored traffic measurement is
    reported only while it matches."""
    import hashlib
    h = hashlib.sha256()
    for f in (src, "common.hpp"):
        with open(os.path.join(ROOT, "paper_2404_18594_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kname, src, dtype):
    path = os.path.join(ROOT, "profiles", f"{kname}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(dtype)
    if not ent or ent.get("source_digest") != kernel_source_digest(src):
        return None
    return ent


def time_batches(cd, prob, batch, n_batches, warmup, rk_steps):
    import torch
    plan = cd.Plan(prob, batch)
    rho = plan.new_state()
    ws = plan.new_workspace()
    rec = list(range(0, rk_steps + 1, RECORD_EVERY))
    if rec[-1] != rk_steps:
        rec.append(rk_steps)
    sums = torch.zeros(len(rec), cd.NOBS, 3, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ev = []

    def one_batch(b, timed):
        plan.sample_noise(12345, b * batch, rho, stream=stream)
        step = 0
        for k, s in enumerate(rec):
            if s > step:
                if timed:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                plan.step_rk4(rho, ws, DT, s - step, stream=stream)
                if timed:
                    e1.record(stream)
                    ev.append((e0, e1, s - step))
                step = s
            plan.accumulate_observables(rho, k, sums, ws, stream=stream)

    for w in range(warmup):
        one_batch(w, False)
    torch.cuda.synchronize()
    sums.zero_()
    t0 = time.perf_counter()
    for b in range(n_batches):
        one_batch(b, True)
        print(f"# batch {b + 1}/{n_batches} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rk_ms = sum(a.elapsed_time(b) for a, b, _ in ev)
    rk_steps_total = sum(n for _, _, n in ev)
    mean, _ = cd.estimates(sums.cpu(), batch * n_batches)
    return wall, rk_ms, rk_steps_total, len(ev), plan, mean


def cv_leg(cd, batch, epochs):
    """Learned control variate on the same quench (FP64 state): 1024
    training trajectories, 4096 evaluation trajectories, 1e6 i.i.d. patches
    for E[g], 64 recorded times over the 400 steps.  Reports the variance
    ratio Var(O - G) / Var(O) of O = (C^sp_(1,0) + C^sp_(0,1)) / 2 and the
    statistical error reached per GPU-second of sampling with and without g
    (one-time costs, simulation of the training set, training and E[g],
    reported apart)."""
    import numpy as np
    import torch
    from paper_2404_18594_amd import cv
    n_train, n_eval, n_eg = 1024, 4096, 1_000_000
    prob = cd.Problem(LX, LY, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F64)
    rec = cv.record_schedule(N_STEPS, cd.MLP_OUT)
    sec = {}

    def lap(name, t0):
        torch.cuda.synchronize()
        sec[name] = sec.get(name, 0.0) + time.perf_counter() - t0
        print(f"# cv: {name} {sec[name]:.1f} s", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    tr = cv.simulate(prob, n_train, seed=4242, traj_offset=0, dt=DT, record_steps=rec, want_obs=False)
    feats, targ = tr.features, tr.targets
    del tr
    lap("train_simulation", t0)
    t0 = time.perf_counter()
    mlp = cd.Mlp(seed=1)
    hist = cv.train(mlp, feats, targ, epochs=epochs, batch=4096, lr=1e-3)
    lap("training", t0)
    del feats, targ
    Os, Gs = [], []
    plan = None
    for b in range(n_eval // batch):
        t0 = time.perf_counter()
        sim = cv.simulate(prob, batch, seed=4243, traj_offset=b * batch, dt=DT, record_steps=rec,
                          want_targets=False)
        lap("eval_simulation", t0)
        t0 = time.perf_counter()
        O, G = cv.observable_and_cv(sim, mlp)
        lap("inference", t0)
        Os.append(O)
        Gs.append(G)
        plan = sim.plan
        del sim
    t0 = time.perf_counter()
    eg, varg = cv.expectation(plan, mlp, seed=4244, n_samples=n_eg)
    lap("expectation", t0)
    O, G = np.concatenate(Os), np.concatenate(Gs)
    est = cv.estimate(O, G, eg, varg, n_eg, plan.n_clusters / plan.n_sites)
    z = np.abs(est["cv_mean"] - est["plain_mean"]) / np.sqrt(est["cv_se"] ** 2 + est["plain_se"] ** 2)
    tau_plain = sec["eval_simulation"] / n_eval
    tau_cv = tau_plain + sec["inference"] / n_eval
    gain = (est["plain_var"] * tau_plain) / np.maximum(est["cv_var"] * tau_cv, 1e-300)
    # figure of merit sigma^2 t: squared standard error averaged over the
    # recorded times times the GPU-seconds spent, one-time costs included
    t_plain = sec["eval_simulation"]
    t_cv = sum(sec.values())
    fom_plain = float(np.mean(est["plain_se"] ** 2) * t_plain)
    fom_cv = float(np.mean(est["cv_se"] ** 2) * t_cv)
    return {
        "workload": "32x32 periodic, 2x2 clusters, d=3, U/J=5, RK4 dt=0.01/J x 400, O = (C^sp_10 + C^sp_01)/2 "
                    "at 64 times",
        "train_trajectories": n_train, "eval_trajectories": n_eval, "eg_samples": n_eg, "epochs": epochs,
        "train_loss_first_last": [hist[0], hist[-1]],
        "var_ratio_t0": float(est["var_ratio"][0]), "var_ratio_median": float(np.median(est["var_ratio"])),
        "var_ratio_T": float(est["var_ratio"][-1]),
        "max_z_cv_vs_plain": float(z.max()),
        "stat_error_per_gpu_second_T": {"plain": float(np.sqrt(est["plain_var"][-1] * tau_plain)),
                                        "cv": float(np.sqrt(est["cv_var"][-1] * tau_cv))},
        "efficiency_gain_median": float(np.median(gain)), "efficiency_gain_T": float(gain[-1]),
        "figure_of_merit_sigma2_t": {"plain": fom_plain, "cv": fom_cv, "gain": fom_plain / fom_cv,
                                     "plain_gpu_s": t_plain, "cv_gpu_s": t_cv},
        "O_T": {"plain": [float(est["plain_mean"][-1]), float(est["plain_se"][-1])],
                "cv": [float(est["cv_mean"][-1]), float(est["cv_se"][-1])]},
        "seconds": {k: round(v, 3) for k, v in sec.items()},
    }


def precision_leg(cd):
    """FP32 state against FP64 state on identical noise (same seed and
    trajectory indices): the 32x32, d = 3 benchmark quench and a 16x16
    lattice with d = 4 (D = 256), both to T = 4/J with dt = 0.01/J.  Per
    observable: the largest relative error of the trajectory mean over the
    recorded times, and of single trajectories; invariant drift (trace,
    Hermiticity, mean-field energy) of each precision; throughput of each."""
    import numpy as np
    import torch
    out = {}
    names = cd.OBS_NAMES
    for label, L, d, n in (("32x32_d3_D81", 32, 3, 128), ("16x16_d4_D256", 16, 4, 64)):
        rec = list(range(0, N_STEPS + 1, 40))
        runs = {}
        for dt_name, dt_code in (("f64", cd.F64), ("f32", cd.F32)):
            prob = cd.Problem(L, L, 2, 2, d=d, periodic=True, J=1.0, U=5.0, dtype=dt_code)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sums, per = cd.run_quench(prob, n, seed=777, dt=DT, record_steps=rec)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            plan = cd.Plan(prob, 1)
            runs[dt_name] = (per.numpy(), wall, plan.n_clusters, plan.path)
            print(f"# precision: {label} {dt_name} {wall:.1f} s", file=sys.stderr, flush=True)
        p64, w64, nc, path64 = runs["f64"]
        p32, w32, _, path32 = runs["f32"]
        m64, m32 = p64.mean(axis=0), p32.mean(axis=0)          # [n_rec][NOBS]
        se64 = p64.std(axis=0, ddof=1) / np.sqrt(n)
        err = {}
        for k in range(11):                                      # C^sp, nn, density
            scale = np.maximum(np.abs(m64[:, k]), 1e-12)
            dm = np.abs(m32[:, k] - m64[:, k])
            err[names[k]] = {"mean_rel_max": float((dm / scale).max()),
                             "mean_rel_T": float(dm[-1] / scale[-1]),
                             "mean_over_stat_err_max": float((dm[1:] / np.maximum(se64[1:, k], 1e-300)).max()),
                             "traj_abs_max": float(np.abs(p32[:, :, k] - p64[:, :, k]).max())}
        drift = {}
        for nm, pp in (("f64", p64), ("f32", p32)):
            drift[nm] = {"trace_dev_max": float(pp[:, :, 13].max()), "herm_dev_max": float(pp[:, :, 14].max()),
                         "energy_drift_max": float(np.abs(pp[:, -1, 11] - pp[:, 0, 11]).max()),
                         "density_drift_max": float(np.abs(pp[:, -1, 10] - pp[:, 0, 10]).max())}
        cs = n * nc * N_STEPS
        out[label] = {"trajectories": n, "clusters": nc, "rk_steps": N_STEPS, "paths": [path64, path32],
                      "cluster_steps_per_s": {"f64": cs / w64, "f32": cs / w32},
                      "worst_mean_rel_err_T": max(v["mean_rel_T"] for v in err.values()),
                      "nn_distance1_mean_rel_err_T": max(err[o]["mean_rel_T"]
                                                         for o in ("csp_10", "csp_01", "nn_10", "nn_01")),
                      "worst_mean_err_over_stat_err": max(v["mean_over_stat_err_max"] for v in err.values()),
                      "observables": err, "drift": drift}
    return out


def batching_leg(cd, steps=20):
    """The 36-instance batch: cluster shapes 1x1 (D = 3), 2x1 (D = 9), 2x2
    (D = 81), d = 3, square periodic lattices of side 8, 16, 24, 48 with
    4096, 2048, 1024, 256 trajectories, U/J in {3, 5, 10}, dt = 0.01/J, FP32
    state (in FP64 the 2x2 members on 48x48, whose 576 clusters exceed the 256
    that can be co-resident, need the per-stage workspace and the whole set
    no longer fits in 288 GB).
    One batch call advances everything: the 1x1 and 2x1 members in one
    mixed-shape launch per stage (graph-captured), the 2x2 members on their
    fused kernel.  Timed over `steps` RK4 steps after one warm-up step
    (which tunes and captures); the 1x1 and 2x1 members are also timed one
    plan at a time on the per-stage path for comparison."""
    import torch
    traj = {8: 4096, 16: 2048, 24: 1024, 48: 256}
    members = [(L, cx, cy, U) for (cx, cy) in ((1, 1), (2, 1), (2, 2)) for L in (8, 16, 24, 48) for U in (3.0, 5.0, 10.0)]
    plans, rhos = [], []
    for i, (L, cx, cy, U) in enumerate(members):
        prob = cd.Problem(L, L, cx, cy, d=3, periodic=True, J=1.0, U=U, dtype=cd.F32)
        p = cd.Plan(prob, traj[L])
        r = p.new_state()
        p.sample_noise(900 + i, 0, r)
        plans.append(p)
        rhos.append(r)
    batch = cd.Batch(plans)
    ws = batch.new_workspaces()
    batch.step_rk4(rhos, ws, DT, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step_rk4(rhos, ws, DT, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cs = {"1x1": 0, "2x1": 0, "2x2": 0}
    for (L, cx, cy, U), p in zip(members, plans):
        cs[f"{cx}x{cy}"] += p.n_traj * p.n_clusters * steps
    # small members alone: batched vs one plan at a time
    small = [i for i, m in enumerate(members) if m[1] * m[2] < 4]
    sb = cd.Batch([plans[i] for i in small])
    sws = [ws[i] for i in small]
    srho = [rhos[i] for i in small]
    sb.step_rk4(srho, sws, DT, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sb.step_rk4(srho, sws, DT, steps)
    torch.cuda.synchronize()
    w_small_batched = time.perf_counter() - t0
    t0 = time.perf_counter()
    for i in small:
        plans[i].step_rk4(rhos[i], ws[i], DT, steps)
    torch.cuda.synchronize()
    w_small_single = time.perf_counter() - t0
    info = batch.info()
    total = sum(cs.values())
    return {"instances": len(members), "dtype": "f32", "rk_steps": steps, "wall_s": wall,
            "cluster_steps_per_s": total / wall, "paths": [p.path for p in plans],
            "cluster_steps": cs, "mixed_members": info["mixed_members"], "tuned_threads": info["threads"],
            "tuned_variants_1x1_2x1_1x2": info["variants"], "workgroups_per_stage": info["workgroups"],
            "small_members": {"batched_s": w_small_batched, "one_plan_at_a_time_s": w_small_single,
                              "cluster_steps_per_s_batched": (cs["1x1"] + cs["2x1"]) / w_small_batched,
                              "speedup": w_small_single / w_small_batched}}


def cpu_baseline():
    import oracle
    cores = len(os.sched_getaffinity(0))
    p = oracle.Problem(LX, LY, 2, 2, d=3, periodic=True, J=1.0, U=5.0)
    tb = oracle.mott_tables(3)
    n_traj, steps = cores, 60
    oracle.run(p, tb, seed=1, traj_offset=0, n_traj=1, dt=DT, n_steps=1, record_steps=[1], nthreads=cores)
    t0 = time.perf_counter()
    oracle.run(p, tb, seed=1, traj_offset=0, n_traj=n_traj, dt=DT, n_steps=steps, record_steps=[steps],
               nthreads=cores)
    dt = time.perf_counter() - t0
    cs = n_traj * p.nc * steps
    return {"value": cs / dt, "unit": "cluster-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_traj} trajectories x {steps} RK4 steps of the 32x32 lattice, 2x2 clusters, d=3 "
                      f"({cs} cluster-steps, {dt:.1f} s, FP64, dense Kronecker-built operators)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs shard trajectories "
                                   "and are not part of it", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2404_18594_amd as cd

    batch = args.batch
    n_batches = args.steps if args.steps is not None else max(1, N_TRAJ_TOTAL // batch)
    prob = cd.Problem(LX, LY, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F64 if args.dtype == "f64" else cd.F32)
    wall, rk_ms, rk_steps_total, n_calls, plan, mean = time_batches(cd, prob, batch, n_batches, args.warmup,
                                                                    args.rk_steps)
    clusters = plan.n_clusters
    cluster_steps = batch * n_batches * clusters * args.rk_steps
    value = cluster_steps / wall
    # dominant kernel: the fused RK4 kernel (one launch per step_rk4 call of
    # RECORD_EVERY steps) or, on the per-stage path, the stage kernel
    if plan.path in KERNELS:
        (kname, ksrc), launches, steps_per_launch = KERNELS[plan.path], n_calls, RECORD_EVERY
    else:
        kname, ksrc, launches, steps_per_launch = "k_stage", None, 4 * rk_steps_total, 0.25
    avg_launch_ms = rk_ms / launches
    flop_per_launch = FLOP_PER_CLUSTER_STEP * steps_per_launch * batch * clusters
    achieved = flop_per_launch / (avg_launch_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if args.dtype == "f64" else PEAK_FP32_TFLOPS
    traffic = stored_traffic(kname, ksrc, args.dtype) if ksrc else None
    out = {
        "metric": "cluster-steps/s (2x2, D=81)",
        "value": value,
        "unit": "cluster-steps/s",
        "n_gpus": 1,
        "steps": n_batches,
        "warmup": args.warmup,
        "ms_per_step": wall / n_batches * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "32x32 periodic Bose-Hubbard, 2x2 clusters (D=81), d=3, Mott quench U/J=5, "
                               f"RK4 dt=0.01/J x {args.rk_steps}, {batch * n_batches} trajectories",
                   "trajectories_per_step": batch, "clusters": clusters, "rk_steps": args.rk_steps,
                   "record_every": RECORD_EVERY},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None if traffic is None else traffic["bytes_per_cluster_step"] * steps_per_launch * batch * clusters,
                     "kernel": kname, "avg_launch_ms": avg_launch_ms, "flop_per_launch": flop_per_launch,
                     "launches": launches},
        "C_sp_r1_at_T": float(0.5 * (mean[-1, 0] + mean[-1, 1])),
    }
    if not args.no_fp32_leg and args.dtype == "f64":
        p32 = cd.Problem(LX, LY, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F32)
        w32, ms32, _, nc32, plan32, _ = time_batches(cd, p32, batch, 1, 1, args.rk_steps)
        ach32 = FLOP_PER_CLUSTER_STEP * RECORD_EVERY * batch * clusters / (ms32 / nc32 * 1e-3) / 1e12
        out["fp32"] = {"value": batch * clusters * args.rk_steps / w32, "unit": "cluster-steps/s",
                       "trajectories": batch, "kernel_tflops": ach32, "frac_of_fp32_peak": ach32 / PEAK_FP32_TFLOPS,
                       "path": plan32.path, "kernel": KERNELS.get(plan32.path, ("k_stage",))[0],
                       "resident_trajectories": plan32.resident, "wall_s": w32}
        del plan32
    if not args.no_cv and args.dtype == "f64" and args.rk_steps == N_STEPS:
        out["control_variate"] = cv_leg(cd, batch, args.cv_epochs)
    if not args.no_batching and args.dtype == "f64" and args.rk_steps == N_STEPS:
        out["batching"] = batching_leg(cd)
    if not args.no_precision and args.dtype == "f64" and args.rk_steps == N_STEPS:
        out["precision"] = precision_leg(cd)
    if args.copy_calib:
        import torch
        n = 1 << 30
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = n
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
