"""Benchmark of the DPD + CGMD multiple-time-stepping hot path on one MI355X.

Workload (synthetic, seeded): Poiseuille channel of 2,000,000 DPD particles (fluid +
frozen wall layers) in a 200 x 50 x 66.7 box, periodic in x and z, body force 0.02
along x, with 4 randomly placed platelets of 2,562 CG beads (level-4 icosphere on a
(3, 1, 3) oblate ellipsoid): 2,010,248 particles in all.  It stands in for the paper's
102-million-particle clot, whose platelet model is not available.

A "step" is one outer step of the whole hot path: cell-list rebuild (counting sort),
DPD outer forces, k inner steps of the platelet group (bonds, angles, WCA, platelet-
fluid forces), RESPA kicks/drifts, diagnostics and platelet features.

Legs, all from the same equilibrated state:
  * MTS (the headline `value`): float32 pair forces, float64 state, fixed ratio k
    (default 4, the controller's fallback) or the learned controller (--controller).
  * STS: float64 forces, ratio 1, run over the same simulated time.
Reported: particle-(outer)steps/s, simulated time per day, the simulated-time speedup
MTS/STS, and the relative difference of their time-averaged peculiar temperatures.
The roofline figure is for the dominant kernel (the DPD outer-force kernel), timed
live with HIP events on the library's stream during the MTS leg.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s and simulated-time/day: FP64 STS vs FP32 AI-MTS at equal T error"
DT_INNER = 0.0025
SECONDS_PER_DAY = 86400.0
# VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-slots per second)
VALU_PEAK = 256 * 64 * 2.4e9
# Algorithmic VALU lane-slots per fluid particle per DPD evaluation (half-shell cell list:
# ~40 distance tests and 6.3 unique pairs per particle at density 3): float32 / float64 pair math
SLOTS_PER_PARTICLE = {True: 1.9e3, False: 2.6e3}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed outer steps of the MTS leg")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--k", type=int, default=4, help="MTS ratio of the MTS leg")
    ap.add_argument("--equil", type=int, default=800, help="untimed float32 STS steps before both legs")
    ap.add_argument("--controller", default="", help="path of trained controller weights (.npy): AI-MTS leg")
    ap.add_argument("--n-total", type=int, default=2_000_000)
    ap.add_argument("--skip-sts", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-outer-steps", type=int, default=3, help="oracle outer steps timed on the host")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this many MiB first (reference for HBM counters)")
    return ap.parse_args()


def workload(n_total):
    import synth
    scale = n_total / 2_000_000
    L = (200.0 * scale, 50.0, 66.7) if n_total != 2_000_000 else (200.0, 50.0, 66.7)
    return synth.channel(n_total=n_total, L=L, n_platelet=4, level=4, seed=20220530, g=0.02)


def cpu_baseline(sysd, k, outer_steps):
    """The oracle as it stands (float64, OpenMP over the host cores for the outer group)
    on a bounded sample: `outer_steps` RESPA outer steps of the same workload."""
    import oracle
    S = oracle.System(sysd)
    nthreads = os.cpu_count() or 1
    x, v = sysd["x"].copy(), sysd["v"].copy()
    t0 = time.perf_counter()
    fo = S.outer_forces(x, v, 0, k * DT_INNER, nthreads=nthreads)
    fi = S.inner_forces(x, v, 0, DT_INNER)
    t1 = time.perf_counter()
    S.respa(x, v, fo, fi, [1, 1], outer_steps, k * DT_INNER, k, nthreads=nthreads)
    t2 = time.perf_counter()
    n = sysd["n"]
    rate = n * outer_steps / (t2 - t1)
    return {"value": rate, "unit": "particle-steps/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d RESPA outer step(s) at k=%d (float64) of the %d-particle channel, after one "
                      "force evaluation (%.1f s); %.1f s timed" % (outer_steps, k, n, t1 - t0, t2 - t1),
            "tau_per_day": outer_steps * k * DT_INNER / (t2 - t1) * SECONDS_PER_DAY}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the sharding design is "
              "described in DESIGN.md); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2205_14121_amd.aimts as A

    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_gen = time.perf_counter()
    d = workload(args.n_total)
    t_gen = time.perf_counter() - t_gen
    N = int(d["n"])
    k = args.k
    series_cap = args.steps + args.warmup + 8

    # --- equilibration from the uniform random start (untimed) ---
    eq = A.from_workload(d, fp32=True, skin=0.4)
    eq.compute_forces(DT_INNER, 1)
    eq.step(args.equil, DT_INNER, 1)
    x_eq, v_eq = eq.state()
    cnt_eq = eq.counters()
    eq.close()
    del eq

    # --- MTS leg (headline) ---
    mts = A.from_workload(d, fp32=True, skin=0.4, series_capacity=series_cap, ctrl_max_batch=8)
    mode = 0
    if args.controller:
        mts.ctrl_set_weights(np.load(args.controller).astype(np.float32))
        mode = 1
    mts.set_state(x_eq, v_eq)
    mts.set_counters(*cnt_eq)
    mts.compute_forces(DT_INNER, k)
    mts.step(args.warmup, DT_INNER, k, mode=mode, diag_every=1)
    mts.profile(1)  # HIP events around the DPD outer-force kernel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mts.step(args.steps, DT_INNER, k, mode=mode, diag_every=1)
    torch.cuda.synchronize()
    t_mts = time.perf_counter() - t0
    prof_ms, prof_n = mts.get_profile()
    rows = mts.series()
    diag = mts.diag()
    sim_mts = float(rows[-1, 0] - rows[args.warmup - 1, 0]) if args.warmup > 0 else float(rows[-1, 0])
    Tpec_mts = float(np.mean(rows[args.warmup:, 3]))
    mean_k = float(np.mean(rows[args.warmup:, 7]))
    value = N * args.steps / t_mts

    # --- STS leg: float64, ratio 1, same simulated time from the same state ---
    sts = None
    if not args.skip_sts:
        n_sts = int(round(sim_mts / DT_INNER))
        ctx = A.from_workload(d, fp32=False, skin=0.4, series_capacity=n_sts + 8)
        ctx.set_state(x_eq, v_eq)
        ctx.set_counters(*cnt_eq)
        ctx.compute_forces(DT_INNER, 1)
        ctx.step(args.warmup, DT_INNER, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(n_sts, DT_INNER, 1, diag_every=1)
        torch.cuda.synchronize()
        t_sts = time.perf_counter() - t0
        srows = ctx.series()
        Tpec_sts = float(np.mean(srows[:, 3]))
        sts = {"particle_steps_per_s": N * n_sts / t_sts, "steps": n_sts, "ms_per_step": 1e3 * t_sts / n_sts,
               "tau_per_day": n_sts * DT_INNER / t_sts * SECONDS_PER_DAY, "T_pec": Tpec_sts}
        ctx.close()

    # --- roofline of the dominant kernel (DPD outer forces, float32) ---
    dpd_ms = prof_ms[0] / max(prof_n[0], 1)
    n_fluid = int(d["n_fluid"])
    slots = n_fluid * SLOTS_PER_PARTICLE[True]
    achieved = slots / (dpd_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK / 1e12, 3),
                "unit": "T lane-slots/s", "frac": round(achieved * 1e12 / VALU_PEAK, 4), "traffic": None,
                "kernel": "k_dpd<float>", "avg_ms": round(dpd_ms, 4), "launches": int(prof_n[0]),
                "algorithmic_slots_per_launch": slots}

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_mts / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-pair-forces/f64-state", "data": "synthetic",
        "config": {"workload": "Poiseuille channel, %d DPD particles (fluid + frozen walls) in %.1fx%.1fx%.1f, "
                               "g=0.02, 4 platelets x 2,562 beads; float32 pair forces, float64 state; "
                               "RESPA %s" % (int(d["n_fluid"] + d["n_wall"]), *d["box_L"],
                                             "learned controller" if mode else "fixed k=%d" % k),
                   "particles": N, "k": k if not mode else "controller", "mean_k": mean_k, "dt_inner": DT_INNER},
        "mts": {"tau_per_day": sim_mts / t_mts * SECONDS_PER_DAY, "T_pec": Tpec_mts, "mean_k": mean_k,
                "controller_inferences": int(diag.inferences), "fallbacks": int(diag.fallbacks)},
        "sts_fp64": sts,
        "roofline": roofline,
    }
    if sts:
        out["simtime_speedup_vs_sts"] = out["mts"]["tau_per_day"] / sts["tau_per_day"]
        out["T_error_vs_sts"] = abs(Tpec_mts - sts["T_pec"]) / sts["T_pec"]
    if not args.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(d, k, args.cpu_outer_steps)
    out["workload_generation_s"] = t_gen
    print(json.dumps(out))


if __name__ == "__main__":
    main()
