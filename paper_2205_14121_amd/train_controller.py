"""Generate controller training data from the simulator itself, train the controller on
the device with the library's own forward/backward/Adam kernels, and evaluate it
against the method without it (fixed fallback ratio 4) on held-out shear rates.

    python -m paper_2205_14121_amd.train_controller --out paper_2205_14121_amd/data/controller.npy

Workload: Poiseuille channels of the benchmark's recipe (frozen walls in y, periodic x
and z, 4 level-4 platelets) shortened in x, with the body force drawn uniformly from
[0.005, 0.05] per training trajectory; held-out trajectories use body forces outside
the training range's middle.  Everything is seeded.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2205_14121_amd import aimts as A  # noqa: E402
from paper_2205_14121_amd import controller as ctl  # noqa: E402

DT = 0.0025
SKIN = 0.8  # room for the largest ratio (16): two outer-step paths of |v| ~ 5 at 0.04 each


def make_workload(n_total, Lx, seed):
    import synth

    def wl(g):
        return synth.channel(n_total=n_total, L=(Lx, 50.0, 66.7), n_platelet=4, level=4, seed=seed, g=float(g))
    return wl


def evaluate(weights, wl, g_values, n_outer, log=print):
    """For each held-out body force, run (a) STS float64 at dt, (b) fixed k = 4 float32 and
    (c) the controller float32, from the same equilibrated state over the same simulated
    time; report simulated time per second of wall time and the peculiar-T deviation."""
    import torch
    out = []
    for g in g_values:
        d = wl(g)
        eq = A.from_workload(d, fp32=True, skin=SKIN)
        eq.compute_forces(DT, 1)
        eq.step(800, DT, 1)
        x, v = eq.state()
        cnt = eq.counters()
        eq.close()
        span = n_outer * 4 * DT
        res = {"g": float(g)}
        for name, fp32, k, mode in (("sts_fp64", False, 1, 0), ("fixed4", True, 4, 0), ("ai", True, 4, 1)):
            n = int(round(span / (k * DT))) if mode == 0 else n_outer * 16
            ctx = A.from_workload(d, fp32=fp32, skin=SKIN, series_capacity=n + 8, ctrl_max_batch=8)
            if mode == 1:
                ctx.ctrl_set_weights(weights)
            ctx.set_state(x, v)
            ctx.set_counters(*cnt)
            ctx.compute_forces(DT, k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == 0:
                ctx.step(n, DT, k, diag_every=1)
            else:
                # advance until the same simulated time is covered
                done = 0.0
                while done < span - 1e-9:
                    ctx.step(64, DT, k, mode=1, diag_every=1)
                    done = ctx.diag().time
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            rows = ctx.series()
            dg = ctx.diag()
            res[name] = {"sim_time": float(rows[-1, 0]), "wall_s": wall, "outer_steps": int(dg.step),
                         "tau_per_s": float(rows[-1, 0]) / wall, "T_pec": ctl.time_average(rows, 3),
                         "mean_k": ctl.time_average(rows, 7), "fallbacks": int(dg.fallbacks)}
            ctx.close()
        ref = res["sts_fp64"]["T_pec"]
        for name in ("fixed4", "ai"):
            res[name]["T_err"] = abs(res[name]["T_pec"] - ref) / ref
        res["gain_simtime_rate_ai_over_fixed4"] = res["ai"]["tau_per_s"] / res["fixed4"]["tau_per_s"]
        log("g=%.4f: STS %.3g tau/s; fixed-4 %.3g tau/s (dT %.2f%%); AI mean k %.2f, %.3g tau/s (dT %.2f%%)" % (
            g, res["sts_fp64"]["tau_per_s"], res["fixed4"]["tau_per_s"], 100 * res["fixed4"]["T_err"],
            res["ai"]["mean_k"], res["ai"]["tau_per_s"], 100 * res["ai"]["T_err"]))
        out.append(res)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "data", "controller.npy"))
    ap.add_argument("--report", default="")
    ap.add_argument("--n-total", type=int, default=200_000)
    ap.add_argument("--lx", type=float, default=20.0)
    ap.add_argument("--train-traj", type=int, default=16)
    ap.add_argument("--heldout", type=int, default=3)
    ap.add_argument("--windows", type=int, default=24)
    ap.add_argument("--label-every", type=int, default=2)
    ap.add_argument("--ae-steps", type=int, default=400)
    ap.add_argument("--head-steps", type=int, default=800)
    ap.add_argument("--eval-outer", type=int, default=400)
    ap.add_argument("--seed", type=int, default=20220531)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    rng = np.random.default_rng(args.seed)
    t0 = time.time()
    wl = make_workload(args.n_total, args.lx, args.seed)

    def make_ctx(d, series_capacity):
        return A.from_workload(d, fp32=True, skin=SKIN, series_capacity=series_capacity)

    g_train = rng.uniform(0.005, 0.05, size=args.train_traj)
    X, Y, meta = ctl.generate(make_ctx, wl, g_train, args.windows, dt=DT, label_every=args.label_every,
                              log=lambda m: print(m, flush=True))
    print("data: %d windows, ratio labels %s, hold labels %s (%.0f s)" % (
        X.shape[0], np.bincount(Y[:, 0], minlength=5).tolist(), np.bincount(Y[:, 1], minlength=4).tolist(),
        time.time() - t0), flush=True)
    ctx = A.from_workload(wl(0.02), fp32=True, skin=SKIN, ctrl_max_batch=256)
    p0 = ctl.set_norm(ctl.init_params(args.seed), X)
    ctx.ctrl_set_weights(p0)
    hist = ctl.train(ctx, X, Y, ae_steps=args.ae_steps, head_steps=args.head_steps, log=lambda m: print(m, flush=True))
    W = ctx.ctrl_get_weights()
    pr, ph = ctl.predict(ctx, X)
    acc_r = float(np.mean(pr == Y[:, 0]))
    acc_h = float(np.mean(ph == Y[:, 1]))
    print("train accuracy: ratio %.3f hold %.3f" % (acc_r, acc_h), flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, W)
    # held-out body forces outside the middle of the training range
    g_held = np.array([0.004, 0.03, 0.055])[:args.heldout]
    ev = evaluate(W, wl, g_held, args.eval_outer, log=lambda m: print(m, flush=True))
    report = {"train_windows": int(X.shape[0]), "ratio_label_counts": np.bincount(Y[:, 0], minlength=5).tolist(),
              "hold_label_counts": np.bincount(Y[:, 1], minlength=4).tolist(),
              "g_train": g_train.tolist(), "ae_loss": [hist["ae"][0], hist["ae"][-1]],
              "head_loss": [hist["head"][0], hist["head"][-1]], "train_acc_ratio": acc_r, "train_acc_hold": acc_h,
              "heldout": ev, "seconds": time.time() - t0}
    path = args.report or os.path.splitext(args.out)[0] + "_report.json"
    with open(path, "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps({k: v for k, v in report.items() if k != "heldout"}))


if __name__ == "__main__":
    main()
