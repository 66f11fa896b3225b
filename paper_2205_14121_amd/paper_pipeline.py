"""Training data, training and evaluation of the paper's own inference pipeline (Sec. 3.3,
Table 2): windows of 50 outer steps of the six platelet measurements (angular velocity
components, translational and rotational kinetic energy, flow speed at the centre of
mass), labelled with the MTS ratio the simulator itself admits; an autoencoder (2-layer
LSTM, 16 and 4 units, 8 latents) trained on reconstruction, then the FCN 8-32-16-8-1 on
the frozen latents against log2 of the ratio.  Every step runs in the library's kernels
(aimts_get_paper_features, aimts_lstm_*); this module only drives them.

    python -m paper_2205_14121_amd.paper_pipeline --out paper_2205_14121_amd/data/paper_pipeline.npy

Labels come from trial re-simulation of the candidate ratios (Sec. 3.3): from the
window's end state the system is re-simulated at every ratio r in {1, 2, 4, 8, 16} over
the same simulated time.  For platelet p and ratio r the normalised deviation is
D_p(r) = max(|T_r - T_1| / (tol_T T_1), max_k |lambda_k,r - lambda_k,1| / (tol_shape lambda_k,1))
(fluid peculiar temperature, the platelet's gyration eigenvalues; tol_T = 1 %,
tol_shape = 2 %).  The FCN's single output is a regression (Sec. 3.3: one output
neuron): its target is the log2 ratio at which D_p reaches 1, interpolated linearly in
log2 r between the last admissible ratio and the first inadmissible one (4 if every
ratio up to 16 is admissible; a branch that fails its stability checks counts as
D = infinity).  Categorisation rounds the prediction to the nearest level.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2205_14121_amd import aimts as A  # noqa: E402
from paper_2205_14121_amd import controller as ctl  # noqa: E402

T, F = 50, 6
STRIDE = 25
DT = 0.0025
SKIN = 0.8
FLOW_R = 4.0


def n_params():
    n = A.C.c_int64()
    A._check(None, A.lib.aimts_lstm_num_params(A.C.byref(n)))
    return int(n.value)


def init_params(seed=0):
    """Uniform(-1/sqrt(fan), 1/sqrt(fan)) weights and biases (fan: the LSTM's units, or the
    linear layer's input width), the normalisation slots at (0, 1)."""
    rng = np.random.default_rng(seed)
    shapes = [(64, 6, 16), (64, 16, 16), (64, 1, 16), (64, 1, 16),  # enc0: w_ih, w_hh, b_ih, b_hh
              (16, 16, 4), (16, 4, 4), (16, 1, 4), (16, 1, 4),      # enc1
              (16, 8, 4), (16, 4, 4), (16, 1, 4), (16, 1, 4),       # dec0
              (64, 4, 16), (64, 16, 16), (64, 1, 16), (64, 1, 16),  # dec1
              (6, 16, 16), (6, 1, 16),                              # read-out
              (32, 8, 8), (32, 1, 8), (16, 32, 32), (16, 1, 32), (8, 16, 16), (8, 1, 16), (1, 8, 8), (1, 1, 8)]
    parts = [rng.uniform(-1.0, 1.0, r * c) / math.sqrt(fan) for r, c, fan in shapes]
    parts += [np.zeros(F), np.ones(F)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == n_params()
    return p


def branch_deviations(brn, d, x, v, counters, horizon, tol_T=0.01, tol_shape=0.02):
    """D[r_index, p]: normalised deviation of every ratio's branch from the ratio-1 branch."""
    from .aimts import AimtsError, E_UNSTABLE
    P = int(d["n_platelet"])
    T1, G1 = ctl._branch_stats(brn, d, x, v, counters, DT, 1, horizon)
    D = np.zeros((len(ctl.RATIOS), P))
    for i, r in enumerate(ctl.RATIOS[1:], start=1):
        try:
            Tr, Gr = ctl._branch_stats(brn, d, x, v, counters, DT, r, horizon)
        except AimtsError as e:
            if e.status != E_UNSTABLE:
                raise
            D[i:] = np.inf
            break
        dt_ = abs(Tr - T1) / (tol_T * T1)
        ds = np.max(np.abs(Gr - G1) / (tol_shape * np.maximum(G1, 1e-12)), axis=1)
        D[i] = np.maximum(dt_, ds)
    return D


def target_from_deviations(Dp):
    """log2 of the ratio at which the deviation of one platelet reaches 1 (see above)."""
    lr = np.log2(np.array(ctl.RATIOS, np.float64))
    for i in range(1, len(lr)):
        if not Dp[i] <= 1.0:
            lo = Dp[i - 1]
            if not np.isfinite(Dp[i]):
                return float(lr[i - 1])
            frac = (1.0 - lo) / max(Dp[i] - lo, 1e-12)
            return float(lr[i - 1] + np.clip(frac, 0.0, 1.0) * (lr[i] - lr[i - 1]))
    return float(lr[-1])


def generate(workload, g_values, windows_per_traj, k_run=(4, 8), equil=200, label_every=2, log=print):
    """One trajectory per body force: every outer step records the six measurements of
    every platelet; every STRIDE outer steps the last 50 rows form a window per platelet,
    labelled (every label_every-th window; the others repeat the last label) by trial
    re-simulation.  Returns (windows [n, 50, 6] float32, log2 targets [n] float32, meta,
    deviations [n, 5])."""
    horizon = 64 * 4 * DT
    X, Y, meta, DV = [], [], [], []
    for ti, g in enumerate(g_values):
        k_tr = k_run[ti % len(k_run)]
        d = workload(g)
        run = A.from_workload(d, fp32=True, skin=SKIN, series_capacity=16)
        brn = A.from_workload(d, fp32=True, skin=SKIN, series_capacity=int(round(horizon / DT)) + 8)
        run.compute_forces(DT, 1)
        run.step(equil, DT, 1)
        run.compute_forces(DT, k_tr)
        rows = []
        for _ in range(T):
            run.step(1, DT, k_tr)
            rows.append(run.paper_features(FLOW_R))
        D = None
        for w in range(windows_per_traj):
            win = np.array(rows[-T:])  # [50, P, 6]
            if w % label_every == 0 or D is None:
                x, v = run.state()
                D = branch_deviations(brn, d, x, v, run.counters(), horizon)
            for p in range(win.shape[1]):
                X.append(win[:, p, :])
                Y.append(target_from_deviations(D[:, p]))
                meta.append((ti, float(g), w, p))
                DV.append(D[:, p])
            for _ in range(STRIDE):
                run.step(1, DT, k_tr)
                rows.append(run.paper_features(FLOW_R))
        log("trajectory %d (g=%.4f, k=%d): %d windows, targets of the last %s" %
            (ti, g, k_tr, windows_per_traj, np.round(Y[-win.shape[1]:], 3).tolist()), flush=True)
        run.close()
        brn.close()
    return np.array(X, np.float32), np.array(Y, np.float32), meta, np.array(DV)


def set_norm(net, params, windows):
    """Per-feature mean and std of the denoised training windows (the library's own filter
    with the normalisation at (0, 1)) into the normalisation slots."""
    import torch
    p = params.copy()
    p[-2 * F:-F] = 0.0
    p[-F:] = 1.0
    dp = torch.from_numpy(p).cuda()
    out = []
    for s in range(0, windows.shape[0], net.max_batch):
        out.append(net.filter(dp, torch.from_numpy(np.ascontiguousarray(windows[s:s + net.max_batch])).cuda()).cpu())
    y = torch.cat(out).numpy().reshape(-1, F).astype(np.float64)
    std = y.std(axis=0)
    std[std < 1e-9] = 1.0
    p[-2 * F:-F] = y.mean(axis=0)
    p[-F:] = std
    return p


def train(net, params, windows, y, ae_steps=600, fcn_steps=1500, batch=256, lr_ae=3e-3, lr_fcn=3e-3, seed=0,
          log=print):
    """Autoencoder on reconstruction, then the FCN on the frozen latents (Sec. 3.3)."""
    import torch
    rng = np.random.default_rng(seed)
    n = windows.shape[0]
    dp = torch.from_numpy(params.copy()).cuda()
    m = torch.zeros_like(dp)
    v = torch.zeros_like(dp)
    dW = torch.from_numpy(np.ascontiguousarray(windows)).cuda()
    dY = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    hist = {"ae": [], "fcn": []}
    for phase, steps, lr, key in ((0, ae_steps, lr_ae, "ae"), (1, fcn_steps, lr_fcn, "fcn")):
        m.zero_()
        v.zero_()
        for it in range(steps):
            idx = torch.from_numpy(rng.choice(n, size=min(batch, n), replace=False)).cuda()
            xb = dW.index_select(0, idx).contiguous()
            yb = dY.index_select(0, idx).contiguous()
            g, loss = net.backward(dp, xb, yb, phase)
            net.adam(dp, m, v, g, phase, it + 1, lr)
            hist[key].append(float(loss.cpu()[0]))
            if it % 200 == 0:
                log("phase %d step %d loss %.5f" % (phase, it, hist[key][-1]))
    return dp.cpu().numpy(), hist


def predict(net, params, windows):
    """Predicted log2 ratio per window (device forward pass) and the categorised ratio."""
    import torch
    dp = torch.from_numpy(np.ascontiguousarray(params)).cuda()
    out = []
    for s in range(0, windows.shape[0], net.max_batch):
        _, pred, _ = net.forward(dp, torch.from_numpy(np.ascontiguousarray(windows[s:s + net.max_batch])).cuda())
        out.append(pred.cpu().numpy())
    y = np.concatenate(out)
    return y, categorize(y)


def categorize(y):
    """Predicted log2 ratios to the integration levels {1, 2, 4, 8, 16} (nearest level)."""
    return np.array(ctl.RATIOS)[np.clip(np.rint(np.asarray(y, np.float64)), 0, len(ctl.RATIOS) - 1).astype(int)]


def control(ctx, params, n_outer, dt, k_start=4, k_max=8, every=STRIDE, levels=False, k_if=2, k_sub=2,
            flow_r=FLOW_R):
    """The paper's AI-MTS loop (Sec. 3.3; Table 1, Table 2) on a context whose forces are
    computed: one outer step at a time, the six measurements of every platelet after each.
    Once 50 rows exist, and then every `every` outer steps, the pipeline predicts each
    platelet's log2 ratio from its last 50 rows (the device forward pass) and categorises
    it.  The outer ratio becomes the smallest platelet's ratio, capped at k_max.  With
    `levels` (a three-level context), a platelet whose own ratio exceeds the outer one
    runs its own terms at the flowing sublevel (every k_sub inner steps), the others at the
    aggregating one (every inner step), as the categorisation rows of Table 2 assign
    platelets to levels.  Returns one record per decision: the outer step after which it
    was made, the windows [P, 50, 6], the predictions, the categorised ratios, the outer
    ratio and the sublevels."""
    import collections
    import torch
    P = int(ctx.desc.n_platelet)
    net = A.LstmPipeline(max(P, 1))
    dp = torch.from_numpy(np.ascontiguousarray(params, np.float32)).cuda()
    rows = collections.deque(maxlen=T)
    k = int(k_start)
    decisions = []
    for n in range(int(n_outer)):
        ctx.step(1, dt, k)
        rows.append(ctx.paper_features(flow_r))
        if len(rows) < T or (n + 1 - T) % every != 0:
            continue
        win = np.ascontiguousarray(np.transpose(np.array(rows), (1, 0, 2)), np.float32)  # [P, 50, 6]
        _, pred, _ = net.forward(dp, torch.from_numpy(win).cuda())
        y = pred.cpu().numpy().astype(np.float64)
        ratio = categorize(y)
        k_new = int(min(int(ratio.min()), int(k_max)))
        lev = None
        if levels:
            lev = np.where(ratio > k_new, 1, 2).astype(np.int32)
            ctx.set_levels(min(k_if, k_new), min(k_sub, k_if, k_new), lev)
            ctx.compute_forces(dt, k_new)
        decisions.append({"step": n + 1, "windows": win, "pred": y, "ratio": ratio, "k": k_new, "levels": lev})
        k = k_new
    return decisions


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=os.path.join(HERE, "data", "paper_pipeline.npy"))
    ap.add_argument("--n-total", type=int, default=200_000)
    ap.add_argument("--lx", type=float, default=20.0)
    ap.add_argument("--trajectories", type=int, default=32)
    ap.add_argument("--windows", type=int, default=12)
    ap.add_argument("--seed", type=int, default=20220534)
    args = ap.parse_args()
    import synth
    t0 = time.time()

    def workload(g):
        return synth.channel(n_total=args.n_total, L=(args.lx, 50.0, 66.7), n_platelet=4, level=4, seed=args.seed,
                             g=float(g))

    rng = np.random.default_rng(args.seed)
    g_train = rng.uniform(0.005, 0.05, args.trajectories)
    g_test = np.array([0.004, 0.03, 0.055])
    Xtr, ytr, _, Dtr = generate(workload, g_train, args.windows)
    Xte, yte, _, Dte = generate(workload, g_test, args.windows)
    net = A.LstmPipeline(256)
    p = set_norm(net, init_params(args.seed), Xtr)
    p, hist = train(net, p, Xtr, ytr)
    yhat_tr, r_tr = predict(net, p, Xtr)
    yhat_te, r_te = predict(net, p, Xte)
    lab_tr, lab_te = categorize(ytr), categorize(yte)
    rmse = lambda a, b: float(np.sqrt(np.mean((np.asarray(a, np.float64) - b) ** 2)))
    report = {
        "windows_train": int(Xtr.shape[0]), "windows_test": int(Xte.shape[0]),
        "target_log2_mean_std_train": [float(np.mean(ytr)), float(np.std(ytr))],
        "target_log2_mean_std_test": [float(np.mean(yte)), float(np.std(yte))],
        "label_counts_train": {str(r): int(np.sum(lab_tr == r)) for r in ctl.RATIOS},
        "label_counts_test": {str(r): int(np.sum(lab_te == r)) for r in ctl.RATIOS},
        "deviation_at_ratio_8_16_median_test": [float(np.median(Dte[:, 3])), float(np.median(Dte[:, 4]))],
        "ae_loss_first_last": [hist["ae"][0], hist["ae"][-1]],
        "fcn_loss_first_last": [hist["fcn"][0], hist["fcn"][-1]],
        "rmse_log2_train": rmse(yhat_tr, ytr), "rmse_log2_test": rmse(yhat_te, yte),
        "rmse_log2_test_constant_mean_predictor": rmse(np.full_like(yte, np.mean(ytr)), yte),
        "correlation_prediction_target_test": float(np.corrcoef(yhat_te, yte)[0, 1]) if np.std(yte) > 0 else None,
        "accuracy_train": float(np.mean(r_tr == lab_tr)), "accuracy_test": float(np.mean(r_te == lab_te)),
        "prediction_std_test": float(np.std(yhat_te)),
        "predicted_ratio_counts_test": {str(r): int(np.sum(r_te == r)) for r in ctl.RATIOS},
        "seconds": time.time() - t0,
    }
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, p)
    with open(os.path.splitext(args.out)[0] + "_report.json", "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps(report))


if __name__ == "__main__":
    main()
