"""Training data, training and evaluation of the learned MTS controller (Sec. 3.3,
AI inference pipeline of Table 2), driving the library through its C ABI.

The paper labels timestep sizes by trying candidate values.  Here a
window is labelled by re-simulating from a checkpoint of its end state with every
candidate ratio r in {1, 2, 4, 8, 16} over the same simulated time, and keeping the
largest r whose time-averaged fluid peculiar temperature stays within `tol_T` (1 %) and
whose platelets keep their shape: the time-averaged eigenvalues of every platelet's
gyration tensor within `tol_shape` (2 %) of the r = 1 branch's.
The hold label is the largest hold h in {16, 32, 64, 128} outer steps over which the
ratio labels of the following windows do not drop below this window's.

Training runs on the device through the library's own forward/backward/Adam kernels:
first the autoencoder on reconstruction, then the head on the frozen latent (the
paper trains its autoencoder and predictor separately).
"""
from __future__ import annotations

import math

import numpy as np

RATIOS = (1, 2, 4, 8, 16)
HOLDS = (16, 32, 64, 128)
WINDOW = 64
STRIDE = 16


def time_average(rows, col):
    """Average of a series column over simulated time: each outer-step row stands for
    k inner steps (column 7), so rows of a variable-ratio run are weighted by their k."""
    w = rows[:, 7]
    return float(np.sum(rows[:, col] * w) / np.sum(w))


def gyration_eigenvalues(x, body, n_platelet, box_L, periodic):
    """Eigenvalues (ascending) of each platelet's gyration tensor, [P][3], from bead
    positions x [n_bead][3] (unwrapped across periodic faces from the platelet's first
    bead)."""
    L = np.asarray(box_L, np.float64)
    out = np.zeros((n_platelet, 3))
    for p in range(n_platelet):
        xs = x[body == p]
        d = xs - xs[0]
        for k in range(3):
            if periodic[k]:
                d[:, k] -= L[k] * np.round(d[:, k] / L[k])
        d -= d.mean(axis=0)
        out[p] = np.linalg.eigvalsh(d.T @ d / d.shape[0])
    return out


def _branch_stats(ctx, sysd, x, v, counters, dt, r, horizon):
    """Time-averaged fluid T_pec and per-platelet gyration eigenvalues of a branch at ratio r."""
    n_outer = max(1, int(round(horizon / (r * dt))))
    ctx.set_state(x, v)
    ctx.set_counters(*counters)
    ctx.compute_forces(dt, r)
    b0 = int(sysd["n_fluid"] + sysd["n_wall"])
    P = int(sysd["n_platelet"])
    lam = []
    chunk = max(1, n_outer // 8)
    done = 0
    while done < n_outer:
        n = min(chunk, n_outer - done)
        ctx.step(n, dt, r, diag_every=1)
        done += n
        xs, _ = ctx.state()
        lam.append(gyration_eigenvalues(xs[b0:], sysd["body"], P, sysd["box_L"], sysd["periodic"]))
    rows = ctx.series()
    return float(np.mean(rows[:, 3])), np.mean(np.array(lam), axis=0)


def ratio_label(ctx, sysd, x, v, counters, dt, horizon, tol_T=0.01, tol_shape=0.02):
    """Index into RATIOS of the largest admissible ratio (0 if none but r = 1)."""
    from .aimts import AimtsError, E_UNSTABLE
    T1, G1 = _branch_stats(ctx, sysd, x, v, counters, dt, 1, horizon)
    best = 0
    for idx, r in enumerate(RATIOS[1:], start=1):
        try:
            Tr, Gr = _branch_stats(ctx, sysd, x, v, counters, dt, r, horizon)
        except AimtsError as e:
            if e.status != E_UNSTABLE:
                raise
            break  # the step is too long for this state: not admissible
        if abs(Tr - T1) / T1 <= tol_T and np.all(np.abs(Gr - G1) / np.maximum(G1, 1e-12) <= tol_shape):
            best = idx
        else:
            break
    return best


def hold_labels(ratio_idx):
    """Hold label per window (index into HOLDS) from the ratio labels of consecutive windows."""
    out = np.zeros(len(ratio_idx), np.int32)
    for w in range(len(ratio_idx)):
        best = 0
        for hi, h in enumerate(HOLDS):
            ahead = int(math.ceil(h / STRIDE))
            nxt = ratio_idx[w + 1:w + 1 + ahead]
            if len(nxt) == ahead and np.all(nxt >= ratio_idx[w]):
                best = hi
        out[w] = best
    return out


def generate(make_ctx, workload, g_values, windows_per_traj, dt=0.0025, k_run=(4, 8), horizon=None, equil=200,
             label_every=1, log=print):
    """Run one trajectory per body force in `g_values`, collect feature windows every STRIDE
    outer steps and label them.  The trajectories record their windows at the ratios the
    controller runs at (k_run, taken in turn: the fallback 4 and the cap 8), since one
    feature row is written per outer step whatever its ratio.

    make_ctx(sysd, series_capacity) -> library context; workload(g) -> workload dict.
    Returns (windows [n, 64, 8] float32, labels [n, 2] int32, meta list)."""
    horizon = horizon if horizon is not None else WINDOW * 4 * dt
    ks = tuple(k_run) if hasattr(k_run, "__len__") else (int(k_run),)
    X, Y, meta = [], [], []
    for ti, g in enumerate(g_values):
        k_tr = ks[ti % len(ks)]
        d = workload(g)
        n_branch_rows = int(round(horizon / dt)) + 8
        run = make_ctx(d, 16)
        brn = make_ctx(d, n_branch_rows)
        run.compute_forces(dt, 1)
        run.step(equil, dt, 1)
        run.compute_forces(dt, k_tr)
        run.step(WINDOW, dt, k_tr)
        wins, ridx = [], []
        for w in range(windows_per_traj):
            wins.append(run.feature_window().copy())
            if w % label_every == 0:
                x, v = run.state()
                cnt = run.counters()
                ridx.append(ratio_label(brn, d, x, v, cnt, dt, horizon))
            else:
                ridx.append(ridx[-1])
            run.step(STRIDE, dt, k_tr)
        ridx = np.array(ridx, np.int32)
        hidx = hold_labels(ridx)
        P = wins[0].shape[0]
        for w, win in enumerate(wins):
            for p in range(P):
                X.append(win[p])
                Y.append((ridx[w], hidx[w]))
                meta.append((ti, g, w, p))
        log("trajectory %d (g=%.4f, windows at k=%d): ratio labels %s" % (ti, g, k_tr,
                                                                        np.bincount(ridx, minlength=5).tolist()))
        run.close()
        brn.close()
    return np.array(X, np.float32), np.array(Y, np.int32), meta


def init_params(seed=0):
    """Initial parameter vector (uniform +-1/sqrt(fan in), like torch's GRU/Linear)."""
    from . import aimts as A
    n = A.Context.ctrl_num_params()
    rng = np.random.default_rng(seed)
    return (rng.uniform(-1.0, 1.0, n) / math.sqrt(64.0)).astype(np.float32)


def set_norm(params, windows):
    """Store per-feature mean/std of the moving-averaged training windows in the
    normalisation slots (the last 16 parameters)."""
    p = params.copy()
    ma = np.empty_like(windows, dtype=np.float64)
    for t in range(windows.shape[1]):
        lo = max(0, t - 4)
        ma[:, t, :] = windows[:, lo:t + 1, :].mean(axis=1)
    mean = ma.reshape(-1, windows.shape[2]).mean(axis=0)
    std = ma.reshape(-1, windows.shape[2]).std(axis=0)
    std[std < 1e-6] = 1.0
    p[-16:-8] = mean
    p[-8:] = std
    return p


def train(ctx, windows, labels, ae_steps=400, head_steps=600, batch=256, lr_ae=2e-3, lr_head=5e-3, seed=0,
          log=print):
    """Two-phase training on the device.  Returns the loss histories."""
    import torch
    rng = np.random.default_rng(seed)
    n = windows.shape[0]
    dW = torch.from_numpy(np.ascontiguousarray(windows)).cuda()
    dY = torch.from_numpy(np.ascontiguousarray(labels)).cuda()
    hist = {"ae": [], "head": []}
    for phase, steps, lr, key in ((0, ae_steps, lr_ae, "ae"), (1, head_steps, lr_head, "head")):
        for it in range(steps):
            idx = torch.from_numpy(rng.choice(n, size=min(batch, n), replace=False)).cuda()
            xb = dW.index_select(0, idx).contiguous()
            yb = dY.index_select(0, idx).contiguous()
            hist[key].append(ctx.ctrl_train_step(xb, yb if phase == 1 else None, phase, lr))
            if it % 100 == 0:
                log("phase %d step %d loss %.4f" % (phase, it, hist[key][-1]))
    return hist


def predict(ctx, windows, batch=256):
    """(ratio index, hold index) per window from the device forward pass."""
    import torch
    out_r, out_h = [], []
    for s in range(0, windows.shape[0], batch):
        xb = torch.from_numpy(np.ascontiguousarray(windows[s:s + batch])).cuda()
        lg = torch.zeros((xb.shape[0], 9), device="cuda")
        ctx.ctrl_forward(xb, None, lg)
        lg = lg.cpu().numpy()
        out_r.append(np.argmax(lg[:, :5], axis=1))
        out_h.append(np.argmax(lg[:, 5:], axis=1))
    return np.concatenate(out_r), np.concatenate(out_h)
