"""FP64 numpy oracle of the learned MTS controller (AI inference pipeline, Table 2).

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see ``oracle/__init__.py``).

Pipeline of the paper's Table 2 with the sizes used here:
  1. raw per-platelet features X [B, T, 8] (time series),
  2. denoise: causal moving average over ``MA`` points (truncated at the window
     start), then a per-feature z-score with stored mean/std,
  3. autoencoder: 2-layer GRU encoder (hidden 64) over the T steps, a linear map
     of the last top-layer state to 16 latent features; a 2-layer GRU decoder
     fed the latent vector at every step and a linear read-out 64 -> 8
     reconstructs the denoised window (training only),
  4. fully connected head 16 -> 32 -> 16 -> 8 (ReLU) -> 9 logits:
     5 over the MTS ratio {1, 2, 4, 8, 16} and 4 over the hold {16, 32, 64, 128},
  5. categorise: argmax of each group.

GRU cell (gate order r, z, n; "reset after the recurrent product"):
  r = sig(W_ir x + b_ir + W_hr h + b_hr)
  z = sig(W_iz x + b_iz + W_hz h + b_hz)
  n = tanh(W_in x + b_in + r * (W_hn h + b_hn))
  h' = (1 - z) * n + z * h,            h_0 = 0.
Losses: mean squared reconstruction error over [B, T, 8] (autoencoder phase);
cross-entropy of both heads averaged over the batch (head phase, latent frozen).
Adam: beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected.

Parameters live in one flat float32 vector in the order of ``LAYOUT``.
"""
from __future__ import annotations

import numpy as np

H = 64
F = 8
LAT = 16
T = 64
MA = 5
RATIOS = (1, 2, 4, 8, 16)
HOLDS = (16, 32, 64, 128)
NOUT = len(RATIOS) + len(HOLDS)


def _gru_shapes(prefix, nin):
    return [(prefix + "w_ih", (3 * H, nin)), (prefix + "w_hh", (3 * H, H)),
            (prefix + "b_ih", (3 * H,)), (prefix + "b_hh", (3 * H,))]


LAYOUT = (_gru_shapes("enc0_", F) + _gru_shapes("enc1_", H) + [("lat_w", (LAT, H)), ("lat_b", (LAT,))]
          + _gru_shapes("dec0_", LAT) + _gru_shapes("dec1_", H) + [("out_w", (F, H)), ("out_b", (F,))]
          + [("h1_w", (32, LAT)), ("h1_b", (32,)), ("h2_w", (16, 32)), ("h2_b", (16,)),
             ("h3_w", (8, 16)), ("h3_b", (8,)), ("h4_w", (NOUT, 8)), ("h4_b", (NOUT,))]
          + [("norm_mean", (F,)), ("norm_std", (F,))])
AE_NAMES = [n for n, _ in LAYOUT if n.split("_")[0] in ("enc0", "enc1", "lat", "dec0", "dec1", "out")]
HEAD_NAMES = [n for n, _ in LAYOUT if n.startswith("h") and n[1].isdigit()]


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in LAYOUT))


def unflatten(vec):
    out, o = {}, 0
    for name, shp in LAYOUT:
        m = int(np.prod(shp))
        out[name] = np.asarray(vec[o:o + m], dtype=np.float64).reshape(shp)
        o += m
    return out


def flatten(d, dtype=np.float64):
    return np.concatenate([np.asarray(d[name], dtype=dtype).reshape(-1) for name, _ in LAYOUT])


def init_params(seed: int = 0) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases; norm = (0, 1)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in LAYOUT:
        if name == "norm_mean":
            d[name] = np.zeros(shp)
        elif name == "norm_std":
            d[name] = np.ones(shp)
        else:
            fan = H if name.startswith(("enc", "dec")) else (shp[1] if len(shp) == 2 else None)
            if fan is None:  # bias of a linear layer: fan-in of its weight
                fan = dict(LAYOUT)[name[:-1] + "w"][1]
            b = 1.0 / np.sqrt(fan)
            d[name] = rng.uniform(-b, b, size=shp)
    return flatten(d, np.float32)


def bf16_round(a) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even), returned as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    nan = np.isnan(a)
    out = r.view(np.float32).copy()
    out[nan] = np.nan
    return out


def weights_for_compute(vec) -> np.ndarray:
    """Network weights as used in the forward/backward pass: every parameter rounded
    to bfloat16 except the normalisation statistics, which stay float32."""
    d = unflatten(np.asarray(vec, np.float32))
    for name in d:
        if not name.startswith("norm_"):
            d[name] = bf16_round(d[name].astype(np.float32)).astype(np.float64)
    return d


# ---------------------------------------------------------------------------
# Step 2: denoising
# ---------------------------------------------------------------------------
def denoise(X, mean, std):
    """Causal moving average over MA points (fewer at the window start), then z-score."""
    X = np.asarray(X, dtype=np.float64)
    out = np.empty_like(X)
    for t in range(X.shape[1]):
        lo = max(0, t - MA + 1)
        out[:, t, :] = X[:, lo:t + 1, :].mean(axis=1)
    return (out - mean[None, None, :]) / std[None, None, :]


# ---------------------------------------------------------------------------
# GRU layer forward/backward over a sequence
# ---------------------------------------------------------------------------
def _sig(a):
    return 1.0 / (1.0 + np.exp(-a))


def gru_forward(x, w_ih, w_hh, b_ih, b_hh):
    """x [B, T, nin] -> hs [B, T, H] plus a cache for the backward pass."""
    B, Tn, _ = x.shape
    h = np.zeros((B, H))
    hs = np.zeros((B, Tn, H))
    cache = []
    for t in range(Tn):
        gi = x[:, t, :] @ w_ih.T + b_ih
        gh = h @ w_hh.T + b_hh
        r = _sig(gi[:, :H] + gh[:, :H])
        z = _sig(gi[:, H:2 * H] + gh[:, H:2 * H])
        n = np.tanh(gi[:, 2 * H:] + r * gh[:, 2 * H:])
        hn = (1.0 - z) * n + z * h
        cache.append((h, r, z, n, gh[:, 2 * H:]))
        h = hn
        hs[:, t, :] = h
    return hs, cache


def gru_backward(x, w_ih, w_hh, cache, dhs):
    """Backpropagation through time.  dhs [B, T, H] is dL/dh_t from above.
    Returns (dx, dw_ih, dw_hh, db_ih, db_hh)."""
    B, Tn, nin = x.shape
    dx = np.zeros_like(x)
    dw_ih = np.zeros_like(w_ih)
    dw_hh = np.zeros_like(w_hh)
    db_ih = np.zeros(3 * H)
    db_hh = np.zeros(3 * H)
    dh = np.zeros((B, H))
    for t in range(Tn - 1, -1, -1):
        hp, r, z, n, ghn = cache[t]
        dh = dh + dhs[:, t, :]
        dn = dh * (1.0 - z)
        dz = dh * (hp - n)
        dhp = dh * z
        dan = dn * (1.0 - n * n)           # d pre-activation of n
        dar = dan * ghn * r * (1.0 - r)    # d pre-activation of r
        daz = dz * z * (1.0 - z)
        dgi = np.concatenate([dar, daz, dan], axis=1)
        dgh = np.concatenate([dar, daz, dan * r], axis=1)
        dw_ih += dgi.T @ x[:, t, :]
        db_ih += dgi.sum(axis=0)
        dw_hh += dgh.T @ hp
        db_hh += dgh.sum(axis=0)
        dx[:, t, :] = dgi @ w_ih
        dh = dhp + dgh @ w_hh
    return dx, dw_ih, dw_hh, db_ih, db_hh


# ---------------------------------------------------------------------------
# Whole network
# ---------------------------------------------------------------------------
def forward(W, X):
    """W: dict of float64 parameters; X [B, T, 8] raw windows.
    Returns dict with latent [B,16], logits [B,9], recon [B,T,8], target [B,T,8], cache."""
    Xt = denoise(X, W["norm_mean"], W["norm_std"])
    h0, c0 = gru_forward(Xt, W["enc0_w_ih"], W["enc0_w_hh"], W["enc0_b_ih"], W["enc0_b_hh"])
    h1, c1 = gru_forward(h0, W["enc1_w_ih"], W["enc1_w_hh"], W["enc1_b_ih"], W["enc1_b_hh"])
    hT = h1[:, -1, :]
    lat = hT @ W["lat_w"].T + W["lat_b"]
    B, Tn, _ = Xt.shape
    zin = np.repeat(lat[:, None, :], Tn, axis=1)
    d0, e0 = gru_forward(zin, W["dec0_w_ih"], W["dec0_w_hh"], W["dec0_b_ih"], W["dec0_b_hh"])
    d1, e1 = gru_forward(d0, W["dec1_w_ih"], W["dec1_w_hh"], W["dec1_b_ih"], W["dec1_b_hh"])
    recon = d1 @ W["out_w"].T + W["out_b"]
    a1 = lat @ W["h1_w"].T + W["h1_b"]
    r1 = np.maximum(a1, 0.0)
    a2 = r1 @ W["h2_w"].T + W["h2_b"]
    r2 = np.maximum(a2, 0.0)
    a3 = r2 @ W["h3_w"].T + W["h3_b"]
    r3 = np.maximum(a3, 0.0)
    logits = r3 @ W["h4_w"].T + W["h4_b"]
    cache = dict(Xt=Xt, h0=h0, c0=c0, h1=h1, c1=c1, zin=zin, d0=d0, e0=e0, d1=d1, e1=e1,
                 a1=a1, r1=r1, a2=a2, r2=r2, a3=a3, r3=r3)
    return dict(latent=lat, logits=logits, recon=recon, target=Xt, cache=cache)


def _softmax(a):
    a = a - a.max(axis=1, keepdims=True)
    e = np.exp(a)
    return e / e.sum(axis=1, keepdims=True)


def loss(W, X, labels, phase):
    """phase 0: reconstruction MSE; phase 1: CE(ratio) + CE(hold).  labels [B, 2] class indices."""
    out = forward(W, X)
    if phase == 0:
        return float(np.mean((out["recon"] - out["target"]) ** 2))
    lg = out["logits"]
    nr = len(RATIOS)
    pr = _softmax(lg[:, :nr])
    ph = _softmax(lg[:, nr:])
    B = lg.shape[0]
    return float(-np.mean(np.log(pr[np.arange(B), labels[:, 0]])) - np.mean(np.log(ph[np.arange(B), labels[:, 1]])))


def backward(W, X, labels, phase):
    """Gradients (dict, same keys as W; zero for parameters the phase does not train)."""
    out = forward(W, X)
    c = out["cache"]
    g = {k: np.zeros_like(v) for k, v in W.items()}
    B, Tn, _ = out["target"].shape
    if phase == 0:
        dre = 2.0 * (out["recon"] - out["target"]) / (B * Tn * F)
        g["out_w"] = np.einsum("bto,bth->oh", dre, c["d1"])
        g["out_b"] = dre.sum(axis=(0, 1))
        dd1 = dre @ W["out_w"]
        dd0, g["dec1_w_ih"], g["dec1_w_hh"], g["dec1_b_ih"], g["dec1_b_hh"] = gru_backward(
            c["d0"], W["dec1_w_ih"], W["dec1_w_hh"], c["e1"], dd1)
        dzin, g["dec0_w_ih"], g["dec0_w_hh"], g["dec0_b_ih"], g["dec0_b_hh"] = gru_backward(
            c["zin"], W["dec0_w_ih"], W["dec0_w_hh"], c["e0"], dd0)
        dlat = dzin.sum(axis=1)
        hT = c["h1"][:, -1, :]
        g["lat_w"] = dlat.T @ hT
        g["lat_b"] = dlat.sum(axis=0)
        dh1 = np.zeros_like(c["h1"])
        dh1[:, -1, :] = dlat @ W["lat_w"]
        dh0, g["enc1_w_ih"], g["enc1_w_hh"], g["enc1_b_ih"], g["enc1_b_hh"] = gru_backward(
            c["h0"], W["enc1_w_ih"], W["enc1_w_hh"], c["c1"], dh1)
        _, g["enc0_w_ih"], g["enc0_w_hh"], g["enc0_b_ih"], g["enc0_b_hh"] = gru_backward(
            c["Xt"], W["enc0_w_ih"], W["enc0_w_hh"], c["c0"], dh0)
        return g
    lg = out["logits"]
    nr = len(RATIOS)
    dlg = np.zeros_like(lg)
    pr = _softmax(lg[:, :nr])
    ph = _softmax(lg[:, nr:])
    pr[np.arange(B), labels[:, 0]] -= 1.0
    ph[np.arange(B), labels[:, 1]] -= 1.0
    dlg[:, :nr] = pr / B
    dlg[:, nr:] = ph / B
    g["h4_w"] = dlg.T @ c["r3"]
    g["h4_b"] = dlg.sum(axis=0)
    da3 = (dlg @ W["h4_w"]) * (c["a3"] > 0)
    g["h3_w"] = da3.T @ c["r2"]
    g["h3_b"] = da3.sum(axis=0)
    da2 = (da3 @ W["h3_w"]) * (c["a2"] > 0)
    g["h2_w"] = da2.T @ c["r1"]
    g["h2_b"] = da2.sum(axis=0)
    da1 = (da2 @ W["h2_w"]) * (c["a1"] > 0)
    g["h1_w"] = da1.T @ out["latent"]
    g["h1_b"] = da1.sum(axis=0)
    return g


def adam_step(p, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma & Ba); step counts from 1.  Returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(W, X):
    """(ratio, hold) per window from the argmax of each logit group."""
    lg = forward(W, X)["logits"]
    nr = len(RATIOS)
    return (np.array(RATIOS)[np.argmax(lg[:, :nr], axis=1)], np.array(HOLDS)[np.argmax(lg[:, nr:], axis=1)])
