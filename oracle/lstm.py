"""FP64 numpy oracle of the paper's own AI inference pipeline (Sec. 3.3, Table 2).

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see ``oracle/__init__.py``).

Pipeline, in the paper's sizes:
  1. raw time series X [B, T, F]: T = 50 points of F = 6 platelet measurements
     (angular velocity components, translational and rotational kinetic energy, flow
     speed at the platelet's centre of mass),
  2. two-stage denoising: a causal moving average over MA = 5 points (fewer at the
     window start), then a one-level Haar wavelet transform per feature whose detail
     coefficients are soft-thresholded at the universal threshold of Donoho and
     Johnstone (1994), lambda = (median |d| / 0.6745) sqrt(2 ln T), and transformed
     back; then a per-feature z-score with stored statistics,
  3. autoencoder: a 2-layer LSTM encoder with 16 and 4 units; the 8 latent features
     are the last hidden and cell states of the 4-unit layer, [h_T, c_T].  The decoder
     (training only) feeds the latent vector at every step to a 2-layer LSTM with 4
     and 16 units and reads out 16 -> 6 per step; loss: mean squared reconstruction
     error,
  4. fully connected network 8 -> 32 -> 16 -> 8 -> 1 (ReLU between layers, linear
     output) predicting log2 of the MTS ratio; loss: mean squared error,
  5. categorise: ratio 2^clip(round(y), 0, 4).
The autoencoder and the FCN are trained separately (the FCN on the frozen latents).

LSTM cell (gate order i, f, g, o, as torch.nn.LSTM documents it):
  i = sig(W_ii x + b_ii + W_hi h + b_hi), f = sig(...), g = tanh(...), o = sig(...)
  c' = f * c + i * g,   h' = o * tanh(c'),   h_0 = c_0 = 0.
Parameters live in one flat float32 vector in the order of ``LAYOUT``; the forward
and backward passes use them in float32 precision, evaluated here in float64.
"""
from __future__ import annotations

import numpy as np

T = 50
F = 6
MA = 5
H1, H2 = 16, 4          # encoder units (layer 1, layer 2); the decoder mirrors them
LAT = 2 * H2            # latent: [h_T, c_T] of the second encoder layer
RATIOS = (1, 2, 4, 8, 16)


def _lstm_shapes(prefix, nin, h):
    return [(prefix + "w_ih", (4 * h, nin)), (prefix + "w_hh", (4 * h, h)),
            (prefix + "b_ih", (4 * h,)), (prefix + "b_hh", (4 * h,))]


LAYOUT = (_lstm_shapes("enc0_", F, H1) + _lstm_shapes("enc1_", H1, H2)
          + _lstm_shapes("dec0_", LAT, H2) + _lstm_shapes("dec1_", H2, H1)
          + [("out_w", (F, H1)), ("out_b", (F,))]
          + [("fc1_w", (32, LAT)), ("fc1_b", (32,)), ("fc2_w", (16, 32)), ("fc2_b", (16,)),
             ("fc3_w", (8, 16)), ("fc3_b", (8,)), ("fc4_w", (1, 8)), ("fc4_b", (1,))]
          + [("norm_mean", (F,)), ("norm_std", (F,))])
AE_NAMES = [n for n, _ in LAYOUT if n.split("_")[0] in ("enc0", "enc1", "dec0", "dec1", "out")]
FCN_NAMES = [n for n, _ in LAYOUT if n.startswith("fc")]


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
    """Uniform(-1/sqrt(fan), 1/sqrt(fan)) weights and biases (fan: the layer's hidden
    size for LSTMs, its input width for linear layers); norm = (0, 1)."""
    rng = np.random.default_rng(seed)
    d = {}
    shapes = dict(LAYOUT)
    for name, shp in LAYOUT:
        if name == "norm_mean":
            d[name] = np.zeros(shp)
        elif name == "norm_std":
            d[name] = np.ones(shp)
        else:
            if name.startswith(("enc", "dec")):
                fan = shapes[name.split("_")[0] + "_w_hh"][1]
            else:
                fan = shapes[name[:-1] + "w"][1]
            b = 1.0 / np.sqrt(fan)
            d[name] = rng.uniform(-b, b, size=shp)
    return flatten(d, np.float32)


# ---------------------------------------------------------------------------
# Step 2: two-stage denoising
# ---------------------------------------------------------------------------
def moving_average(X):
    """Causal moving average over MA points (fewer at the window start)."""
    X = np.asarray(X, dtype=np.float64)
    out = np.empty_like(X)
    for t in range(X.shape[1]):
        lo = max(0, t - MA + 1)
        out[:, t, :] = X[:, lo:t + 1, :].mean(axis=1)
    return out


def haar_denoise(X):
    """One-level Haar transform along time, soft thresholding of the details at the
    universal threshold, inverse transform.  X [B, T, F] with T even."""
    X = np.asarray(X, dtype=np.float64)
    s2 = np.sqrt(2.0)
    a = (X[:, 0::2, :] + X[:, 1::2, :]) / s2
    d = (X[:, 0::2, :] - X[:, 1::2, :]) / s2
    sigma = np.median(np.abs(d), axis=1, keepdims=True) / 0.6745
    lam = sigma * np.sqrt(2.0 * np.log(X.shape[1]))
    d = np.sign(d) * np.maximum(np.abs(d) - lam, 0.0)
    out = np.empty_like(X)
    out[:, 0::2, :] = (a + d) / s2
    out[:, 1::2, :] = (a - d) / s2
    return out


def denoise(X, mean, std):
    """Moving average, Haar wavelet denoising, z-score."""
    Y = haar_denoise(moving_average(X))
    return (Y - mean[None, None, :]) / std[None, None, :]


# ---------------------------------------------------------------------------
# LSTM layer over a sequence
# ---------------------------------------------------------------------------
def _sig(a):
    return 1.0 / (1.0 + np.exp(-a))


def lstm_forward(x, w_ih, w_hh, b_ih, b_hh):
    """x [B, T, nin] -> (hs [B, T, h], cT [B, h], cache)."""
    B, Tn, _ = x.shape
    h_units = w_hh.shape[1]
    h = np.zeros((B, h_units))
    c = np.zeros((B, h_units))
    hs = np.zeros((B, Tn, h_units))
    cache = []
    for t in range(Tn):
        a = x[:, t, :] @ w_ih.T + b_ih + h @ w_hh.T + b_hh
        i = _sig(a[:, :h_units])
        f = _sig(a[:, h_units:2 * h_units])
        g = np.tanh(a[:, 2 * h_units:3 * h_units])
        o = _sig(a[:, 3 * h_units:])
        cn = f * c + i * g
        tc = np.tanh(cn)
        cache.append((h, c, i, f, g, o, tc))
        h, c = o * tc, cn
        hs[:, t, :] = h
    return hs, c, cache


def lstm_backward(x, w_ih, w_hh, cache, dhs, dcT=None):
    """Backpropagation through time: dhs [B, T, h] is dL/dh_t from above, dcT [B, h]
    dL/dc_T.  Returns (dx, dw_ih, dw_hh, db_ih, db_hh); db_hh equals db_ih."""
    B, Tn, _ = x.shape
    h_units = w_hh.shape[1]
    dx = np.zeros_like(x)
    dw_ih = np.zeros_like(w_ih)
    dw_hh = np.zeros_like(w_hh)
    db = np.zeros(4 * h_units)
    dh = np.zeros((B, h_units))
    dc = np.zeros((B, h_units)) if dcT is None else np.array(dcT, dtype=np.float64)
    for t in range(Tn - 1, -1, -1):
        hp, cp, i, f, g, o, tc = cache[t]
        dh = dh + dhs[:, t, :]
        do = dh * tc
        dc = dc + dh * o * (1.0 - tc * tc)
        di, df, dg = dc * g, dc * cp, dc * i
        da = np.concatenate([di * i * (1.0 - i), df * f * (1.0 - f), dg * (1.0 - g * g), do * o * (1.0 - o)], axis=1)
        dw_ih += da.T @ x[:, t, :]
        dw_hh += da.T @ hp
        db += da.sum(axis=0)
        dx[:, t, :] = da @ w_ih
        dh = da @ w_hh
        dc = dc * f
    return dx, dw_ih, dw_hh, db, db.copy()


# ---------------------------------------------------------------------------
# Whole pipeline
# ---------------------------------------------------------------------------
def forward(W, X):
    """W: dict of float64 parameters; X [B, T, F] raw windows."""
    Xt = denoise(X, W["norm_mean"], W["norm_std"])
    h0, _, e0 = lstm_forward(Xt, W["enc0_w_ih"], W["enc0_w_hh"], W["enc0_b_ih"], W["enc0_b_hh"])
    h1, c1T, e1 = lstm_forward(h0, W["enc1_w_ih"], W["enc1_w_hh"], W["enc1_b_ih"], W["enc1_b_hh"])
    lat = np.concatenate([h1[:, -1, :], c1T], axis=1)
    B, Tn, _ = Xt.shape
    zin = np.repeat(lat[:, None, :], Tn, axis=1)
    d0, _, f0 = lstm_forward(zin, W["dec0_w_ih"], W["dec0_w_hh"], W["dec0_b_ih"], W["dec0_b_hh"])
    d1, _, f1 = lstm_forward(d0, W["dec1_w_ih"], W["dec1_w_hh"], W["dec1_b_ih"], W["dec1_b_hh"])
    recon = d1 @ W["out_w"].T + W["out_b"]
    a1 = lat @ W["fc1_w"].T + W["fc1_b"]
    r1 = np.maximum(a1, 0.0)
    a2 = r1 @ W["fc2_w"].T + W["fc2_b"]
    r2 = np.maximum(a2, 0.0)
    a3 = r2 @ W["fc3_w"].T + W["fc3_b"]
    r3 = np.maximum(a3, 0.0)
    y = (r3 @ W["fc4_w"].T + W["fc4_b"])[:, 0]
    cache = dict(Xt=Xt, h0=h0, e0=e0, h1=h1, e1=e1, zin=zin, d0=d0, f0=f0, d1=d1, f1=f1,
                 a1=a1, r1=r1, a2=a2, r2=r2, a3=a3, r3=r3)
    return dict(latent=lat, pred=y, recon=recon, target=Xt, cache=cache)


def loss(W, X, y_label, phase):
    """phase 0: reconstruction MSE; phase 1: MSE of the predicted log2 ratio."""
    out = forward(W, X)
    if phase == 0:
        return float(np.mean((out["recon"] - out["target"]) ** 2))
    return float(np.mean((out["pred"] - np.asarray(y_label, np.float64)) ** 2))


def backward(W, X, y_label, phase):
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
        dd0, g["dec1_w_ih"], g["dec1_w_hh"], g["dec1_b_ih"], g["dec1_b_hh"] = lstm_backward(
            c["d0"], W["dec1_w_ih"], W["dec1_w_hh"], c["f1"], dd1)
        dzin, g["dec0_w_ih"], g["dec0_w_hh"], g["dec0_b_ih"], g["dec0_b_hh"] = lstm_backward(
            c["zin"], W["dec0_w_ih"], W["dec0_w_hh"], c["f0"], dd0)
        dlat = dzin.sum(axis=1)
        dh1 = np.zeros_like(c["h1"])
        dh1[:, -1, :] = dlat[:, :H2]
        dh0, g["enc1_w_ih"], g["enc1_w_hh"], g["enc1_b_ih"], g["enc1_b_hh"] = lstm_backward(
            c["h0"], W["enc1_w_ih"], W["enc1_w_hh"], c["e1"], dh1, dcT=dlat[:, H2:])
        _, g["enc0_w_ih"], g["enc0_w_hh"], g["enc0_b_ih"], g["enc0_b_hh"] = lstm_backward(
            c["Xt"], W["enc0_w_ih"], W["enc0_w_hh"], c["e0"], dh0)
        return g
    dy = 2.0 * (out["pred"] - np.asarray(y_label, np.float64)) / B
    g["fc4_w"] = dy[None, :] @ c["r3"]
    g["fc4_b"] = np.array([dy.sum()])
    da3 = (dy[:, None] @ W["fc4_w"]) * (c["a3"] > 0)
    g["fc3_w"] = da3.T @ c["r2"]
    g["fc3_b"] = da3.sum(axis=0)
    da2 = (da3 @ W["fc3_w"]) * (c["a2"] > 0)
    g["fc2_w"] = da2.T @ c["r1"]
    g["fc2_b"] = da2.sum(axis=0)
    da1 = (da2 @ W["fc2_w"]) * (c["a1"] > 0)
    g["fc1_w"] = da1.T @ out["latent"]
    g["fc1_b"] = da1.sum(axis=0)
    return g


def categorize(y):
    """Predicted log2 ratio -> MTS ratio of the nearest allowed level."""
    return np.array(RATIOS)[np.clip(np.rint(np.asarray(y, np.float64)), 0, len(RATIOS) - 1).astype(int)]
