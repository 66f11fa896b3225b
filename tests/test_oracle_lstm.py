"""Pins of the oracle of the paper's own inference pipeline (Sec. 3.3, Table 2): MA +
Haar wavelet denoising, the 2-layer LSTM autoencoder (16 and 4 units, 8 latents) and
the FCN 32-16-8-1.  torch.nn.LSTM in float64 on the CPU is the library routine for the
LSTM equations (forward and autograd); central finite differences check every
backward pass of the whole pipeline; the wavelet stage is checked against the
orthogonality of the Haar transform, a hand-worked universal threshold and the exact
removal of a pure alternating component."""
import numpy as np
import pytest
import torch

from oracle import lstm


def _rand_windows(B, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, lstm.T, lstm.F)) * np.array([0.2, 0.3, 0.1, 2.0, 0.5, 1.5])


def test_layout_sizes():
    def lstm_n(nin, h):
        return 4 * h * (nin + h + 2)
    ae = lstm_n(6, 16) + lstm_n(16, 4) + lstm_n(8, 4) + lstm_n(4, 16) + 6 * 17
    fcn = 32 * 9 + 16 * 33 + 8 * 17 + 1 * 9
    assert lstm.n_params() == ae + fcn + 12
    assert lstm.LAT == 8 and (lstm.T, lstm.F) == (50, 6)


@pytest.mark.parametrize("nin,h", [(6, 16), (16, 4), (8, 4)])
def test_lstm_layer_matches_torch_float64(nin, h):
    rng = np.random.default_rng(1)
    B = 4
    x = rng.standard_normal((B, 20, nin))
    m = torch.nn.LSTM(nin, h, num_layers=1, batch_first=True).double()
    with torch.no_grad():
        for p in m.parameters():
            p.copy_(torch.from_numpy(rng.uniform(-0.5, 0.5, size=tuple(p.shape))))
    xt = torch.from_numpy(x).requires_grad_(True)
    ref, (hT, cT) = m(xt)
    w = [m.weight_ih_l0, m.weight_hh_l0, m.bias_ih_l0, m.bias_hh_l0]
    hs, c, cache = lstm.lstm_forward(x, *[t.detach().numpy() for t in w])
    assert np.max(np.abs(hs - ref.detach().numpy())) < 1e-13
    assert np.max(np.abs(c - cT[0].detach().numpy())) < 1e-13
    dhs = rng.standard_normal(hs.shape)
    dcT = rng.standard_normal(c.shape)
    ((ref * torch.from_numpy(dhs)).sum() + (cT[0] * torch.from_numpy(dcT)).sum()).backward()
    dx, dwi, dwh, dbi, dbh = lstm.lstm_backward(x, w[0].detach().numpy(), w[1].detach().numpy(), cache, dhs, dcT)
    assert np.max(np.abs(dx - xt.grad.numpy())) < 1e-12
    for mine, t in ((dwi, w[0]), (dwh, w[1]), (dbi, w[2]), (dbh, w[3])):
        assert np.max(np.abs(mine - t.grad.numpy())) < 1e-12


@pytest.mark.parametrize("phase", [0, 1])
def test_pipeline_gradient_by_finite_differences(phase):
    W = lstm.unflatten(lstm.init_params(3).astype(np.float64))
    W["norm_mean"] = np.full(6, 0.1)
    W["norm_std"] = np.full(6, 1.3)
    X = _rand_windows(3, seed=4)
    y = np.array([1.0, 2.7, 3.2])
    g = lstm.backward(W, X, y, phase)
    names = lstm.AE_NAMES if phase == 0 else lstm.FCN_NAMES
    rng = np.random.default_rng(6)
    for name in names:
        flat = W[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(4, flat.size), replace=False)
        for q in idx:
            old = flat[q]
            h = 1e-6
            flat[q] = old + h
            lp = lstm.loss(W, X, y, phase)
            flat[q] = old - h
            lm = lstm.loss(W, X, y, phase)
            flat[q] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[q]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), name
    # the other phase's parameters get no gradient
    for name in (lstm.FCN_NAMES if phase == 0 else lstm.AE_NAMES):
        assert np.all(g[name] == 0.0)


def test_haar_stage_is_orthogonal_and_thresholds_by_hand():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((2, lstm.T, lstm.F))
    s2 = np.sqrt(2.0)
    a = (X[:, 0::2] + X[:, 1::2]) / s2
    d = (X[:, 0::2] - X[:, 1::2]) / s2
    # Parseval: the one-level Haar transform preserves the energy
    assert np.allclose((a ** 2).sum(axis=1) + (d ** 2).sum(axis=1), (X ** 2).sum(axis=1), rtol=1e-13)
    # a hand-worked universal threshold on one series: details 0.1 k for k = 1..25,
    # median |d| = 1.3, sigma = 1.3 / 0.6745 = 1.92735, sqrt(2 ln 50) = 2.79715, lambda = 5.39110
    x = np.zeros((1, lstm.T, 1))
    dd = 0.1 * np.arange(1, 26)
    x[0, 0::2, 0] = dd / s2
    x[0, 1::2, 0] = -dd / s2
    lam = 1.3 / 0.6745 * np.sqrt(2.0 * np.log(50.0))
    assert lam == pytest.approx(5.39110, rel=1e-5)
    out = lstm.haar_denoise(x)
    # no detail exceeds lambda: every pair collapses to its mean, here 0
    assert np.allclose(out, 0.0, atol=1e-15)
    # scale the last detail past lambda: it keeps |d| - lambda
    x[0, 48, 0], x[0, 49, 0] = 10.0 / s2, -10.0 / s2
    out = lstm.haar_denoise(x)
    keep = 10.0 - lam
    assert out[0, 48, 0] == pytest.approx(keep / s2, rel=1e-12)
    assert out[0, 49, 0] == pytest.approx(-keep / s2, rel=1e-12)


def test_denoise_removes_a_pure_alternating_component_and_keeps_constants():
    B = 2
    const = np.full((B, lstm.T, lstm.F), 2.5)
    assert np.allclose(lstm.haar_denoise(const), 2.5, atol=1e-14)
    assert np.allclose(lstm.denoise(const, np.full(6, 0.5), np.full(6, 2.0)), 1.0, atol=1e-14)
    alt = const + 0.3 * (-1.0) ** np.arange(lstm.T)[None, :, None]
    # every detail has the same size, so all lie below the universal threshold
    assert np.allclose(lstm.haar_denoise(alt), 2.5, atol=1e-14)


def test_categorize_and_zero_fcn():
    assert list(lstm.categorize([-0.7, 0.4, 1.6, 2.5, 3.49, 9.0])) == [1, 1, 4, 4, 8, 16]
    W = lstm.unflatten(lstm.init_params(1).astype(np.float64))
    for name in lstm.FCN_NAMES:
        W[name] = np.zeros_like(W[name])
    W["fc4_b"] = np.array([2.25])
    out = lstm.forward(W, _rand_windows(3))
    assert np.all(out["pred"] == 2.25)
