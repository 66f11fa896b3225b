"""Pins of the controller oracle (AI inference pipeline, Table 2): torch.nn.GRU in
float64 on the CPU as the library routine for the GRU equations, central finite
differences for every backward pass, Adam's closed-form first step, torch's
bfloat16 rounding and the moving-average filter's exact responses."""
import numpy as np
import pytest
import torch

from oracle import gru


def _rand_windows(B, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, gru.T, gru.F)) * np.array([1, 1, 1, 0.5, 2, 0.1, 3, 1.0])


def test_layout_sizes():
    # 2-layer GRU encoder/decoder (hidden 64, latent 16), read-out 64->8, head 16-32-16-8-9, norm stats
    ae = 3 * 64 * (8 + 64 + 2) + 3 * 64 * (64 + 64 + 2) + 16 * 65 + 3 * 64 * (16 + 64 + 2) + 3 * 64 * (64 + 64 + 2) + 8 * 65
    head = 32 * 17 + 16 * 33 + 8 * 17 + 9 * 9
    assert gru.n_params() == ae + head + 16


def test_gru_layer_matches_torch_float64():
    rng = np.random.default_rng(1)
    B, nin = 5, 8
    x = rng.standard_normal((B, 20, nin))
    g = torch.nn.GRU(nin, gru.H, num_layers=1, batch_first=True).double()
    with torch.no_grad():
        for p in g.parameters():
            p.copy_(torch.from_numpy(rng.uniform(-0.3, 0.3, size=tuple(p.shape))))
    xt = torch.from_numpy(x).requires_grad_(True)
    ref, _ = g(xt)
    hs, cache = gru.gru_forward(x, g.weight_ih_l0.detach().numpy(), g.weight_hh_l0.detach().numpy(),
                                g.bias_ih_l0.detach().numpy(), g.bias_hh_l0.detach().numpy())
    assert np.max(np.abs(hs - ref.detach().numpy())) < 1e-13
    dhs = rng.standard_normal(hs.shape)
    (ref * torch.from_numpy(dhs)).sum().backward()
    dx, dwi, dwh, dbi, dbh = gru.gru_backward(x, g.weight_ih_l0.detach().numpy(), g.weight_hh_l0.detach().numpy(),
                                              cache, dhs)
    assert np.max(np.abs(dx - xt.grad.numpy())) < 1e-12
    assert np.max(np.abs(dwi - g.weight_ih_l0.grad.numpy())) < 1e-12
    assert np.max(np.abs(dwh - g.weight_hh_l0.grad.numpy())) < 1e-12
    assert np.max(np.abs(dbi - g.bias_ih_l0.grad.numpy())) < 1e-12
    assert np.max(np.abs(dbh - g.bias_hh_l0.grad.numpy())) < 1e-12


def test_zero_weights_keep_state_zero():
    x = np.random.default_rng(2).standard_normal((3, 10, 8))
    z = np.zeros((192, 8))
    hs, _ = gru.gru_forward(x, z, np.zeros((192, 64)), np.zeros(192), np.zeros(192))
    # r = z = 1/2, n = 0 -> h stays 0
    assert np.all(hs == 0.0)


@pytest.mark.parametrize("phase", [0, 1])
def test_network_gradient_by_finite_differences(phase):
    W = gru.unflatten(gru.init_params(3).astype(np.float64))
    W["norm_mean"] = np.full(8, 0.1)
    W["norm_std"] = np.full(8, 1.3)
    X = _rand_windows(3, seed=4)[:, :, :]
    labels = np.array([[0, 3], [4, 1], [2, 2]])
    g = gru.backward(W, X, labels, phase)
    names = gru.AE_NAMES if phase == 0 else gru.HEAD_NAMES
    rng = np.random.default_rng(5)
    h = 1e-6
    for name in names:
        flat = W[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = gru.loss(W, X, labels, phase)
            flat[idx] = old - h
            lm = gru.loss(W, X, labels, phase)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (name, idx, fd, an)
    other = gru.HEAD_NAMES if phase == 0 else gru.AE_NAMES
    assert all(np.all(g[n] == 0.0) for n in other)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    gr = np.array([0.3, -4.0, 1e-3])
    p1, m, v = gru.adam_step(p, gr, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, p - 0.01 * gr / (np.abs(gr) + 1e-8), rtol=0, atol=1e-15)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(6)
    a = np.concatenate([rng.standard_normal(10000).astype(np.float32),
                        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 3.0e38, 1e-40], np.float32)])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(gru.bf16_round(a), ref)
    assert gru.bf16_round(np.float32(1 + 2 ** -8)) == 1.0
    assert gru.bf16_round(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)


def test_denoise_filter_responses():
    B = 2
    const = np.full((B, gru.T, gru.F), 2.5)
    out = gru.denoise(const, np.full(8, 0.5), np.full(8, 2.0))
    assert np.allclose(out, 1.0, atol=1e-15)
    ramp = np.broadcast_to(np.arange(gru.T, dtype=float)[None, :, None], (B, gru.T, gru.F))
    out = gru.denoise(ramp, np.zeros(8), np.ones(8))
    # interior: a causal average of 5 points of a unit ramp lags it by 2
    assert np.allclose(out[:, gru.MA - 1:, :], ramp[:, gru.MA - 1:, :] - 2.0, atol=1e-13)
    assert np.allclose(out[:, 1, :], 0.5)
