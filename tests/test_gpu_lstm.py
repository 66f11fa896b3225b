"""The paper's own inference pipeline (Sec. 3.3, Table 2) on the HIP path, through the C
ABI, against the oracle (oracle/lstm.py, float64): the two-stage filter, the forward
pass (latents, prediction, reconstruction), the gradients of both training phases per
tensor, an Adam step, and bitwise determinism.  The kernels run in float32."""
import numpy as np
import pytest

from oracle import gru as gru_oracle
from oracle import lstm as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14121_amd.aimts as A
    return A


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def _case(B=24, seed=0):
    rng = np.random.default_rng(seed)
    # windows with a trend, an oscillation and noise per feature, on the measurements' scales
    t = np.arange(O.T)[None, :, None]
    scale = np.array([0.2, 0.3, 0.1, 2.0, 0.5, 1.5])
    X = (rng.standard_normal((B, 1, O.F)) + 0.02 * t * rng.standard_normal((B, 1, O.F))
         + 0.5 * np.sin(0.4 * t + rng.uniform(0, 6, (B, 1, O.F))) + 0.3 * rng.standard_normal((B, O.T, O.F))) * scale
    p = O.init_params(seed + 1)
    W = O.unflatten(p)
    W["norm_mean"] = np.array([0.01, -0.02, 0.0, 0.3, 0.05, 0.2])
    W["norm_std"] = np.array([0.2, 0.3, 0.1, 2.0, 0.5, 1.5])
    p = O.flatten(W, np.float32)
    y = rng.uniform(0.0, 4.0, B)
    return X.astype(np.float32), p, y.astype(np.float32)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_filter_matches_oracle(A):
    X, p, _ = _case()
    net = A.LstmPipeline(64)
    out = net.filter(_dev(p), _dev(X)).cpu().numpy()
    W = O.unflatten(p)
    ref = O.denoise(X.astype(np.float64), W["norm_mean"], W["norm_std"])
    err = rel_l2(out, ref)
    print("filter rel L2 %.2e" % err)
    assert err <= 1e-6


def test_forward_matches_oracle(A):
    X, p, _ = _case()
    net = A.LstmPipeline(64)
    lat, pred, rec = net.forward(_dev(p), _dev(X), recon=True)
    ref = O.forward(O.unflatten(p), X.astype(np.float64))
    e = [rel_l2(lat.cpu().numpy(), ref["latent"]), rel_l2(pred.cpu().numpy(), ref["pred"]),
         rel_l2(rec.cpu().numpy(), ref["recon"])]
    print("forward rel L2: latent %.2e pred %.2e recon %.2e" % tuple(e))
    assert max(e) <= 1e-5
    assert np.array_equal(O.categorize(pred.cpu().numpy()), O.categorize(ref["pred"]))


@pytest.mark.parametrize("phase", [0, 1])
def test_gradients_match_oracle(A, phase):
    X, p, y = _case(B=16, seed=3)
    net = A.LstmPipeline(64)
    g, loss = net.backward(_dev(p), _dev(X), _dev(y), phase)
    g = g.cpu().numpy()
    W = O.unflatten(p)
    ref = O.backward(W, X.astype(np.float64), y.astype(np.float64), phase)
    ref_loss = O.loss(W, X.astype(np.float64), y.astype(np.float64), phase)
    assert float(loss.cpu()[0]) == pytest.approx(ref_loss, rel=1e-5)
    gd = O.unflatten(g)
    names = O.AE_NAMES if phase == 0 else O.FCN_NAMES
    worst = 0.0
    for name in names:
        e = rel_l2(gd[name], ref[name])
        worst = max(worst, e)
        assert e <= 1e-3, name
    for name in (O.FCN_NAMES if phase == 0 else O.AE_NAMES):
        assert np.all(gd[name] == 0.0)
    print("phase %d: worst per-tensor gradient rel L2 %.2e, loss %.6g" % (phase, worst, ref_loss))
    # deterministic: a second call gives the same bits
    g2, _ = net.backward(_dev(p), _dev(X), _dev(y), phase)
    assert np.array_equal(g, g2.cpu().numpy())


def test_adam_step_matches_oracle(A):
    import torch
    X, p, y = _case(B=8, seed=5)
    net = A.LstmPipeline(16)
    pd, g = _dev(p), None
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    g, _ = net.backward(pd, _dev(X), _dev(y), 1)
    gh = g.cpu().numpy().astype(np.float64)
    net.adam(pd, m, v, g, 1, 1, 1e-3)
    L = O.unflatten(np.arange(O.n_params()))
    lo, hi = int(L["fc1_w"].reshape(-1)[0]), int(L["fc4_b"].reshape(-1)[0]) + 1
    ref, _, _ = gru_oracle.adam_step(p.astype(np.float64)[lo:hi], gh[lo:hi], np.zeros(hi - lo), np.zeros(hi - lo), 1,
                                     1e-3)
    got = pd.cpu().numpy()
    assert np.allclose(got[lo:hi], ref, rtol=1e-6, atol=1e-7)
    assert np.array_equal(got[:lo], p[:lo]) and np.array_equal(got[hi:], p[hi:])
