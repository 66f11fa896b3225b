"""Host-side pieces of the controller's training (CPU): the normalisation statistics
follow the same moving-average filter as the oracle's denoising stage, and the shape
criterion of the labels is the gyration tensor's spectrum."""
import numpy as np

from oracle import gru
from paper_2205_14121_amd import controller as ctl


def test_norm_statistics_follow_the_oracles_filter():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(37, 64, 8)) * np.array([1, 2, 3, 0.1, 40, 0.01, 5, 20.0])
    p = ctl.set_norm(np.zeros(gru.n_params(), np.float32), X.astype(np.float32))
    ma = gru.denoise(X.astype(np.float32), np.zeros(8), np.ones(8)).reshape(-1, 8)
    assert np.allclose(p[-16:-8], ma.mean(axis=0), rtol=1e-5, atol=1e-6)
    assert np.allclose(p[-8:], ma.std(axis=0), rtol=1e-5, atol=1e-6)


def test_gyration_eigenvalues_of_an_ellipsoid_shell_across_a_periodic_face():
    """Points of a sphere of radius R: each eigenvalue R^2/3; scaled by (a, b, c): a^2 R^2/3
    etc.; the platelet straddles the periodic x face and is rotated."""
    import synth
    tm = synth.platelet_template(level=4, semi_axes=(3.0, 1.0, 3.0))
    rest = tm["rest"]
    lam_rest = np.sort(np.linalg.eigvalsh(np.cov(rest.T, bias=True)))
    R = synth.random_rotation(np.random.default_rng(2))
    x = rest @ R.T + np.array([9.5, 5.0, 5.0])
    x[:, 0] = np.mod(x[:, 0], 10.0)
    body = np.zeros(x.shape[0], np.int32)
    lam = ctl.gyration_eigenvalues(x, body, 1, (10.0, 10.0, 10.0), (1, 0, 1))[0]
    assert np.allclose(lam, lam_rest, rtol=1e-12)
    # a uniformly dense sphere surface: R^2 / 3 each, to the mesh's discreteness
    tm_s = synth.platelet_template(level=4, semi_axes=(2.0, 2.0, 2.0))
    lam_s = ctl.gyration_eigenvalues(tm_s["rest"], np.zeros(tm_s["rest"].shape[0], np.int32), 1, (10.0,) * 3,
                                     (0, 0, 0))[0]
    assert np.allclose(lam_s, 4.0 / 3.0, rtol=2e-2)
