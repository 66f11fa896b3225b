"""Checks of the seeded input generators: mesh invariants, counts, placement rules."""
import numpy as np

import synth


def test_icosphere_invariants():
    for n in (0, 1, 2, 3, 4):
        t = synth.platelet_template(level=n)
        V, E, F = t["rest"].shape[0], t["bonds"].shape[0], t["faces"].shape[0]
        assert (V, E, F) == (10 * 4 ** n + 2, 30 * 4 ** n, 20 * 4 ** n)
        assert V - E + F == 2
        assert t["angles"].shape[0] == 3 * F
        # every edge lies in exactly two faces (closed surface)
        cnt = {}
        for a, b, c in t["faces"]:
            for p, q in ((a, b), (b, c), (c, a)):
                key = (min(p, q), max(p, q))
                cnt[key] = cnt.get(key, 0) + 1
        assert set(cnt.values()) == {2} and len(cnt) == E
        # the three corner angles of each face sum to pi
        if n == 2:
            th = {}
            for (e1, vtx, e2), a in zip(t["angles"], t["angle_th0"]):
                th[(vtx, min(e1, e2), max(e1, e2))] = a
            for a, b, c in t["faces"]:
                s = th[(a, min(b, c), max(b, c))] + th[(b, min(a, c), max(a, c))] + th[(c, min(a, b), max(a, b))]
                assert abs(s - np.pi) < 1e-12


def test_level4_platelet_sizes():
    t = synth.platelet_template(level=4, semi_axes=(3.0, 1.0, 3.0))
    assert t["rest"].shape[0] == 2562 and t["bonds"].shape[0] == 7680 and t["angles"].shape[0] == 15360
    assert 0.15 < t["bond_r0"].mean() < 0.22
    assert np.allclose(t["rest"].max(axis=0), [3.0, 1.0, 3.0], atol=1e-12)


def test_workloads_are_seeded_and_respect_placement():
    a = synth.platelet_box(n_fluid=4000, L=(12.0, 12.0, 12.0), level=2, semi_axes=(2.0, 0.8, 2.0), seed=3)
    b = synth.platelet_box(n_fluid=4000, L=(12.0, 12.0, 12.0), level=2, semi_axes=(2.0, 0.8, 2.0), seed=3)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["v"], b["v"])
    xf, xb = a["x"][:a["n_fluid"]], a["x"][a["n_fluid"]:]
    d = np.linalg.norm(xf[:, None, :] - xb[None, :, :], axis=2)
    assert d.min() >= a["params"]["lj_sig"]
    assert np.allclose(a["v"].mean(axis=0), 0.0, atol=1e-12)
    c = synth.channel(n_total=60000, L=(40.0, 20.0, 25.0), n_platelet=2, level=2, semi_axes=(2.0, 0.8, 2.0), seed=5)
    nf, nw = c["n_fluid"], c["n_wall"]
    assert nf + nw == 60000
    yw = c["x"][nf:nf + nw, 1]
    assert np.all((yw < 1.0) | (yw > 19.0))
    yf = c["x"][:nf, 1]
    assert yf.min() >= 1.0 and yf.max() <= 19.0
    assert np.all(c["v"][nf:nf + nw] == 0.0)
