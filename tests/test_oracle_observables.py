"""Pins of the oracle's platelet measurements for the paper's own inference pipeline
(Sec. 3.3: angular velocity components, kinetic energies, flow speed at the centre of
mass) and of the per-bead membrane stress (Sec. 4.2, Fig. 5).

The measurements are checked on rigid motions, where the angular velocity is known
exactly and the kinetic energies follow from the bead velocities directly, and on a
uniform fluid flow.  The stress is checked against a stretched bond and a free bead
in closed form, against the total pair virial that the energy routine computes along
a separate code path, and against the scale invariance of the angle term (its virial
vanishes)."""
import numpy as np
import pytest

import synth
from test_oracle_forces import _tiny


def _platelet(level=2, semi=(2.0, 0.8, 2.0), centre=(5.0, 5.0, 5.0)):
    tm = synth.platelet_template(level=level, semi_axes=semi)
    return tm["rest"] - tm["rest"].mean(axis=0) + np.asarray(centre)


def test_paper_features_of_a_rigid_motion(oracle_lib):
    xb = _platelet()
    nb = xb.shape[0]
    rng = np.random.default_rng(3)
    nf = 400
    xf = rng.uniform(0.0, 10.0, (nf, 3))
    x = np.concatenate([xf, xb])
    d = _tiny(x, nf, L=(10.0, 10.0, 10.0), beads=dict(body=np.zeros(nb, np.int32), rest=xb.copy(),
                                                     platelet_area=np.ones(1)))
    d["n_platelet"] = 1
    w0, V0 = np.array([0.3, -1.1, 0.7]), np.array([0.5, 0.2, -0.4])
    com = xb.mean(axis=0)
    u0 = np.array([0.8, -0.3, 0.25])
    v = np.zeros_like(x)
    v[nf:] = V0 + np.cross(w0, xb - com)
    near = np.linalg.norm(xf - com, axis=1) < 4.0
    v[:nf][near] = u0
    v[:nf][~near] = rng.normal(0.0, 3.0, (int((~near).sum()), 3))  # outside the flow radius: ignored
    S = oracle_lib.System(d)
    f = S.paper_features(x, v, flow_r=4.0)[0]
    assert np.allclose(f[:3], w0, rtol=1e-12, atol=1e-12)
    M = float(nb)
    assert f[3] == pytest.approx(0.5 * M * V0 @ V0, rel=1e-12)
    # rotational energy: the beads' kinetic energy relative to the centre of mass
    rel = v[nf:] - V0
    assert f[4] == pytest.approx(0.5 * np.sum(rel * rel), rel=1e-12)
    assert f[5] == pytest.approx(np.linalg.norm(u0), rel=1e-12)
    assert near.sum() > 50


def test_bead_stress_closed_forms(oracle_lib):
    # a stretched bond at rest: each bead carries half of r.F = -2 kb (r - r0) r, over 3
    kb, r0, r = 100.0, 1.0, 1.07
    x = np.array([[3.0, 3.0, 3.0], [3.0 + r, 3.0, 3.0], [1.0, 1.0, 1.0]])
    d = _tiny(x, 0, beads=dict(body=np.array([0, 0, 1], np.int32), bonds=np.array([[0, 1]]), bond_r0=np.array([r0]),
                              rest=np.zeros((3, 3)), platelet_area=np.ones(2)), lj_eps=0.0, kb=kb)
    d["n_platelet"] = 2
    v = np.zeros_like(x)
    v[2] = [0.3, -0.4, 1.2]  # a free bead: kinetic part only
    s = oracle_lib.System(d).bead_stress(x, v)
    assert s[0] == pytest.approx(-kb * (r - r0) * r / 3.0, rel=1e-13)
    assert s[1] == pytest.approx(s[0], rel=1e-13)
    assert s[2] == pytest.approx(v[2] @ v[2] / 3.0, rel=1e-13)


def test_bead_stress_sums_to_the_pair_virial(oracle_lib):
    """Beads of two jittered platelets with bonds, WCA, a few Morse bonds and the Eq. 4
    aggregation term (angle term off, see below): the per-bead shares add up to the
    total virial of the energy routine."""
    xa = _platelet(centre=(5.0, 4.0, 5.0))
    xb = _platelet(centre=(5.0, 6.1, 5.0))
    x = np.concatenate([xa, xb]) + np.random.default_rng(2).normal(0.0, 0.01, (2 * xa.shape[0], 3))
    nb = x.shape[0]
    tm = synth.platelet_template(level=2, semi_axes=(2.0, 0.8, 2.0))
    n1 = xa.shape[0]
    bonds = np.concatenate([tm["bonds"], tm["bonds"] + n1])
    morse = np.array([[0, n1], [5, n1 + 7]])
    d = _tiny(x, 0, L=(12.0, 12.0, 12.0), beads=dict(
        body=np.repeat([0, 1], n1).astype(np.int32), rest=np.concatenate([xa, xb]), bonds=bonds,
        bond_r0=np.concatenate([tm["bond_r0"], tm["bond_r0"]]), morse=morse, platelet_area=np.ones(2)),
        ka=0.0, agg_rc=1.5)
    d["n_platelet"] = 2
    v = np.random.default_rng(4).normal(0.0, 1.0, x.shape)
    S = oracle_lib.System(d)
    s = S.bead_stress(x, v)
    virial = S.energy(x)[5]
    assert np.sum(3.0 * s - np.sum(v * v, axis=1)) == pytest.approx(virial, rel=1e-10)
    assert S.energy(x)[4] != 0.0  # Morse and aggregation terms present


def test_angle_term_carries_no_virial(oracle_lib):
    """U = ka (theta - theta0)^2 does not change under a uniform dilation, so the
    virial of every angle, and each bead's share of it, vanishes."""
    x = _platelet() + np.random.default_rng(6).normal(0.0, 0.03, (_platelet().shape[0], 3))
    tm = synth.platelet_template(level=2, semi_axes=(2.0, 0.8, 2.0))
    nb = x.shape[0]
    d = _tiny(x, 0, L=(10.0, 10.0, 10.0), beads=dict(body=np.zeros(nb, np.int32), rest=x.copy(), angles=tm["angles"],
                                                     angle_th0=tm["angle_th0"], platelet_area=np.ones(1)),
              lj_eps=0.0, kb=0.0)
    d["n_platelet"] = 1
    s = oracle_lib.System(d).bead_stress(x, np.zeros_like(x))
    assert np.max(np.abs(s)) < 1e-10
