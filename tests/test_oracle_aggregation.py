"""Pins of the oracle's inter-platelet aggregation term (Sec. 3.2, Eq. 4): a non-bonded
Morse potential plus the receptor term f^A (1 - r/r0), acting between beads of
different platelets closer than the aggregation cutoff.

Each pin checks the oracle against something other than its own formula: special
values of the receptor term that Eq. 4 fixes, the depth and the minimum of the Morse
well written in the paper's own parameterisation (Eq. 2, epsilon and alpha), the force
as minus the gradient of the separately coded energy, Newton's third law, the
exclusion of pairs within one platelet and beyond the cutoff, and the small-oscillation
frequency of a bound dimer, whose curvature 2 a^2 D + f^A / r0 involves both terms.
"""
import numpy as np
import pytest

from test_oracle_forces import _fd_grad, _tiny

AGG = dict(agg_D=5.0, agg_a=2.0, agg_r0=1.0, agg_fA=10.0, agg_rc=1.8)


def _beads(x, body, **par):
    """Beads only (no fluid), one bead per row, platelet ids `body`, WCA off unless given."""
    x = np.asarray(x, float)
    nb = x.shape[0]
    P = int(np.max(body)) + 1
    par = dict(dict(lj_eps=0.0, kb=0.0, ka=0.0), **par)
    d = _tiny(x, 0, L=(12.0, 12.0, 12.0), beads=dict(body=np.asarray(body, np.int32), rest=np.zeros((nb, 3)),
                                                    platelet_area=np.ones(P)), **par)
    d["n_platelet"] = P
    return d


def _dimer_force(oracle_lib, r, **par):
    e = np.array([0.36, 0.48, 0.8])  # unit vector (3-4-5 scaled)
    x = np.array([[6.0, 6.0, 6.0], 6.0 + r * e])
    d = _beads(x, [0, 1], **par)
    S = oracle_lib.System(d)
    f = S.inner_forces(d["x"], d["v"], 0, 0.001, brute=True)
    # force on bead 0 along e_01 = (x0 - x1) / r = -e
    return float(np.dot(f[0], -e)), f, S, d


@pytest.mark.parametrize("r,expect", [(0.25, 0.75), (0.5, 0.5), (0.8, 0.2), (1.0, 0.0), (1.2, -0.2), (1.5, -0.5)])
def test_receptor_term_special_values(oracle_lib, r, expect):
    """Eq. 4's receptor term alone (D = 0): the force along e_ij is f^A (1 - r/r0)."""
    par = dict(AGG, agg_D=0.0)
    fr, f, *_ = _dimer_force(oracle_lib, r, **par)
    assert fr == pytest.approx(expect * par["agg_fA"], rel=1e-13, abs=1e-13)
    assert np.max(np.abs(f[0] + f[1])) < 1e-13  # Newton's third law


def test_morse_well_in_the_papers_parameterisation(oracle_lib):
    """Eq. 2 writes U_M = eps [e^{alpha (1 - r/r0)} - 2 e^{alpha (1 - r/r0)/2}]; with
    eps = D and alpha = 2 a r0 it is the oracle's well.  Depth: U(r0) - U(r) for a few r
    against that form; minimum: zero force at r0 and restoring forces on both sides."""
    par = dict(AGG, agg_fA=0.0)
    eps, alpha, r0 = par["agg_D"], 2.0 * par["agg_a"] * par["agg_r0"], par["agg_r0"]

    def paper(r):
        q = alpha * (1.0 - r / r0)
        return eps * (np.exp(q) - 2.0 * np.exp(q / 2.0))

    def oracle_U(r):
        _, _, S, d = _dimer_force(oracle_lib, r, **par)
        return S.energy(d["x"])[4]

    for r in (0.7, 0.9, 1.3, 1.7):
        assert oracle_U(r0) - oracle_U(r) == pytest.approx(paper(r0) - paper(r), rel=1e-12)
    assert paper(r0) == pytest.approx(-eps)
    assert abs(_dimer_force(oracle_lib, r0, **par)[0]) < 1e-12
    assert _dimer_force(oracle_lib, 0.9, **par)[0] > 0.0  # pushed apart inside r0
    assert _dimer_force(oracle_lib, 1.1, **par)[0] < 0.0  # pulled together beyond


def test_cutoff_and_same_platelet_exclusion(oracle_lib):
    """No aggregation force beyond agg_rc, none within one platelet, and the term is off
    at agg_rc = 0."""
    assert _dimer_force(oracle_lib, 1.81, **AGG)[0] == 0.0
    assert _dimer_force(oracle_lib, 1.2, **dict(AGG, agg_rc=0.0))[0] == 0.0
    e = np.array([0.36, 0.48, 0.8])
    x = np.array([[6.0, 6.0, 6.0], 6.0 + 1.2 * e])
    d = _beads(x, [0, 0], **AGG)
    d["n_platelet"] = 1
    d["platelet_area"] = np.ones(1)
    S = oracle_lib.System(d)
    assert np.all(S.inner_forces(d["x"], d["v"], 0, 0.001, brute=True) == 0.0)


def test_force_is_minus_gradient_of_energy(oracle_lib):
    """Six beads of three platelets with every separation inside the cutoff and away
    from it: the inner force equals -grad of the aggregation energy (WCA on too, so the
    two terms add), by central differences; the forces sum to zero."""
    rng = np.random.default_rng(11)
    while True:
        x = 6.0 + rng.uniform(-0.7, 0.7, (6, 3))
        r = np.linalg.norm(x[:, None] - x[None], axis=2)[np.triu_indices(6, 1)]
        if r.min() > 0.5 and np.all(np.abs(r - AGG["agg_rc"]) > 0.05) and np.all(np.abs(r - 0.8 * 2 ** (1 / 6)) > 0.05):
            break
    d = _beads(x, [0, 0, 1, 1, 2, 2], lj_eps=1.0, r_excl=0.0, **AGG)
    S = oracle_lib.System(d)
    f = S.inner_forces(d["x"], d["v"], 0, 0.001, brute=True)
    g = _fd_grad(lambda y: float(np.sum(S.energy(y)[[1, 4]])), d["x"])
    assert np.allclose(f, -g, rtol=1e-7, atol=1e-6)
    assert np.max(np.abs(f.sum(axis=0))) < 1e-11
    # the cell list gives the brute-force result
    fc = S.inner_forces(d["x"], d["v"], 0, 0.001, brute=False)
    assert np.allclose(fc, f, rtol=1e-12, atol=1e-12)


def test_bound_dimer_small_oscillation_frequency(oracle_lib):
    """Two one-bead platelets released from rest at r0 + q0 (q0 small) oscillate with
    the curvature of the summed well at r0: k = 2 a^2 D (Morse) + f^A / r0 (receptor
    spring), reduced mass m/2.  Velocity Verlet advances the phase by theta per step
    with cos(theta) = 1 - (w dt)^2 / 2; the trajectory's phase over ~4 periods must
    match to 1e-4 (anharmonic corrections are O((a q0)^2))."""
    p = AGG
    r0, q0, dt = p["agg_r0"], 1e-3, 0.002
    e = np.array([1.0, 0.0, 0.0])
    x = np.array([[5.0, 6.0, 6.0], [5.0 + r0 + q0, 6.0, 6.0]])
    d = _beads(x, [0, 1], **p)
    S = oracle_lib.System(d)
    kk = 2.0 * p["agg_a"] ** 2 * p["agg_D"] + p["agg_fA"] / r0
    w = np.sqrt(kk / 0.5)
    theta = np.arccos(1.0 - (w * dt) ** 2 / 2.0)
    xx, vv = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(xx, vv, 0, dt, brute=True)
    fi = S.inner_forces(xx, vv, 0, dt, brute=True)
    n_per = int(round(2 * np.pi / theta))
    rs = []
    cnt = [1, 1]
    for _ in range(4 * n_per):
        cnt = S.respa(xx, vv, fo, fi, cnt, 1, dt, 1, brute=True)
        rs.append(np.dot(xx[1] - xx[0], e) - r0)
    n = np.arange(1, len(rs) + 1)
    # least-squares phase of q0 cos(n phi): scan phi near theta
    phis = theta * (1.0 + np.linspace(-2e-3, 2e-3, 4001))
    err = [np.sum((np.asarray(rs) - q0 * np.cos(n * ph)) ** 2) for ph in phis]
    phi = phis[int(np.argmin(err))]
    assert phi == pytest.approx(theta, rel=1e-4)
    # a well with either term missing or doubled is far off
    for bad in (2.0 * p["agg_a"] ** 2 * p["agg_D"], p["agg_fA"] / r0, kk + p["agg_fA"] / r0):
        tb = np.arccos(1.0 - (np.sqrt(bad / 0.5) * dt) ** 2 / 2.0)
        assert abs(tb / theta - 1.0) > 1e-2


def test_three_level_groups_place_aggregation_at_the_finest_sublevel(oracle_lib):
    """Eq. 4 joins platelets, so the three-level scheme evaluates it with the other
    inter-platelet terms in the aggregating group P2 whatever the platelets' sublevels;
    the three groups add up to the two-group inner force."""
    rng = np.random.default_rng(4)
    x = 6.0 + rng.uniform(-0.6, 0.6, (6, 3))
    d = _beads(x, [0, 0, 1, 1, 2, 2], lj_eps=1.0, r_excl=0.0, **AGG)
    S = oracle_lib.System(d)
    f2 = S.inner_forces(d["x"], d["v"], 0, 0.001, brute=True)
    for lev in ([1, 1, 1], [2, 2, 2], [1, 2, 1]):
        fm, fp1, fp2 = S.inner_forces3(d["x"], d["v"], 0, 0.001, np.array(lev, np.int32), brute=True)
        assert np.allclose(fm + fp1 + fp2, f2, rtol=1e-12, atol=1e-12)
        # with the WCA cut at ~0.9, the aggregation force between platelets sits in P2
        dd = _beads(x, [0, 0, 1, 1, 2, 2], lj_eps=0.0, r_excl=0.0, **AGG)
        Sa = oracle_lib.System(dd)
        fm_a, fp1_a, fp2_a = Sa.inner_forces3(dd["x"], dd["v"], 0, 0.001, np.array(lev, np.int32), brute=True)
        assert np.all(fp1_a == 0.0) and np.all(fm_a == 0.0) and np.any(fp2_a != 0.0)
