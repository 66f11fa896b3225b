"""Pins of the oracle's RESPA integrator (Table 1), diagnostics and platelet features:
closed-form discrete trajectories, energy conservation order, time reversibility,
the DPD fluctuation-dissipation temperature and exact invariances."""
import numpy as np
import pytest

import synth
from test_oracle_forces import _tiny


def _run(S, d, n_outer, dt_outer, k, brute=True):
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, 0, dt_outer, brute=brute)
    fi = S.inner_forces(x, v, 0, dt_outer / k, brute=brute)
    cnt = S.respa(x, v, fo, fi, [1, 1], n_outer, dt_outer, k, brute=brute)
    return x, v, fo, fi, cnt


@pytest.mark.parametrize("k", [1, 3])
def test_harmonic_dimer_closed_form(oracle_lib, k):
    """Velocity Verlet on U = kb (r - r0)^2 from rest: r_n = r0 + q0 cos(n theta),
    cos(theta) = 1 - (w dt)^2 / 2 with w^2 = 2 * 2 kb / m (reduced mass m/2)."""
    kb, r0, q0, dt = 100.0, 1.0, 0.05, 0.01
    x = np.array([[3.0, 3.0, 3.0], [3.0 + r0 + q0, 3.0, 3.0]])
    d = _tiny(x, 0, beads=dict(body=np.array([0, 0]), bonds=np.array([[0, 1]]), bond_r0=np.array([r0])),
              lj_eps=0.0, kb=kb)
    S = oracle_lib.System(d)
    dti = dt / k
    n = 37
    xx, vv, *_ = _run(S, d, n, dt, k)
    theta = np.arccos(1.0 - (4.0 * kb * dti * dti) / 2.0)
    r = xx[1, 0] - xx[0, 0]
    assert r == pytest.approx(r0 + q0 * np.cos(n * k * theta), abs=1e-12)
    assert abs(xx[0, 0] + xx[1, 0] - (6.0 + r0 + q0)) < 1e-12  # centre of mass at rest


def _total_energy(S, x, v):
    m = 1.0
    return 0.5 * m * np.sum(v * v) + np.sum(S.energy(x)[:5])


def test_conservative_dpd_energy_order_and_reversibility(oracle_lib):
    d = synth.dpd_box(n=648, L=(6.0, 6.0, 6.0), seed=21, gamma=0.0, sigma=0.0)
    S = oracle_lib.System(d)
    flucts = []
    for dt in (0.004, 0.002):
        x, v = d["x"].copy(), d["v"].copy()
        fo = S.outer_forces(x, v, 0, dt)
        fi = S.inner_forces(x, v, 0, dt)
        E = []
        for _ in range(40):
            S.respa(x, v, fo, fi, [1, 1], int(round(0.02 / dt)), dt, 1)
            E.append(_total_energy(S, x, v))
        flucts.append(np.std(E))
    ratio = flucts[0] / flucts[1]
    assert 4.0 * 0.8 < ratio < 4.0 * 1.2  # second-order integrator
    # time reversibility: n steps, reverse velocities, n steps
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, 0, 0.01)
    fi = S.inner_forces(x, v, 0, 0.01)
    S.respa(x, v, fo, fi, [1, 1], 100, 0.01, 1)
    v *= -1.0
    S.respa(x, v, fo, fi, [1, 1], 100, 0.01, 1)
    dx = x - d["x"]
    dx -= 6.0 * np.round(dx / 6.0)
    assert np.max(np.abs(dx)) < 1e-9
    assert np.max(np.abs(v + d["v"])) < 1e-9


def test_two_group_respa_energy_order_and_reversibility(oracle_lib):
    d = synth.platelet_box(n_fluid=1300, L=(8.0, 8.0, 8.0), level=2, semi_axes=(2.0, 0.8, 2.0), seed=22,
                           gamma=0.0, sigma=0.0, gamma_pf=0.0, sigma_pf=0.0)
    S = oracle_lib.System(d)
    d["v"] *= 0.3
    flucts = []
    for dti in (0.002, 0.001):
        x, v = d["x"].copy(), d["v"].copy()
        dto = 4 * dti
        fo = S.outer_forces(x, v, 0, dto, brute=False)
        fi = S.inner_forces(x, v, 0, dti, brute=False)
        E = []
        for _ in range(30):
            S.respa(x, v, fo, fi, [1, 1], int(round(0.016 / dto)), dto, 4)
            E.append(_total_energy(S, x, v))
        flucts.append(np.std(E))
    assert 4.0 * 0.75 < flucts[0] / flucts[1] < 4.0 * 1.25
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, 0, 0.008)
    fi = S.inner_forces(x, v, 0, 0.002)
    S.respa(x, v, fo, fi, [1, 1], 50, 0.008, 4)
    v *= -1.0
    S.respa(x, v, fo, fi, [1, 1], 50, 0.008, 4)
    dx = x - d["x"]
    dx -= 8.0 * np.round(dx / 8.0)
    assert np.max(np.abs(dx)) < 1e-9


def test_dpd_thermostat_reaches_kT_and_conserves_momentum(oracle_lib):
    """Fluctuation-dissipation (sigma^2 = 2 gamma kT): the DPD fluid equilibrates at kT = 1."""
    d = synth.dpd_box(n=375, L=(5.0, 5.0, 5.0), seed=23)
    p = d["params"]
    assert p["sigma"] ** 2 == pytest.approx(2.0 * p["gamma"] * p["kT"])
    S = oracle_lib.System(d)
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, 0, 0.01)
    fi = S.inner_forces(x, v, 0, 0.01)
    cnt = S.respa(x, v, fo, fi, [1, 1], 300, 0.01, 1)
    T = []
    for _ in range(400):
        cnt = S.respa(x, v, fo, fi, cnt, 20, 0.01, 1)
        T.append(S.thermo(x, v)[1])
        assert np.all(np.abs(v.sum(axis=0)) < 1e-9)
    assert abs(np.mean(T) - 1.0) < 0.015


def test_walls_bounce_back_and_stay_frozen(oracle_lib):
    x = np.array([[2.0, 1.02, 2.0], [2.0, 0.5, 2.0], [2.0, 5.0, 2.0]])
    v = np.array([[1.0, -3.0, 0.5], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    d = _tiny(x, 1, n_wall=2, L=(4.0, 6.0, 4.0), periodic=(1, 0, 1), a=0.0, gamma=0.0, sigma=0.0,
              wall_axis=1, wall_lo=1.0, wall_hi=5.0)
    d["v"] = v
    S = oracle_lib.System(d)
    xx, vv, *_ = _run(S, d, 1, 0.01, 1)
    # y: 1.02 - 0.03 = 0.99 -> reflected to 1.01, velocity reversed entirely
    assert xx[0, 1] == pytest.approx(1.01, abs=1e-14)
    assert np.allclose(vv[0], [-1.0, 3.0, -0.5], atol=1e-14)
    assert np.array_equal(xx[1:], x[1:]) and np.all(vv[1:] == 0.0)


def test_thermo_closed_forms(oracle_lib):
    rng = np.random.default_rng(31)
    n = 500
    x = rng.random((n, 3)) * np.array([4.0, 10.0, 4.0])
    v = rng.standard_normal((n, 3))
    d = _tiny(x, n, L=(4.0, 10.0, 4.0), periodic=(1, 0, 1))
    S = oracle_lib.System(d)
    ke, T, Tp, *p = S.thermo(x, v, n_bins=10)
    assert ke == pytest.approx(0.5 * np.sum(v * v), rel=1e-14)
    assert T == pytest.approx(np.sum(v * v) / (3 * n - 3), rel=1e-14)
    assert np.allclose(p, v.sum(axis=0), rtol=0, atol=1e-12)
    # peculiar temperature ignores any flow that is constant within each y bin
    flow = np.zeros_like(v)
    b = np.floor(x[:, 1]).astype(int)
    flow[:, 0] = 0.3 * b ** 2
    flow[:, 2] = -0.1 * b
    Tp2 = S.thermo(x, v + flow, n_bins=10)[2]
    assert Tp2 == pytest.approx(Tp, rel=1e-12)
    assert S.thermo(x, v + flow, n_bins=10)[1] > T


def test_features_rigid_motion(oracle_lib):
    tm = synth.platelet_template(level=2, semi_axes=(2.0, 0.8, 2.0))
    nb = tm["rest"].shape[0]
    R = synth.random_rotation(np.random.default_rng(5))
    xb = tm["rest"] @ R.T + np.array([9.8, 5.0, 5.0])  # straddles the periodic x boundary
    xb[:, 0] = np.mod(xb[:, 0], 10.0)
    omega = np.array([0.3, -1.2, 0.5])
    V = np.array([0.2, 0.1, -0.4])
    rel = tm["rest"] @ R.T
    vb = V[None, :] + np.cross(omega[None, :], rel - rel.mean(axis=0))
    d = _tiny(xb, 0, L=(10.0, 10.0, 10.0), beads=dict(
        body=np.zeros(nb, np.int32), rest=tm["rest"], bonds=tm["bonds"], bond_r0=tm["bond_r0"],
        angles=tm["angles"], angle_th0=tm["angle_th0"], platelet_area=np.array([tm["area"]])))
    d["n_platelet"] = 1
    S = oracle_lib.System(d)
    f = S.features(xb, vb)[0]
    assert np.allclose(f[:3], V, atol=1e-12)
    assert f[3] == pytest.approx(np.linalg.norm(omega), rel=1e-10)
    assert f[4] == pytest.approx(0.5 * np.sum((vb - V) ** 2), rel=1e-12)
    assert f[5] < 1e-12 and f[6] == 0.0 and f[7] == 0.0
    # inflate the platelet by 10% about its centre: every bond strains by exactly 0.1
    xs = rel.mean(axis=0) + 1.1 * (rel - rel.mean(axis=0)) + np.array([9.8, 5.0, 5.0])
    xs[:, 0] = np.mod(xs[:, 0], 10.0)
    assert S.features(xs, vb)[0][5] == pytest.approx(0.1, rel=1e-9)


def _feature_layout():
    """Two platelets near a wall and two fluid particles, placed so that every term of
    the interfacial traction and every contact is known by hand.

    Platelet 0: bead A = (5, 1.5, 5) and bead D = (5, 1.5, 3); platelet 1: beads
    B = (5, 1.5, 5.95) and C = (5, 1.5, 6.05).  Wall particles w1 = (5, 0.9, 5) and
    w2 = (5.9, 0.7, 5).  Fluid f1 = A - (0.64, -0.48, 0) (distance 0.8 = sigma_LJ) with
    velocity -e1, e1 = (0.8, -0.6, 0), and f2 = A - (0.54, 0, 0.72) (distance 0.9, just
    beyond the WCA cutoff 2^(1/6) 0.8 = 0.898 and inside rc_pf = 1) with velocity -e2,
    e2 = (0.6, 0, 0.8).  A is at rest.
    """
    A, D, B, C = (5, 1.5, 5), (5, 1.5, 3), (5, 1.5, 5.95), (5, 1.5, 6.05)
    w1, w2 = (5, 0.9, 5), (5.9, 0.7, 5)
    f1 = (5 - 0.64, 1.5 + 0.48, 5)
    f2 = (5 - 0.54, 1.5, 5 - 0.72)
    x = np.array([f1, f2, w1, w2, A, D, B, C], dtype=np.float64)
    d = _tiny(x, 2, n_wall=2, L=(10.0, 10.0, 10.0), periodic=(1, 0, 1), wall_axis=1, wall_lo=1.0, wall_hi=9.0,
              beads=dict(body=np.array([0, 0, 1, 1], np.int32), rest=np.zeros((4, 3)),
                         platelet_area=np.array([2.0, 3.0])))
    d["n_platelet"] = 2
    d["v"][0] = [-0.8, 0.6, 0.0]
    d["v"][1] = [-0.6, 0.0, -0.8]
    return d


def test_features_traction_and_contacts_by_hand(oracle_lib):
    """Features 6 and 7 on a layout counted by hand (sigma_pf = 3: the random term must
    stay out of the traction).

    Traction of platelet 0, sum over its beads' fluid and wall partners of
    (y_bead - y_partner) F_x / area:
      f1 at r = sigma_LJ: the WCA force there is 24 eps / sigma = 30 along e1, i.e.
         (24, -18, 0), times d_y = -0.48 gives -11.52; the dissipative force,
         -gamma_pf w^2 (e1 . v_rel) e1 with w = 1 - 0.8 = 0.2 and e1 . v_rel = 1, is
         -0.18 e1, F_x = -0.144, times -0.48 gives +0.06912;
      f2 at r = 0.9: dissipative only, but d_y = 0 (a traction on the wrong axis, z,
         would give 0.72 * (-0.045 * 0.6) = -0.01944);
      w1 lies straight below A (d_x = 0, so F_x = 0); w2 is beyond every cutoff;
    so feature 6 = (-11.52 + 0.06912) / 2.0.  Platelet 1 has no fluid or wall partner.
    Contacts (walls and beads of other platelets within 1.0): A-w1 (0.6) and A-B (0.95)
    for platelet 0; B-A for platelet 1; A-C (1.05), A-w2 (1.20), D-w1 (2.09) and the
    same-platelet pairs do not count.
    """
    d = _feature_layout()
    S = oracle_lib.System(d)
    f = S.features(d["x"], d["v"])
    assert f[0, 6] == pytest.approx((-11.52 + 0.06912) / 2.0, rel=1e-12)
    assert f[1, 6] == 0.0
    assert f[0, 7] == 2.0 and f[1, 7] == 1.0


def test_interface_dissipative_random_pair_thermostats_beads_at_kT(oracle_lib):
    """Eq. 3's dissipative + random bead-fluid terms alone (WCA off) hold free beads at
    kT: the random term is scaled by 1/sqrt(dt_inner) of the inner group it belongs to
    (sigma_pf^2 = 2 gamma_pf kT).  Sixty single-bead platelets start at rest in a DPD
    fluid at kT = 1 and run 1,200 RESPA outer steps at k = 4.  A random term scaled
    with the outer step (4 dt_inner) has a quarter of the variance, which is what
    sigma_pf / 2 gives here: that control must leave the beads far colder."""
    def bead_T(sigma_pf):
        rng = np.random.default_rng(3)
        L, nb = 7.0, 60
        nf = int(3 * L ** 3)
        x = np.concatenate([rng.random((nf, 3)) * L, rng.random((nb, 3)) * L])
        d = _tiny(x, nf, L=(L, L, L), beads=dict(body=np.arange(nb, dtype=np.int32), rest=np.zeros((nb, 3)),
                                                 platelet_area=np.ones(nb)), lj_eps=0.0, sigma_pf=sigma_pf)
        d["n_platelet"] = nb
        vf = synth.maxwell(rng, nf)
        d["v"][:nf] = vf - vf.mean(axis=0)
        S = oracle_lib.System(d)
        x, v = d["x"].copy(), d["v"].copy()
        k, dto = 4, 0.01
        fo = S.outer_forces(x, v, 0, dto)
        fi = S.inner_forces(x, v, 0, dto / k)
        cnt = S.respa(x, v, fo, fi, [1, 1], 200, dto, k)
        T = []
        for _ in range(200):
            cnt = S.respa(x, v, fo, fi, cnt, 5, dto, k)
            T.append(np.mean(v[nf:] ** 2))
        return float(np.mean(T))

    p = synth.dpd_params()
    assert p["sigma_pf"] ** 2 == pytest.approx(2.0 * p["gamma_pf"] * p["kT"])
    assert abs(bead_T(3.0) - 1.0) < 0.06
    assert bead_T(1.5) < 0.6
