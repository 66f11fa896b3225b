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
