"""Pins of the oracle's three-level MTS with per-platelet sublevels (Sec. 3.3, Table 1):
the group split adds up to the two-group inner force, the scheme reduces to two-group
RESPA when the levels coincide, a harmonic dimer follows the closed-form Verlet
trajectory of its own sublevel's step, inter-platelet terms stay at the finest step,
the interface's dissipative + random terms hold beads at kT with the random term scaled
by the interface step, and the conservative scheme is second order and reversible."""
import numpy as np
import pytest

import synth
from test_oracle_forces import _tiny


def _small_platelet(**over):
    return synth.platelet_box(n_fluid=1300, L=(8.0, 8.0, 8.0), level=2, semi_axes=(2.0, 0.8, 2.0), seed=22, **over)


def _run3(S, d, n_outer, dt, k, k_if, k_sub, level, counters=(1, 1)):
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, counters[0], k * dt)
    fm, f1, f2 = S.inner_forces3(x, v, counters[1], k_if * dt, level)
    cnt = S.respa3(x, v, fo, fm, f1, f2, [counters[0] + 1, counters[1] + 1], n_outer, dt, k, k_if, k_sub, level)
    return x, v, cnt


def test_groups_add_up_to_the_two_group_inner_force(oracle_lib):
    d = synth.aggregate_box(n_fluid=3000, L=(12.0, 12.0, 12.0), level=2)
    S = oracle_lib.System(d)
    P = int(d["n_platelet"])
    assert P == 2 and d["morse"].shape[0] > 0
    ref = S.inner_forces(d["x"], d["v"], 5, 0.0025)
    for level in ([1, 1], [1, 2], [2, 1], [2, 2]):
        fm, f1, f2 = S.inner_forces3(d["x"], d["v"], 5, 0.0025, level)
        tot = fm + f1 + f2
        assert np.max(np.abs(tot - ref)) <= 1e-12 * np.max(np.abs(ref))
        # P1 holds exactly the terms of the sublevel-1 platelets' own beads
        b0 = int(d["n_fluid"] + d["n_wall"])
        for q in range(2):
            rows = f1[b0:][d["body"] == q]
            assert np.any(rows != 0.0) if level[q] == 1 else np.all(rows == 0.0)
        assert np.all(f1[:b0] == 0.0) and np.all(f2[:b0] == 0.0)
    # with bonds, angles and WCA off, what is left of the platelet groups is the Morse
    # bonds: in P2 even when both platelets are at sublevel 1
    S0 = oracle_lib.System(d, params=dict(kb=0.0, ka=0.0, lj_eps=0.0))
    fm, f1, f2 = S0.inner_forces3(d["x"], d["v"], 5, 0.0025, [1, 1])
    assert np.all(f1 == 0.0) and np.count_nonzero(np.any(f2 != 0.0, axis=1)) == 2 * d["morse"].shape[0]
    # the interface group alone is the bead-fluid force: beads' partners only
    fm, f1, f2 = S.inner_forces3(d["x"], d["v"], 5, 0.0025, [1, 1], due=S.G_M)
    assert np.all(f1 == 0.0) and np.all(f2 == 0.0) and np.any(fm != 0.0)


def test_reduces_to_two_group_respa_when_levels_coincide(oracle_lib):
    d = _small_platelet()
    S = oracle_lib.System(d)
    k, dt = 4, 0.0025
    x3, v3, c3 = _run3(S, d, 6, dt, k, 1, 1, [1])
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, 1, k * dt)
    fi = S.inner_forces(x, v, 1, dt)
    c2 = S.respa(x, v, fo, fi, [2, 2], 6, k * dt, k)
    assert list(c3) == list(c2)
    assert np.max(np.abs(x3 - x)) < 1e-12 and np.max(np.abs(v3 - v)) < 1e-10


@pytest.mark.parametrize("level,k_sub", [(1, 2), (2, 2), (1, 1)])
def test_harmonic_dimer_follows_its_sublevel_step(oracle_lib, level, k_sub):
    """U = kb (r - r0)^2 from rest: velocity Verlet at step h gives r_n = r0 + q0 cos(n theta),
    cos theta = 1 - (w h)^2 / 2, w^2 = 4 kb / m.  h = k_sub dt at sublevel 1, dt at sublevel 2."""
    kb, r0, q0, dt, k, k_if = 100.0, 1.0, 0.05, 0.0025, 8, 4
    x = np.array([[3.0, 3.0, 3.0], [3.0 + r0 + q0, 3.0, 3.0]])
    d = _tiny(x, 0, beads=dict(body=np.array([0, 0]), bonds=np.array([[0, 1]]), bond_r0=np.array([r0]),
                               rest=np.array([[0.0, 0.0, 0.0], [r0, 0.0, 0.0]])), lj_eps=0.0, kb=kb)
    d["n_platelet"] = 1
    S = oracle_lib.System(d)
    n = 9
    xx, vv, _ = _run3(S, d, n, dt, k, k_if, k_sub, [level])
    h = k_sub * dt if level == 1 else dt
    steps = n * k * dt / h
    theta = np.arccos(1.0 - (4.0 * kb * h * h) / 2.0)
    r = xx[1, 0] - xx[0, 0]
    assert r == pytest.approx(r0 + q0 * np.cos(steps * theta), abs=1e-12)
    assert abs(xx[0, 0] + xx[1, 0] - (6.0 + r0 + q0)) < 1e-12


def test_inter_platelet_terms_stay_at_the_finest_step(oracle_lib):
    """Two one-bead platelets joined by a Morse bond: the bond is integrated at dt whatever
    the platelets' sublevels, exactly as in two-group RESPA at inner step dt."""
    x = np.array([[3.0, 3.0, 3.0], [4.2, 3.1, 3.0]])
    d = _tiny(x, 0, beads=dict(body=np.array([0, 1]), morse=np.array([[0, 1]]), platelet_area=np.ones(2)),
              lj_eps=0.0)
    d["n_platelet"] = 2
    d["v"][0] = [0.3, -0.2, 0.1]
    S = oracle_lib.System(d)
    dt, k = 0.0025, 8
    runs = [_run3(S, d, 7, dt, k, 4, 2, lv)[:2] for lv in ([1, 1], [2, 2], [1, 2])]
    for xx, vv in runs[1:]:
        assert np.array_equal(xx, runs[0][0]) and np.array_equal(vv, runs[0][1])
    x2, v2 = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x2, v2, 1, k * dt)
    fi = S.inner_forces(x2, v2, 1, dt)
    S.respa(x2, v2, fo, fi, [2, 2], 7, k * dt, k)
    assert np.max(np.abs(runs[0][0] - x2)) < 1e-13


def test_interface_random_term_scaled_by_the_interface_step(oracle_lib):
    """Free beads coupled to a DPD fluid at kT = 1 by the interface's dissipative + random
    terms only (WCA off), evaluated every k_if = 2 inner steps: they equilibrate at kT when
    the random term is scaled by 1/sqrt(Delta t_m); scaled by the inner step instead it
    has twice the variance, which sigma_pf sqrt(2) reproduces here: far hotter."""
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
        lv = np.full(nb, 1, np.int32)
        x, v = d["x"].copy(), d["v"].copy()
        dt, k, k_if = 0.0025, 4, 2
        fo = S.outer_forces(x, v, 0, k * dt)
        fm, f1, f2 = S.inner_forces3(x, v, 0, k_if * dt, lv)
        cnt = S.respa3(x, v, fo, fm, f1, f2, [1, 1], 200, dt, k, k_if, 2, lv)
        T = []
        for _ in range(200):
            cnt = S.respa3(x, v, fo, fm, f1, f2, cnt, 5, dt, k, k_if, 2, lv)
            T.append(np.mean(v[nf:] ** 2))
        return float(np.mean(T))

    assert abs(bead_T(3.0) - 1.0) < 0.06
    assert bead_T(3.0 * np.sqrt(2.0)) > 1.5


def test_conservative_three_level_energy_order_and_reversibility(oracle_lib):
    d = _small_platelet(gamma=0.0, sigma=0.0, gamma_pf=0.0, sigma_pf=0.0)
    S = oracle_lib.System(d)
    d["v"] *= 0.3
    lv = [1]
    flucts = []
    for dt in (0.001, 0.0005):
        x, v = d["x"].copy(), d["v"].copy()
        k = 8
        fo = S.outer_forces(x, v, 0, k * dt)
        fm, f1, f2 = S.inner_forces3(x, v, 0, 4 * dt, lv)
        cnt = [1, 1]
        E = []
        for _ in range(25):
            cnt = S.respa3(x, v, fo, fm, f1, f2, cnt, int(round(0.016 / (k * dt))), dt, k, 4, 2, lv)
            E.append(0.5 * np.sum(v * v) + np.sum(S.energy(x)[:5]))
        flucts.append(np.std(E))
    assert 4.0 * 0.75 < flucts[0] / flucts[1] < 4.0 * 1.25
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, 0, 0.008)
    fm, f1, f2 = S.inner_forces3(x, v, 0, 0.004, lv)
    S.respa3(x, v, fo, fm, f1, f2, [1, 1], 40, 0.001, 8, 4, 2, lv)
    v *= -1.0
    S.respa3(x, v, fo, fm, f1, f2, [1, 1], 40, 0.001, 8, 4, 2, lv)
    dx = x - d["x"]
    dx -= 8.0 * np.round(dx / 8.0)
    assert np.max(np.abs(dx)) < 1e-9
