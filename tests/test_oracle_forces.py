"""Pins of the oracle's force laws (Sec. 3.2, Eqs. 1-4) against things other than itself:
energy gradients by central finite differences, special points of the potentials,
Newton's third law, brute-force pair sets, and physical invariants."""
import numpy as np
import pytest

import synth


def _tiny(x, n_fluid, n_wall=0, L=(6.0, 6.0, 6.0), periodic=(1, 1, 1), beads=None, **par):
    """A hand-built system: fluid/wall particles then optional beads of one or two platelets."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    nb = n - n_fluid - n_wall
    d = dict(box_lo=np.zeros(3), box_L=np.asarray(L, float), periodic=periodic, n_fluid=n_fluid, n_wall=n_wall,
             n_bead=nb, n_platelet=0, x=x, v=np.zeros_like(x), body=np.zeros(nb, np.int32),
             rest=np.zeros((nb, 3)), bonds=np.zeros((0, 2), np.int32), bond_r0=np.zeros(0),
             angles=np.zeros((0, 3), np.int32), angle_th0=np.zeros(0), morse=np.zeros((0, 2), np.int32),
             platelet_area=np.ones(1), params=synth.dpd_params(**par), n=n)
    if beads:
        d.update(beads)
    for k in ("x", "v", "rest", "bond_r0", "angle_th0", "platelet_area"):
        d[k] = np.ascontiguousarray(d[k], dtype=np.float64)
    for k in ("body", "bonds", "angles", "morse"):
        d[k] = np.ascontiguousarray(d[k], dtype=np.int32)
    return d


def _fd_grad(efun, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(x.shape[0]):
        for k in range(3):
            xp = x.copy()
            xm = x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            g[i, k] = (efun(xp) - efun(xm)) / (2 * h)
    return g


def test_dpd_conservative_is_minus_grad_of_energy(oracle_lib):
    rng = np.random.default_rng(1)
    x = rng.random((40, 3)) * 3.0
    d = _tiny(x, 40, L=(3.0, 3.0, 3.0), gamma=0.0, sigma=0.0)
    S = oracle_lib.System(d)
    f = S.outer_forces(x, d["v"], 0, 0.01, brute=True)
    g = _fd_grad(lambda y: S.energy(y)[0], x)
    assert np.max(np.abs(f + g)) / np.max(np.abs(f)) < 1e-8


def test_dpd_two_particle_special_values(oracle_lib):
    # r = 0.5 along x: conservative force a (1 - r/rc) = 12.5, repulsive on the first particle
    x = np.array([[2.5, 3.0, 3.0], [2.0, 3.0, 3.0]])
    d = _tiny(x, 2, gamma=0.0, sigma=0.0)
    f = oracle_lib.System(d).outer_forces(x, d["v"], 0, 0.01, brute=True)
    assert f[0, 0] == pytest.approx(12.5, rel=1e-15) and f[1, 0] == pytest.approx(-12.5, rel=1e-15)
    assert np.all(f[:, 1:] == 0.0)
    # at and beyond the cutoff the pair contributes nothing
    x2 = np.array([[2.0, 3.0, 3.0], [3.0, 3.0, 3.0]])
    assert np.all(oracle_lib.System(_tiny(x2, 2)).outer_forces(x2, np.ones((2, 3)), 0, 0.01, brute=True) == 0.0)
    # minimum image across the periodic boundary: same force as the unwrapped pair
    x3 = np.array([[0.1, 3.0, 3.0], [5.6, 3.0, 3.0]])
    f3 = oracle_lib.System(_tiny(x3, 2, gamma=0.0, sigma=0.0)).outer_forces(x3, np.zeros((2, 3)), 0, 0.01, brute=True)
    assert f3[0, 0] == pytest.approx(25.0 * 0.5, rel=1e-12)


def test_dpd_pair_antisymmetric_bitwise_and_momentum(oracle_lib):
    d = synth.dpd_box(n=600, L=(5.0, 5.0, 5.0), seed=3)
    S = oracle_lib.System(d)
    f = S.outer_forces(d["x"], d["v"], 17, 0.01, brute=True)
    assert np.all(np.abs(f.sum(axis=0)) < 1e-10 * np.abs(f).sum())
    x = np.array([[1.0, 1.0, 1.0], [1.3, 1.4, 0.9]])
    v = np.array([[0.3, -1.0, 2.0], [-0.7, 0.2, 0.1]])
    d2 = _tiny(x, 2)
    f2 = oracle_lib.System(d2).outer_forces(x, v, 5, 0.01, brute=True)
    assert np.array_equal(f2[0], -f2[1])


def test_cell_list_equals_brute_force(oracle_lib):
    d = synth.dpd_box(n=3000, seed=4)
    S = oracle_lib.System(d)
    pb = S.pairs(d["x"], d["n"], 1.0, cells=False)
    pc = S.pairs(d["x"], d["n"], 1.0, cells=True)
    sb = set(map(tuple, pb))
    sc = set(map(tuple, pc))
    assert sb == sc and len(pc) == len(sc)
    # the expected count of pairs within rc at density 3: N * (4 pi/3) * rho / 2
    assert abs(len(sb) / (3000 * 4 * np.pi / 3 * 3 / 2) - 1) < 0.05
    fb = S.outer_forces(d["x"], d["v"], 3, 0.01, brute=True)
    fc = S.outer_forces(d["x"], d["v"], 3, 0.01, brute=False)
    assert np.max(np.abs(fb - fc)) < 1e-11 * np.max(np.abs(fb))


def test_dissipation_is_galilean_invariant_and_removes_energy(oracle_lib):
    d = synth.dpd_box(n=600, L=(5.0, 5.0, 5.0), seed=5, a=0.0, sigma=0.0)
    S = oracle_lib.System(d)
    f = S.outer_forces(d["x"], d["v"], 0, 0.01, brute=True)
    f2 = S.outer_forces(d["x"], d["v"] + np.array([0.7, -2.0, 5.0]), 0, 0.01, brute=True)
    assert np.max(np.abs(f - f2)) < 1e-12 * np.max(np.abs(f))
    assert np.sum(f * d["v"]) < 0.0  # dissipative power is negative


def test_lj_special_points_and_gradient(oracle_lib):
    sig = 0.8
    rmin = sig * 2 ** (1 / 6)
    # two beads of different platelets at the WCA cutoff: zero force, zero energy
    for r, fexp in ((rmin * (1 - 1e-12), 0.0), (rmin * (1 + 1e-9), 0.0)):
        x = np.array([[3.0, 3.0, 3.0], [3.0 + r, 3.0, 3.0]])
        d = _tiny(x, 0, beads=dict(body=np.array([0, 1])), gamma_pf=0.0, sigma_pf=0.0)
        S = oracle_lib.System(d)
        f = S.inner_forces(x, d["v"], 0, 0.01, brute=True)
        assert np.max(np.abs(f)) < 1e-9
        assert abs(S.energy(x)[1]) < 1e-9
    # at r = sigma: U = eps (shift), |F| = 24 eps / sigma
    x = np.array([[3.0, 3.0, 3.0], [3.0 + sig, 3.0, 3.0]])
    d = _tiny(x, 0, beads=dict(body=np.array([0, 1])))
    S = oracle_lib.System(d)
    f = S.inner_forces(x, d["v"], 0, 0.01, brute=True)
    assert f[0, 0] == pytest.approx(-24.0 / sig, rel=1e-13) and f[1, 0] == pytest.approx(24.0 / sig, rel=1e-13)
    assert S.energy(x)[1] == pytest.approx(1.0, rel=1e-13)
    # gradient of the LJ energy for a random cluster of beads and fluid (conservative part only)
    rng = np.random.default_rng(8)
    xb = 2.0 + rng.random((12, 3)) * 1.6
    xf = 2.0 + rng.random((10, 3)) * 1.6
    xx = np.concatenate([xf, xb])
    body = np.array([0] * 6 + [1] * 6, np.int32)
    d = _tiny(xx, 10, beads=dict(body=body, rest=rng.random((12, 3)) * 5.0), gamma_pf=0.0, sigma_pf=0.0)
    S = oracle_lib.System(d)
    f = S.inner_forces(xx, d["v"], 0, 0.01, brute=True)
    g = _fd_grad(lambda y: S.energy(y)[1], xx, h=1e-7)
    assert np.max(np.abs(f + g)) / np.max(np.abs(f)) < 1e-6


def test_same_platelet_exclusion_uses_rest_distance(oracle_lib):
    x = np.array([[3.0, 3.0, 3.0], [3.6, 3.0, 3.0]])
    for rest_sep, expect_force in ((1.0, False), (2.0, True)):
        rest = np.array([[0.0, 0.0, 0.0], [rest_sep, 0.0, 0.0]])
        d = _tiny(x, 0, beads=dict(body=np.array([0, 0]), rest=rest))
        f = oracle_lib.System(d).inner_forces(x, d["v"], 0, 0.01, brute=True)
        assert (np.max(np.abs(f)) > 1.0) == expect_force


def test_bonded_terms_are_minus_grad_of_energy(oracle_lib):
    tm = synth.platelet_template(level=1, semi_axes=(1.5, 0.5, 1.5))
    nb = tm["rest"].shape[0]
    rng = np.random.default_rng(9)
    x = tm["rest"] + 3.0 + 0.05 * rng.standard_normal((nb, 3))
    morse = np.array([[0, 5], [3, 20]], np.int32)
    d = _tiny(x, 0, L=(8.0, 8.0, 8.0), beads=dict(
        body=np.zeros(nb, np.int32), rest=tm["rest"] * 100.0, bonds=tm["bonds"], bond_r0=tm["bond_r0"],
        angles=tm["angles"], angle_th0=tm["angle_th0"], morse=morse), lj_eps=0.0)
    S = oracle_lib.System(d)
    f = S.inner_forces(x, d["v"], 0, 0.01, brute=True)
    g = _fd_grad(lambda y: S.energy(y)[2] + S.energy(y)[3] + S.energy(y)[4], x)
    assert np.max(np.abs(f + g)) / np.max(np.abs(f)) < 1e-7
    assert np.all(np.abs(f.sum(axis=0)) < 1e-10 * np.abs(f).sum())
    # at rest every bond and angle force vanishes
    d0 = dict(d)
    d0["morse"] = np.zeros((0, 2), np.int32)
    S0 = oracle_lib.System(d0)
    f0 = S0.inner_forces(tm["rest"] + 3.0, d["v"], 0, 0.01, brute=True)
    assert np.max(np.abs(f0)) < 1e-9


def test_morse_special_points(oracle_lib):
    for r, fexp in ((1.0, 0.0),):
        x = np.array([[3.0, 3.0, 3.0], [3.0 + r, 3.0, 3.0]])
        d = _tiny(x, 0, beads=dict(body=np.array([0, 1]), morse=np.array([[0, 1]])), lj_eps=0.0)
        S = oracle_lib.System(d)
        assert np.max(np.abs(S.inner_forces(x, d["v"], 0, 0.01, brute=True))) < 1e-13
        assert S.energy(x)[4] == pytest.approx(-5.0, rel=1e-14)
    # stretched: attractive with |F| = 2 a D (e^{-2a dr} - e^{-a dr}) at dr = 0.25
    x = np.array([[3.0, 3.0, 3.0], [4.25, 3.0, 3.0]])
    d = _tiny(x, 0, beads=dict(body=np.array([0, 1]), morse=np.array([[0, 1]])), lj_eps=0.0)
    f = oracle_lib.System(d).inner_forces(x, d["v"], 0, 0.01, brute=True)
    assert f[0, 0] == pytest.approx(-2 * 2 * 5 * (np.exp(-1.0) - np.exp(-0.5)), rel=1e-13)


def test_inner_forces_cells_equal_brute_and_conserve_momentum(oracle_lib):
    d = synth.platelet_box(n_fluid=3000, L=(10.0, 10.0, 10.0), level=2, semi_axes=(2.0, 0.8, 2.0), seed=11)
    S = oracle_lib.System(d)
    fb = S.inner_forces(d["x"], d["v"], 9, 0.0025, brute=True)
    fc = S.inner_forces(d["x"], d["v"], 9, 0.0025, brute=False)
    assert np.max(np.abs(fb - fc)) < 1e-11 * np.max(np.abs(fb))
    assert np.all(np.abs(fb.sum(axis=0)) < 1e-10 * np.abs(fb).sum())
    assert np.count_nonzero(np.abs(fb[:d["n_fluid"]]).sum(axis=1)) > 20  # fluid feels the platelet
