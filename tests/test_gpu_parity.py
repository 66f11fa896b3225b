"""Parity of the HIP path (through the C ABI) with the CPU oracle on identical seeded
inputs and identical random-number counters.

Tolerances (float64 forces): relative RMS force error <= 1e-10 per force group;
positions after 100 outer steps within 1e-8 (minimum image).  Float32 pair forces:
relative RMS error <= 1e-5 against the float64 oracle.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

REL_RMS_F64 = 1e-10
POS_TOL = 1e-8
REL_RMS_F32 = 1e-5


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14121_amd.aimts as A
    return A


def rel_rms(a, b):
    den = np.sum(b * b)
    return float(np.sqrt(np.sum((a - b) ** 2) / den)) if den > 0 else float(np.sqrt(np.sum(a * a)))


def max_image_dx(a, b, sysd):
    d = a - b
    L = np.asarray(sysd["box_L"])
    for k in range(3):
        if sysd["periodic"][k]:
            d[:, k] -= L[k] * np.round(d[:, k] / L[k])
    return float(np.max(np.abs(d)))


def _c0():
    return synth.dpd_box()


def _c1():
    return synth.platelet_box()


def _small_channel():
    return synth.channel(n_total=60000, L=(40.0, 20.0, 25.0), n_platelet=2, level=3, seed=77, g=0.05)


def _forces_case(A, oracle_lib, sysd, k, dt_inner, fp32=False, counters=(5, 9), diag=None, **kw):
    ctx = A.from_workload(sysd, fp32=fp32, **kw)
    ctx.set_counters(*counters)
    ctx.compute_forces(dt_inner, k)
    if diag is not None:
        diag.append(ctx.diag())
    fo, fi = ctx.forces()
    S = oracle_lib.System(sysd)
    ro = S.outer_forces(sysd["x"], sysd["v"], counters[0], k * dt_inner)
    ri = S.inner_forces(sysd["x"], sysd["v"], counters[1], dt_inner)
    assert ctx.counters() == (counters[0] + 1, counters[1] + 1)
    return fo, fi, ro, ri


def test_c0_outer_forces_f64(A, oracle_lib):
    d = _c0()
    fo, fi, ro, ri = _forces_case(A, oracle_lib, d, 1, 0.01)
    print("C0 F_outer rel RMS", rel_rms(fo, ro))
    assert rel_rms(fo, ro) <= REL_RMS_F64
    assert np.all(fi == 0.0) and np.all(ri == 0.0)
    assert np.all(np.abs(fo.sum(axis=0)) < 1e-9)


def test_c1_both_groups_f64(A, oracle_lib):
    d = _c1()
    fo, fi, ro, ri = _forces_case(A, oracle_lib, d, 4, 0.0025)
    eo, ei = rel_rms(fo, ro), rel_rms(fi, ri)
    print("C1 F_outer rel RMS %.3e  F_inner rel RMS %.3e" % (eo, ei))
    assert eo <= REL_RMS_F64 and ei <= REL_RMS_F64
    # fluid starts >= lj_sig from every bead, so only a thin shell [0.8, 1.0) feels the membrane
    assert np.count_nonzero(np.abs(fi[:d["n_fluid"]]).sum(axis=1)) > 50


def test_c1_wide_skins_long_lists(A, oracle_lib):
    """Skins of 1.5 for fluid and beads: bead lists of 424-834 partners (counted on the CPU
    from the same layout: 1,098 of the 2,562 beads have more than the 512 kept by the
    counting pass), so the re-scan path writes those lists and counts their fluid
    members' partners; forces must not change."""
    d = _c1()
    dg = []
    fo, fi, ro, ri = _forces_case(A, oracle_lib, d, 4, 0.0025, skin=1.5, skin_bead=1.5, diag=dg)
    eo, ei = rel_rms(fo, ro), rel_rms(fi, ri)
    print("C1 wide skins: F_outer rel RMS %.3e  F_inner rel RMS %.3e, %d beads scanned again"
          % (eo, ei, dg[0].rescanned))
    assert eo <= REL_RMS_F64 and ei <= REL_RMS_F64
    assert dg[0].rescanned > 0


@pytest.mark.parametrize("fp32", [False, True])
def test_dense_fluid_forces(A, oracle_lib, fp32):
    """Density 12 (about 50 partners per particle): every per-thread partner list of the
    DPD kernel overflows its buffer mid-scan, so the overflow path is exercised."""
    d = synth.dpd_box(n=12000, seed=4242)
    fo, fi, ro, ri = _forces_case(A, oracle_lib, d, 1, 0.01, fp32=fp32)
    e = rel_rms(fo, ro)
    print("dense fluid F_outer rel RMS (fp32=%s) %.3e" % (fp32, e))
    assert e <= (REL_RMS_F32 if fp32 else REL_RMS_F64)


def test_small_channel_forces_f64(A, oracle_lib):
    d = _small_channel()
    fo, fi, ro, ri = _forces_case(A, oracle_lib, d, 8, 0.0025, counters=(123, 456))
    eo, ei = rel_rms(fo, ro), rel_rms(fi, ri)
    print("channel F_outer rel RMS %.3e  F_inner rel RMS %.3e" % (eo, ei))
    assert eo <= REL_RMS_F64 and ei <= REL_RMS_F64
    nf, nw = d["n_fluid"], d["n_wall"]
    assert np.all(fo[nf:nf + nw] == 0.0) and np.all(fi[nf:nf + nw] == 0.0)


@pytest.mark.parametrize("case", ["c0", "c1"])
def test_fp32_pair_forces_error(A, oracle_lib, case):
    d = _c0() if case == "c0" else _c1()
    k = 1 if case == "c0" else 4
    dt = 0.01 if case == "c0" else 0.0025
    fo, fi, ro, ri = _forces_case(A, oracle_lib, d, k, dt, fp32=True)
    eo = rel_rms(fo, ro)
    print("%s float32 forces: F_outer rel RMS %.3e" % (case, eo))
    assert eo <= REL_RMS_F32
    if case == "c1":
        ei = rel_rms(fi, ri)
        print("%s float32 forces: F_inner rel RMS %.3e" % (case, ei))
        assert ei <= REL_RMS_F32


def _oracle_run(oracle_lib, sysd, n_outer, k, dt_inner, perturb=0.0):
    S = oracle_lib.System(sysd)
    x, v = sysd["x"].copy(), sysd["v"].copy()
    if perturb:
        x = x * (1.0 + perturb * np.random.default_rng(0).standard_normal(x.shape))
    fo = S.outer_forces(x, v, 0, k * dt_inner)
    fi = S.inner_forces(x, v, 0, dt_inner)
    S.respa(x, v, fo, fi, [1, 1], n_outer, k * dt_inner, k)
    return x, v


def _gpu_run(A, sysd, n_outer, k, dt_inner, skin=0.4):
    ctx = A.from_workload(sysd, skin=skin)
    ctx.set_counters(0, 0)
    ctx.compute_forces(dt_inner, k)
    ctx.step(n_outer, dt_inner, k)
    x, v = ctx.state()
    return x, v, ctx


def test_c0_trajectory_100_steps(A, oracle_lib):
    d = _c0()
    xg, vg, ctx = _gpu_run(A, d, 100, 1, 0.01)
    xo, vo = _oracle_run(oracle_lib, d, 100, 1, 0.01)
    err = max_image_dx(xg, xo, d)
    print("C0 100-step max |dx| %.3e  max |dv| %.3e" % (err, np.max(np.abs(vg - vo))))
    assert err <= POS_TOL
    assert ctx.counters() == (101, 101)


@pytest.mark.parametrize("case,k", [("c1", 4), ("channel", 8), ("c1", 1), ("c1", 3), ("channel", 3)],
                         ids=["c1_k4", "channel_k8", "c1_k1", "c1_k3", "channel_k3"])
def test_trajectory_100_inner_steps(A, oracle_lib, case, k):
    """About 100 steps of the finest (inner) level: 25 outer steps at k = 4, 12 at k = 8,
    100 at k = 1 and 33 at k = 3.  An odd ratio sends the members' first drift to the
    second state buffer (and the frozen walls of the channel with it), an even one keeps
    it in place: both orders of the buffer alternation are covered."""
    d = _c1() if case == "c1" else _small_channel()
    n_outer = 100 // k
    xg, vg, ctx = _gpu_run(A, d, n_outer, k, 0.0025)
    xo, vo = _oracle_run(oracle_lib, d, n_outer, k, 0.0025)
    err = max_image_dx(xg, xo, d)
    print("%s %d outer steps (k=%d) max |dx| %.3e" % (case, n_outer, k, err))
    assert err <= POS_TOL
    if case == "channel":
        nf, nw = d["n_fluid"], d["n_wall"]
        assert np.array_equal(xg[nf:nf + nw], d["x"][nf:nf + nw])  # frozen walls


@pytest.mark.parametrize("case", ["c1", "channel"])
def test_long_trajectory_within_intrinsic_chaos(A, oracle_lib, case):
    """Over longer windows any roundoff-level difference grows exponentially (the
    platelet is chaotic): the GPU may not drift from the oracle by more than ten times
    the oracle's own divergence from a copy of itself started 1e-15 (relative) away."""
    d, k, n_outer = (_c1(), 4, 100) if case == "c1" else (_small_channel(), 8, 40)
    xg, vg, ctx = _gpu_run(A, d, n_outer, k, 0.0025)
    xo, vo = _oracle_run(oracle_lib, d, n_outer, k, 0.0025)
    xp, vp = _oracle_run(oracle_lib, d, n_outer, k, 0.0025, perturb=1e-15)
    err = max_image_dx(xg, xo, d)
    chaos = max_image_dx(xp, xo, d)
    print("%s %d outer steps (k=%d): gpu-oracle %.3e, oracle self-divergence %.3e" % (case, n_outer, k, err, chaos))
    assert err <= max(POS_TOL, 10.0 * chaos)


def test_bitwise_determinism(A):
    d = _c1()
    out = []
    for _ in range(2):
        ctx = A.from_workload(d)
        ctx.compute_forces(0.0025, 4)
        ctx.step(10, 0.0025, 4)
        out.append(ctx.state())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_momentum_conserved_periodic(A):
    d = _c1()
    ctx = A.from_workload(d)
    ctx.compute_forces(0.0025, 4)
    p0 = ctx.diag().p[:]
    ctx.step(50, 0.0025, 4)
    p1 = ctx.diag().p[:]
    assert np.max(np.abs(np.array(p1) - np.array(p0))) < 1e-9


def test_thermo_and_energy_match_oracle(A, oracle_lib):
    d = _small_channel()
    ctx = A.from_workload(d)
    ctx.compute_forces(0.0025, 4)
    ctx.step(5, 0.0025, 4)
    x, v = ctx.state()
    g = ctx.diag(energy=True)
    S = oracle_lib.System(d)
    ke, T, Tp, px, py, pz = S.thermo(x, v, bin_axis=1)
    assert g.ke == pytest.approx(ke, rel=1e-12) and g.T == pytest.approx(T, rel=1e-12)
    assert g.T_pec == pytest.approx(Tp, rel=1e-10)
    assert np.allclose(g.p[:], [px, py, pz], rtol=0, atol=1e-9)
    c0 = _c1()
    ctx0 = A.from_workload(c0)
    ctx0.compute_forces(0.0025, 4)
    g0 = ctx0.diag(energy=True)
    e = oracle_lib.System(c0).energy(c0["x"])
    got = np.array(list(g0.pe[:]) + [g0.virial])
    print("energies gpu", got, "oracle", e)
    assert np.allclose(got, e, rtol=1e-10, atol=1e-8)


def test_features_match_oracle(A, oracle_lib):
    d = _small_channel()
    ctx = A.from_workload(d)
    ctx.compute_forces(0.0025, 4)
    ctx.step(3, 0.0025, 4)
    x, v = ctx.state()
    _, feat = ctx.diag(features=True)
    ref = oracle_lib.System(d).features(x, v)
    print("features gpu", feat, "oracle", ref)
    assert np.allclose(feat, ref.astype(np.float32), rtol=2e-6, atol=1e-6)


def test_aggregate_with_morse_bonds(A, oracle_lib):
    """Two stacked platelets bound by inter-platelet Morse bonds (Eq. 2, Eq. 4): forces and
    100 inner steps against the oracle."""
    d = synth.aggregate_box()
    assert d["morse"].shape[0] > 50
    fo, fi, ro, ri = _forces_case(A, oracle_lib, d, 4, 0.0025, counters=(7, 3))
    eo, ei = rel_rms(fo, ro), rel_rms(fi, ri)
    print("aggregate F_outer rel RMS %.3e  F_inner rel RMS %.3e" % (eo, ei))
    assert eo <= REL_RMS_F64 and ei <= REL_RMS_F64
    xg, vg, ctx = _gpu_run(A, d, 25, 4, 0.0025)
    xo, vo = _oracle_run(oracle_lib, d, 25, 4, 0.0025)
    err = max_image_dx(xg, xo, d)
    print("aggregate 25 outer steps (k=4) max |dx| %.3e" % err)
    assert err <= POS_TOL


def _mini_clot():
    # the recipe of the largest system at a size the oracle evaluates in about a second:
    # level-5 platelets in a packed 1 x 2 x 2 aggregate on the lower wall with mutual-nearest
    # Morse bonds, walls in y
    return synth.clot_channel(n_total=6_200, L=(14.0, 12.0, 14.8), n_free=0, n_packed=4, packed_grid=(1, 2, 2))


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_mini_clot_forces(A, oracle_lib, fp32):
    """Level-5 platelets in a packed aggregate (the largest system's recipe, with its short
    bead-bead skin): both force groups against the oracle."""
    d = _mini_clot()
    assert d["morse"].shape[0] > 100
    fo, fi, ro, ri = _forces_case(A, oracle_lib, d, 8, 0.00125, fp32=fp32, counters=(21, 34), skin=0.5, skin_bead=0.2)
    eo, ei = rel_rms(fo, ro), rel_rms(fi, ri)
    print("mini clot (fp32=%s) F_outer rel RMS %.3e  F_inner rel RMS %.3e" % (fp32, eo, ei))
    tol = REL_RMS_F32 if fp32 else REL_RMS_F64
    assert eo <= tol and ei <= tol


def test_angle_pass_modes_agree_bitwise(A):
    """The separate angle pass (one thread per angle, gathered by the beads) and the
    in-kernel evaluation (every bead evaluates its own angle entries) give the same
    inner forces and trajectories bit for bit."""
    d = _c1()
    out = []
    for mode in (1, 2):
        ctx = A.from_workload(d, angle_pass=mode)
        ctx.set_counters(3, 7)
        ctx.compute_forces(0.0025, 4)
        fo, fi = ctx.forces()
        ctx.step(10, 0.0025, 4)
        x, v = ctx.state()
        out.append((fi, x, v))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def test_features_hand_layout(A, oracle_lib):
    """The hand-counted layout of the oracle's feature pin (interfacial traction of a bead
    at sigma_LJ from a fluid particle, contacts with a wall particle and with a bead of
    the other platelet at 0.95, none at 1.05) through the HIP path."""
    from test_oracle_integrator import _feature_layout
    d = _feature_layout()
    ctx = A.from_workload(d, skin=0.4)
    ctx.compute_forces(0.0025, 4)
    _, feat = ctx.diag(features=True)
    ref = oracle_lib.System(d).features(d["x"], d["v"])
    print("hand layout features gpu", feat[:, 6:], "oracle", ref[:, 6:])
    assert feat[0, 6] == pytest.approx((-11.52 + 0.06912) / 2.0, rel=1e-6)
    assert feat[1, 6] == 0.0 and feat[0, 7] == 2.0 and feat[1, 7] == 1.0
    assert np.allclose(feat, ref.astype(np.float32), rtol=2e-6, atol=1e-6)


def test_step_features_equal_diag_features(A):
    """An outer step takes its features before its closing half kick, with the fluid
    partners' end-of-step velocities formed from the pending kick (shear traction); the
    window row it writes must equal the features that aimts_get_diag computes for the
    same state after the kick.  The two platelets bound by Morse bonds have ~100
    contacts each.  The window exists after 64 outer steps."""
    d = synth.aggregate_box()
    ctx = A.from_workload(d)
    ctx.compute_forces(0.0025, 4)
    ctx.step(64, 0.0025, 4)
    w = ctx.feature_window()
    _, feat = ctx.diag(features=True)
    print("step row", w[:, -1, :], "diag", feat)
    assert np.all(feat[:, 7] > 0) and np.all(feat[:, 6] != 0)
    assert np.allclose(w[:, -1, :], feat, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("skin_bead", [0.02, 0.2])
def test_mini_clot_features_with_contacts(A, oracle_lib, skin_bead):
    """Features of the packed aggregate after 10 outer steps, once the Morse bonds have
    drawn facing beads within the contact radius: hundreds of contacts per platelet,
    counted exactly as the oracle counts them, also with a bead skin far below the gap
    between the WCA cutoff and the contact radius."""
    d = _mini_clot()
    run = A.from_workload(d, skin=0.5, skin_bead=0.2)
    run.compute_forces(0.00125, 4)
    run.step(10, 0.00125, 4)
    x, v = run.state()
    run.close()
    dd = dict(d)
    dd["x"], dd["v"] = x, v
    ctx = A.from_workload(dd, skin=0.5, skin_bead=skin_bead)
    ctx.compute_forces(0.00125, 4)
    _, feat = ctx.diag(features=True)
    ref = oracle_lib.System(d).features(x, v)
    print("mini clot contacts gpu", feat[:, 7], "oracle", ref[:, 7])
    assert np.all(ref[:, 7] > 0)
    assert np.array_equal(feat[:, 7], ref[:, 7].astype(np.float32))
    assert np.allclose(feat, ref.astype(np.float32), rtol=2e-6, atol=1e-6)
