"""Three-level MTS with per-platelet sublevels (Sec. 3.3, Table 1) on the HIP path,
through the C ABI, against the oracle's three-level scheme: the forces of each group
(interface M, flowing sublevel P1, aggregating sublevel P2) per step, trajectories over
about 100 inner steps, the reduction to two-group RESPA, the controller's per-platelet
sublevels (Table 2, rows 5-6) and a checkpoint of a three-level run."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2205_14121_amd", "data",
                       "controller.npy")


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


def _aggregate():
    return synth.aggregate_box()  # two level-3 platelets stacked 1.0 apart, Morse bonds


CASES = {
    "platelet_box_level1": (lambda: synth.platelet_box(), [1], 4, 2, 2),
    "aggregate_levels_1_2": (_aggregate, [1, 2], 8, 4, 2),
    "aggregate_levels_2_1": (_aggregate, [2, 1], 8, 2, 1),
}


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_group_forces_match_oracle(A, oracle_lib, name, fp32):
    mk, level, k, k_if, k_sub = CASES[name]
    d = dict(mk())
    # the generated platelets sit in their rest shapes, where bonds and angles exert
    # round-off forces only: jitter the beads so that every group carries real forces
    b0 = int(d["n_fluid"] + d["n_wall"])
    d["x"] = d["x"].copy()
    d["x"][b0:] += np.random.default_rng(5).normal(0.0, 0.02, size=d["x"][b0:].shape)
    dt = 0.0025
    ctx = A.from_workload(d, fp32=fp32, skin=0.5, three_level=True)
    ctx.set_levels(k_if, k_sub, level)
    ctx.set_counters(7, 11)
    ctx.compute_forces(dt, k)
    gm, g1, g2 = ctx.level_forces()
    fo, fi = ctx.forces()
    S = oracle_lib.System(d)
    rm, r1, r2 = S.inner_forces3(d["x"], d["v"], 11, k_if * dt, level)
    ro = S.outer_forces(d["x"], d["v"], 7, k * dt)
    tol = 1e-5 if fp32 else 1e-10
    errs = [rel_rms(g, r) for g, r in ((gm, rm), (g1, r1), (g2, r2))]
    print("%s fp32=%s: group rel RMS M %.2e P1 %.2e P2 %.2e, outer %.2e" % (name, fp32, *errs, rel_rms(fo, ro)))
    assert max(errs) <= tol and rel_rms(fo, ro) <= tol
    # the whole inner force is the sum of the groups
    assert np.max(np.abs(fi - (gm + g1 + g2))) <= 1e-12 * max(1.0, np.max(np.abs(fi)))
    for g, r in ((g1, r1), (g2, r2)):
        assert np.array_equal(np.any(g != 0.0, axis=1), np.any(r != 0.0, axis=1))


@pytest.mark.parametrize("name", list(CASES))
def test_trajectory_matches_oracle(A, oracle_lib, name):
    """About 100 inner steps in float64 from identical state and counters."""
    mk, level, k, k_if, k_sub = CASES[name]
    d = mk()
    dt = 0.0025
    n_outer = 100 // k
    ctx = A.from_workload(d, skin=0.5, three_level=True)
    ctx.set_levels(k_if, k_sub, level)
    ctx.set_counters(3, 5)
    ctx.compute_forces(dt, k)
    ctx.step(n_outer, dt, k)
    xg, vg = ctx.state()
    S = oracle_lib.System(d)
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, 3, k * dt)
    fm, f1, f2 = S.inner_forces3(x, v, 5, k_if * dt, level)
    cnt = S.respa3(x, v, fo, fm, f1, f2, [4, 6], n_outer, dt, k, k_if, k_sub, level)
    err = max_image_dx(xg, x, d)
    print("%s: %d outer steps (k=%d, k_if=%d, k_sub=%d), max |dx| %.3e, counters gpu %s oracle %s"
          % (name, n_outer, k, k_if, k_sub, err, ctx.counters(), list(cnt)))
    assert ctx.counters() == tuple(int(c) for c in cnt)
    assert err <= 1e-8


def test_reduces_to_two_group_when_levels_coincide(A):
    d = synth.platelet_box()
    out = []
    for three in (False, True):
        ctx = A.from_workload(d, skin=0.5, three_level=three)
        if three:
            ctx.set_levels(1, 1, [2])
        ctx.set_counters(3, 5)
        ctx.compute_forces(0.0025, 4)
        ctx.step(10, 0.0025, 4)
        out.append(ctx.state())
        ctx.close()
    dx = max_image_dx(out[0][0], out[1][0], d)
    print("three-level at k_if = k_sub = 1 against two-group RESPA: max |dx| %.3e" % dx)
    assert dx < 1e-12


def test_controller_sets_the_sublevels(A):
    """In controller mode, every decision sets each platelet's sublevel from its own
    prediction: sublevel 1 above the system's ratio (the minimum over platelets, capped
    at k_max), 2 otherwise.  The first decision falls at the end of the 64th outer step,
    on the window that aimts_get_feature_window returns right after it."""
    import torch
    d = synth.channel(n_total=60000, L=(40.0, 20.0, 25.0), n_platelet=3, level=3, seed=78, g=0.05)
    ctx = A.from_workload(d, fp32=True, skin=0.5, series_capacity=200, ctrl_max_batch=8, three_level=True)
    ctx.ctrl_set_weights(np.load(WEIGHTS).astype(np.float32))
    ctx.set_levels(2, 2)
    assert ctx.levels()[2].tolist() == [2, 2, 2]
    ctx.compute_forces(0.0025, 4)
    ctx.step(64, 0.0025, 4, mode=1, diag_every=1, k_max=8)
    dg = ctx.diag()
    assert dg.inferences == 1
    k_if, k_sub, lv = ctx.levels()
    win = torch.from_numpy(ctx.feature_window()).cuda()
    logits = torch.empty(win.shape[0], 9, device="cuda")
    ctx.ctrl_forward(win, None, logits)
    r = np.array([1, 2, 4, 8, 16])[logits[:, :5].argmax(dim=1).cpu().numpy()]
    k_sys = min(int(r.min()), 8)
    expect = np.where(r > k_sys, 1, 2)
    print("per-platelet predicted ratios %s, system ratio %d (in force %d), sublevels %s"
          % (r.tolist(), k_sys, dg.k, lv.tolist()))
    assert (k_if, k_sub) == (2, 2) and dg.k == k_sys
    assert np.array_equal(lv, expect)
    # and the run goes on at those sublevels
    ctx.step(8, 0.0025, 4, mode=1, diag_every=1, k_max=8)
    x, v = ctx.state()
    assert np.isfinite(x).all() and np.isfinite(v).all()


def test_three_level_checkpoint_resume_is_bitwise(A):
    d = _aggregate()
    dt, k, n = 0.0025, 8, 6

    def ctx():
        c = A.from_workload(d, skin=0.5, series_capacity=64, three_level=True)
        c.set_levels(4, 2, [1, 2])
        return c

    ref = ctx()
    ref.compute_forces(dt, k)
    ref.step(2 * n, dt, k, diag_every=1)
    x_ref, v_ref = ref.state()
    a = ctx()
    a.compute_forces(dt, k)
    a.step(n, dt, k, diag_every=1)
    blob = a.save_checkpoint()
    b = A.from_workload(d, skin=0.5, series_capacity=64, three_level=True)
    b.load_checkpoint(blob)
    assert b.levels()[:2] == (4, 2) and b.levels()[2].tolist() == [1, 2]
    b.step(n, dt, k, diag_every=1)
    x, v = b.state()
    assert np.array_equal(x, x_ref) and np.array_equal(v, v_ref)
    assert np.array_equal(b.series(), ref.series())
