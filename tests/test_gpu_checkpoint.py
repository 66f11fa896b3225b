"""Checkpoint and resume through the C ABI: n outer steps, a checkpoint, a fresh context
loaded from it and n more steps give bit for bit the state, the diagnostics series and
the controller's decisions of 2n uninterrupted steps."""
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


def _ctx(A, d, fp32, weights):
    ctx = A.from_workload(d, fp32=fp32, skin=0.5, series_capacity=400, ctrl_max_batch=8)
    if weights is not None:
        ctx.ctrl_set_weights(weights)
    return ctx


CASES = {
    # float64 forces at a fixed ratio (the oracle-parity configuration of the platelet box)
    "platelet_box_fixed_k4": dict(d=lambda: synth.platelet_box(), fp32=False, n=20, k=4, mode=0, rollback=0),
    # float32 pair forces under the learned controller (its first decision after 64 steps
    # falls in the first half), in checkpointed rollback segments of 16
    "channel_controller": dict(d=lambda: synth.channel(n_total=60000, L=(40.0, 20.0, 25.0), n_platelet=2, level=3,
                                                        seed=77, g=0.05), fp32=True, n=80, k=4, mode=1, rollback=16),
}


@pytest.mark.parametrize("name", list(CASES))
def test_resume_is_bitwise(A, name):
    cfg = CASES[name]
    d = cfg["d"]()
    w = np.load(WEIGHTS).astype(np.float32) if cfg["mode"] else None
    dt, n, k = 0.0025, cfg["n"], cfg["k"]
    kw = dict(mode=cfg["mode"], diag_every=1, k_max=8 if cfg["mode"] else 0, rollback=cfg["rollback"])

    ref = _ctx(A, d, cfg["fp32"], w)
    ref.set_counters(11, 13)
    ref.compute_forces(dt, k)
    ref.step(2 * n, dt, k, **kw)
    x_ref, v_ref = ref.state()
    rows_ref, diag_ref, cnt_ref = ref.series(), ref.diag(), ref.counters()
    ref.close()

    first = _ctx(A, d, cfg["fp32"], w)
    first.set_counters(11, 13)
    first.compute_forces(dt, k)
    first.step(n, dt, k, **kw)
    blob = first.save_checkpoint()
    first.close()

    # a fresh context, set up the same way (its own generated start state is overwritten)
    second = _ctx(A, d, cfg["fp32"], None)
    second.load_checkpoint(blob)
    second.step(n, dt, k, **kw)
    x, v = second.state()
    rows, dg = second.series(), second.diag()
    print("%s: checkpoint %.1f MB, inferences %d / %d, rollbacks %d" % (name, blob.nbytes / 1e6, dg.inferences,
                                                                       diag_ref.inferences, dg.rollbacks))
    assert np.array_equal(x, x_ref) and np.array_equal(v, v_ref)
    assert rows.shape == rows_ref.shape and np.array_equal(rows, rows_ref)
    assert (dg.step, dg.time, dg.k, dg.hold, dg.inferences, dg.fallbacks, dg.rollbacks) == \
        (diag_ref.step, diag_ref.time, diag_ref.k, diag_ref.hold, diag_ref.inferences, diag_ref.fallbacks,
         diag_ref.rollbacks)
    assert second.counters() == cnt_ref
    if cfg["mode"]:
        assert dg.inferences >= 1
    second.close()


def test_checkpoint_of_another_system_is_refused(A):
    d = synth.platelet_box()
    a = _ctx(A, d, False, None)
    a.compute_forces(0.0025, 4)
    blob = a.save_checkpoint()
    a.close()
    other = A.from_workload(d, params=dict(gamma=4.0, sigma=float(np.sqrt(8.0))), skin=0.5, series_capacity=400,
                            ctrl_max_batch=8)
    with pytest.raises(A.AimtsError, match="another system"):
        other.load_checkpoint(blob)
    with pytest.raises(A.AimtsError, match="truncated|too short"):
        b = _ctx(A, d, False, None)
        b.load_checkpoint(blob[: blob.size // 2])
