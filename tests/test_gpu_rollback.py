"""Rollback of failed segments (aimts_schedule.rollback) on the one-platelet box of 24,000
DPD particles.

An outer step whose bead displacements exceed the bead skin is caught by the skin check
of the next rebuild.  Without rollback the call ends with E_UNSTABLE; with rollback the
segment is restored from the device checkpoint and run again at half its ratio.  The
bead skin is set between the largest bead displacement sums of ratio 4 and ratio 8
(measured first, from the error report of runs with a tiny bead skin), so that ratio 8
fails and its fallback ratio 4 passes.
"""
import re

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

DT = 0.0025


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14121_amd.aimts as A
    return A


@pytest.fixture(scope="module")
def box():
    return synth.platelet_box()


def _start(A, d, k, skin_bead, **kw):
    ctx = A.from_workload(d, fp32=True, skin=0.5, skin_bead=skin_bead, **kw)
    ctx.set_counters(0, 0)
    ctx.compute_forces(DT, k)
    return ctx


def _bead_sum(A, d, k, n):
    """Largest sum of the two largest bead displacements of one outer step over n steps."""
    ctx = _start(A, d, k, 1e-3)
    with pytest.raises(A.AimtsError) as e:
        ctx.step(n, DT, k)
    m = re.search(r"bead displacement sum ([0-9.eE+-]+)", str(e.value))
    assert m, str(e.value)
    ctx.close()
    return float(m.group(1))


def test_rollback_reruns_failed_segments_at_half_ratio(A, box):
    s4, s8 = _bead_sum(A, box, 4, 64), _bead_sum(A, box, 8, 64)
    print("largest bead displacement sums: ratio 4 %.4f, ratio 8 %.4f" % (s4, s8))
    assert s8 > 1.6 * s4  # displacements in one outer step grow with its length
    sb = 1.5 * s4
    # without rollback, ratio 8 fails the bead skin
    ctx = _start(A, box, 8, sb)
    with pytest.raises(A.AimtsError, match="bead displacement sum"):
        ctx.step(32, DT, 8)
    ctx.close()
    # with rollback every failed segment is rerun at ratio 4 and the call completes
    ctx = _start(A, box, 8, sb, series_capacity=64)
    ctx.step(32, DT, 8, diag_every=1, rollback=8)
    dg = ctx.diag()
    rows = ctx.series()
    x, v = ctx.state()
    print("rollbacks %d, ratios of the 32 rows %s" % (dg.rollbacks, np.unique(rows[:, 7], return_counts=True)))
    assert dg.rollbacks >= 1 and dg.step == 32
    assert rows.shape[0] == 32
    assert set(np.unique(rows[:, 7]).tolist()) <= {4.0, 8.0}
    assert np.sum(rows[:, 7] == 4.0) == 8 * dg.rollbacks
    # the simulated time adds up over the ratios actually run
    assert abs(rows[-1, 0] - DT * rows[:, 7].sum()) < 1e-9
    assert np.isfinite(x).all() and np.isfinite(v).all()
    ctx.close()
    # the same simulated time at ratio 4 from the same start (other random numbers): the
    # box starts from uniform random positions and is still cooling from the initial
    # overlaps, so compare temperatures with that run rather than with kT
    ref = _start(A, box, 4, sb, series_capacity=64)
    ref.step(32, DT, 4, diag_every=1)
    T_ref = ref.series()[-1, 3]
    ref.close()
    print("T_pec after the rolled-back run %.4f, plain ratio-4 run %.4f" % (rows[-1, 3], T_ref))
    assert abs(rows[-1, 3] - T_ref) < 0.05 * T_ref


def test_rollback_halves_down_to_ratio_one_then_fails(A, box):
    """A segment that fails at every ratio (a bead skin far below one step's displacement)
    is rerun at 4, 2 and 1 after failing at 8, and the call then ends with E_UNSTABLE."""
    ctx = _start(A, box, 8, 1e-4)
    status = ctx.step_status(16, DT, 8, rollback=8)
    assert status == A.E_UNSTABLE
    assert "bead displacement sum" in A.lib.aimts_last_error(ctx.ctx).decode()
    assert ctx.diag().rollbacks == 3
    ctx.close()


def test_far_position_is_an_instability(A, box):
    """A particle flung far out of the box in one outer step (a velocity of 1e6) is caught
    when the next rebuild bins it: such particles are spread over the bins rather than
    piled into one clamped edge cell (where the sort, the pair kernel and the lists would
    do work growing with the square of its size).  Without rollback the call ends with
    E_UNSTABLE naming it; with rollback the segment is first rerun at ratios 2 and 1."""
    x, v = None, None
    for rollback, reruns in ((0, 0), (4, 2)):
        ctx = _start(A, box, 4, 0.5)
        if x is None:
            x, v = ctx.state()
            v[0] = [1.0e6, 0.0, 0.0]  # particle 0 is a fluid particle
        ctx.set_state(x, v)
        ctx.compute_forces(DT, 4)
        status = ctx.step_status(8, DT, 4, rollback=rollback)
        msg = A.lib.aimts_last_error(ctx.ctx).decode()
        print("rollback %d: status %d, %d reruns: %s" % (rollback, status, ctx.diag().rollbacks, msg))
        assert status == A.E_UNSTABLE
        assert "far outside the box" in msg
        assert ctx.diag().rollbacks == reruns
        ctx.close()
