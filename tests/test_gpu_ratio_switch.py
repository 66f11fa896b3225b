"""A change of the MTS ratio between outer steps (Sec. 3.3: the controller resets the
step on the fly) re-evaluates the outer force so that the random impulse of the instant
between the two steps has the variance of the half steps it spans.  Scaled for the old
step throughout, that variance is off by (Dn + Dt)^2 / (4 Dn) / ((Dn + Dt) / 2): 1.5
going 4 -> 8, 0.75 going 8 -> 4, +12 % on average under a 4 <-> 8 alternation, which
heats the fluid; rescaled to the new step for the opening half only, it is 2.9 % short
either way (a run alternating at every step measured 1.9 % cold).  With the exact
scaling, a run switching the ratio at every step keeps the temperature of runs at fixed
ratios."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14121_amd.aimts as A
    return A


def test_alternating_ratio_keeps_the_temperature(A):
    """From one equilibrated state, the same simulated time at fixed ratio 4, at fixed
    ratio 8 and alternating 4, 8 every outer step (a third of the time at 4): the
    alternating run's time-averaged temperature is the time-weighted mean of the fixed
    runs' within 1 %."""
    from paper_2205_14121_amd.controller import time_average
    d = synth.dpd_box(n=24000, L=(20.0, 20.0, 20.0), seed=31)
    dt = 0.0025
    eq = A.from_workload(d, fp32=True)
    eq.compute_forces(dt, 4)
    eq.step(600, dt, 4)  # 6 time units: the initial overlaps have relaxed
    x, v = eq.state()
    cnt = eq.counters()
    eq.close()
    span = 2.4

    def run(pattern):
        n = int(round(span / (dt * sum(pattern)) * len(pattern)))
        ctx = A.from_workload(d, fp32=True, series_capacity=n + 8)
        ctx.set_state(x, v)
        ctx.set_counters(*cnt)
        ctx.compute_forces(dt, pattern[0])
        for q in range(n):
            ctx.step(1, dt, pattern[q % len(pattern)], diag_every=1)
        rows = ctx.series()
        ctx.close()
        return time_average(rows, 2)  # total T of this periodic fluid (no flow)

    T4, T8, Tal = run([4]), run([8]), run([4, 8])
    expect = (T4 + 2.0 * T8) / 3.0
    print("T: fixed 4 %.4f, fixed 8 %.4f, alternating %.4f (time-weighted mean of the fixed runs %.4f)"
          % (T4, T8, Tal, expect))
    assert abs(Tal - expect) < 0.01 * expect
