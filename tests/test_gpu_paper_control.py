"""The paper's own AI-MTS loop (Sec. 3.3; Table 1, Table 2) driven by the trained pipeline
(paper_2205_14121_amd/data/paper_pipeline.npy) on the device: each decision's predictions
against the float64 oracle's forward pass on the same windows, its categorisation, the
ratio rule (the smallest platelet's ratio, capped at 8) and, in a three-level context,
the sublevels it assigns."""
import os

import numpy as np
import pytest

import synth
from oracle import lstm as O

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2205_14121_amd", "data", "paper_pipeline.npy")


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14121_amd.aimts as A
    return A


@pytest.mark.parametrize("levels", [False, True], ids=["two-group", "three-level"])
def test_paper_control_decisions(A, levels):
    from paper_2205_14121_amd import paper_pipeline as PP
    # the pipeline's training channel at a body force it was not trained on
    d = synth.channel(n_total=200_000, L=(20.0, 50.0, 66.7), n_platelet=4, level=4, seed=7, g=0.03)
    ctx = A.from_workload(d, fp32=True, skin=PP.SKIN, three_level=levels)
    ctx.compute_forces(PP.DT, 1)
    ctx.step(100, PP.DT, 1)
    ctx.compute_forces(PP.DT, 4)
    params = np.load(WEIGHTS)
    # three-level: the interface every 2 inner steps; the flowing sublevel keeps the inner
    # step (k_sub = 2 let these level-4 meshes heat up and fail the bead skin at ratio 8)
    dec = PP.control(ctx, params, 100, PP.DT, k_start=4, k_max=8, levels=levels, k_if=2, k_sub=1)
    assert [r["step"] for r in dec] == [50, 75, 100]
    W = O.unflatten(params.astype(np.float64))
    for r in dec:
        ref = O.forward(W, r["windows"].astype(np.float64))["pred"]
        err = float(np.max(np.abs(r["pred"] - ref)))
        print("step %d: predictions %s (oracle %s, max |diff| %.1e), ratios %s, outer ratio %d, sublevels %s"
              % (r["step"], np.round(r["pred"], 4).tolist(), np.round(ref, 4).tolist(), err, r["ratio"].tolist(),
                 r["k"], None if r["levels"] is None else r["levels"].tolist()))
        assert np.allclose(r["pred"], ref, rtol=1e-4, atol=1e-5)
        assert np.array_equal(r["ratio"], O.categorize(r["pred"]))
        assert r["k"] == min(int(r["ratio"].min()), 8)
        if levels:
            assert np.array_equal(r["levels"], np.where(r["ratio"] > r["k"], 1, 2))
    if levels:
        _, _, lv = ctx.levels()
        assert np.array_equal(lv, dec[-1]["levels"])
    x, v = ctx.state()
    assert np.isfinite(x).all() and np.isfinite(v).all()
    assert ctx.diag().step == 200
    ctx.close()
