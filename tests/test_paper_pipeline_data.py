"""The stored weights of the paper's own inference pipeline (Sec. 3.3, Table 2), as
trained by paper_2205_14121_amd/paper_pipeline.py, evaluated with the float64 oracle:
the vector has the pipeline's layout, its normalisation is usable, and the forward pass
gives finite log2 ratios that categorise into the paper's levels.  The stored report
must show the learned predictor beating the best constant on its test windows."""
import json
import os

import numpy as np

from oracle import lstm as O

DATA = os.path.join(os.path.dirname(__file__), "..", "paper_2205_14121_amd", "data")


def test_stored_weights_evaluate():
    p = np.load(os.path.join(DATA, "paper_pipeline.npy"))
    assert p.dtype == np.float32 and p.shape == (O.n_params(),)
    assert np.all(np.isfinite(p))
    W = O.unflatten(p.astype(np.float64))
    assert np.all(W["norm_std"] > 0.0)
    rng = np.random.default_rng(0)
    X = W["norm_mean"] + W["norm_std"] * rng.standard_normal((8, O.T, O.F))
    out = O.forward(W, X)
    assert np.all(np.isfinite(out["pred"])) and out["latent"].shape == (8, O.LAT)
    assert set(O.categorize(out["pred"]).tolist()) <= set(O.RATIOS)


def test_stored_report_beats_constant():
    with open(os.path.join(DATA, "paper_pipeline_report.json")) as fh:
        r = json.load(fh)
    assert r["rmse_log2_test"] < r["rmse_log2_test_constant_mean_predictor"]
    assert r["correlation_prediction_target_test"] > 0.0
    assert r["ae_loss_first_last"][1] < r["ae_loss_first_last"][0]
