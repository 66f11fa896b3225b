"""Inter-platelet aggregation of Eq. 4 (non-bonded Morse + receptor term) on the HIP path,
through the C ABI, against the oracle: both force groups (float64 and float32 pair
forces), a trajectory of 100 inner steps, the energies and virial, and the three-level
groups.  Two level-3 platelets stacked 0.8 apart with no fixed Morse bonds: they are
held together by the aggregation term alone."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

AGG = dict(agg_rc=1.5)  # D = 5, a = 2, r0 = 1, f^A = 10 from the shared parameters


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


def _stack(jitter=0.02, **over):
    d = synth.aggregate_box(n_fluid=4000, L=(12.0, 12.0, 12.0), morse_cut=0.0, **dict(AGG, **over))
    assert d["morse"].shape[0] == 0
    if jitter:
        b0 = int(d["n_fluid"] + d["n_wall"])
        d["x"] = d["x"].copy()
        d["x"][b0:] += np.random.default_rng(8).normal(0.0, jitter, size=d["x"][b0:].shape)
    return d


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_aggregation_forces_match_oracle(A, oracle_lib, fp32):
    d = _stack()
    k, dt, counters = 4, 0.0025, (5, 9)
    ctx = A.from_workload(d, fp32=fp32, skin=0.4, skin_bead=0.3)
    ctx.set_counters(*counters)
    ctx.compute_forces(dt, k)
    fo, fi = ctx.forces()
    S = oracle_lib.System(d)
    ro = S.outer_forces(d["x"], d["v"], counters[0], k * dt)
    ri = S.inner_forces(d["x"], d["v"], counters[1], dt)
    # the term is not vacuous: without it the beads' inner forces differ by far more
    r_off = oracle_lib.System(d, params=dict(agg_rc=0.0)).inner_forces(d["x"], d["v"], counters[1], dt)
    b0 = int(d["n_fluid"])
    assert rel_rms(r_off[b0:], ri[b0:]) > 1e-2
    eo, ei = rel_rms(fo, ro), rel_rms(fi, ri)
    print("aggregation (fp32=%s): F_outer rel RMS %.3e, F_inner rel RMS %.3e (without the term: %.3e)"
          % (fp32, eo, ei, rel_rms(r_off[b0:], ri[b0:])))
    tol = 1e-5 if fp32 else 1e-10
    assert eo <= tol and ei <= tol


def test_aggregation_trajectory(A, oracle_lib):
    """100 inner steps (25 outer steps at k = 4) in float64 from identical state and counters."""
    d = _stack(jitter=0.0)
    k, dt, n = 4, 0.0025, 25
    ctx = A.from_workload(d, skin=0.4, skin_bead=0.3)
    ctx.set_counters(0, 0)
    ctx.compute_forces(dt, k)
    ctx.step(n, dt, k)
    xg, _ = ctx.state()
    S = oracle_lib.System(d)
    x, v = d["x"].copy(), d["v"].copy()
    fo = S.outer_forces(x, v, 0, k * dt)
    fi = S.inner_forces(x, v, 0, dt)
    S.respa(x, v, fo, fi, [1, 1], n, k * dt, k)
    err = max_image_dx(xg, x, d)
    print("aggregation, 25 outer steps at k = 4: max |dx| %.3e" % err)
    assert err <= 1e-8


def test_aggregation_energy_and_virial(A, oracle_lib):
    d = _stack()
    ctx = A.from_workload(d, skin=0.4, skin_bead=0.3)
    ctx.compute_forces(0.0025, 4)
    g = ctx.diag(energy=True)
    got = np.array(list(g.pe[:]) + [g.virial])
    e = oracle_lib.System(d).energy(d["x"])
    print("energies gpu", got, "oracle", e)
    assert e[4] != 0.0
    assert np.allclose(got, e, rtol=1e-10, atol=1e-8)


@pytest.mark.parametrize("level", [[1, 2], [2, 1], [1, 1]])
def test_aggregation_three_level_groups(A, oracle_lib, level):
    d = _stack()
    dt, k, k_if = 0.0025, 8, 4
    ctx = A.from_workload(d, skin=0.5, skin_bead=0.3, three_level=True)
    ctx.set_levels(k_if, 2, level)
    ctx.set_counters(7, 11)
    ctx.compute_forces(dt, k)
    gm, g1, g2 = ctx.level_forces()
    rm, r1, r2 = oracle_lib.System(d).inner_forces3(d["x"], d["v"], 11, k_if * dt, level)
    errs = [rel_rms(g, r) for g, r in ((gm, rm), (g1, r1), (g2, r2))]
    print("levels %s: group rel RMS M %.2e P1 %.2e P2 %.2e" % (level, *errs))
    assert max(errs) <= 1e-10
