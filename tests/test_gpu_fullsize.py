"""Parity at the full size of the bench workload: the 2,010,248-particle channel (2,000,000
DPD particles in 200 x 50 x 66.7 with frozen walls in y, body force 0.02 along x, four
level-4 platelets), in the three configurations bench.py times:

  * float32 pair forces, fixed ratio 4, skin 0.4 (the fixed-ratio leg);
  * float32 pair forces, ratio 8, skin 0.5 (the controller leg at its ratio cap);
  * float64 forces, ratio 1 (the STS leg).

Both force groups are compared on every particle (the oracle's outer group runs on 16
host threads, about a second at this size).  Same tolerances as the small cases:
relative RMS 1e-10 in float64, 1e-5 for float32 pair forces.  Per particle, so that no
particle's error hides in the mean, the largest force-vector difference stays within
1e-10 (float64) or 1e-4 (float32: ten times the RMS target, room for the rounding of a
single close WCA contact) of the group's RMS force; the particles next to the walls,
the periodic faces and the platelets are also checked as a group of their own.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

DT_INNER = 0.0025


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14121_amd.aimts as A
    return A


@pytest.fixture(scope="module")
def channel():
    # the bench workload, generated the same way
    return synth.channel(n_total=2_000_000, L=(200.0, 50.0, 66.7), n_platelet=4, level=4, seed=20220530, g=0.02)


@pytest.fixture(scope="module")
def oracle_system(oracle_lib, channel):
    return oracle_lib.System(channel)


def rel_rms(a, b):
    den = np.sum(b * b)
    return float(np.sqrt(np.sum((a - b) ** 2) / den)) if den > 0 else float(np.sqrt(np.sum(a * a)))


def _sample(d, n_random=3000, n_edge=500, seed=11):
    """Fluid particles: random ones, the closest to each wall, to the periodic x and z
    faces, and to the platelets' centres."""
    rng = np.random.default_rng(seed)
    nf = int(d["n_fluid"])
    x = d["x"][:nf]
    L = np.asarray(d["box_L"])
    picks = [rng.choice(nf, n_random, replace=False)]
    p = d["params"]
    picks.append(np.argsort(x[:, 1] - p["wall_lo"])[:n_edge])
    picks.append(np.argsort(p["wall_hi"] - x[:, 1])[:n_edge])
    picks.append(np.argsort(np.minimum(x[:, 0], L[0] - x[:, 0]))[:n_edge])
    picks.append(np.argsort(np.minimum(x[:, 2], L[2] - x[:, 2]))[:n_edge])
    nb = int(d["n_bead"])
    xb = d["x"][nf + int(d["n_wall"]):]
    per = xb.shape[0] // int(d["n_platelet"])
    for q in range(int(d["n_platelet"])):
        c = xb[q * per:(q + 1) * per].mean(axis=0)
        dd = x - c
        for k in (0, 2):
            dd[:, k] -= L[k] * np.round(dd[:, k] / L[k])
        picks.append(np.argsort(np.einsum("ij,ij->i", dd, dd))[:n_edge // 2])
    assert nb > 0
    return np.unique(np.concatenate(picks))


@pytest.mark.parametrize("fp32,k,skin,tol,tol_max", [(True, 4, 0.4, 1e-5, 1e-4), (True, 8, 0.5, 1e-5, 1e-4),
                                                     (False, 1, 0.4, 1e-10, 1e-10)],
                         ids=["fp32_k4", "fp32_k8", "fp64_k1"])
def test_full_size_channel_forces(A, oracle_system, channel, fp32, k, skin, tol, tol_max):
    d = channel
    counters = (1001, 2003)
    ctx = A.from_workload(d, fp32=fp32, skin=skin)
    ctx.set_counters(*counters)
    ctx.compute_forces(DT_INNER, k)
    fo, fi = ctx.forces()
    ctx.close()
    nt = 16
    ro = oracle_system.outer_forces(d["x"], d["v"], counters[0], k * DT_INNER, nthreads=nt)
    ri = oracle_system.inner_forces(d["x"], d["v"], counters[1], DT_INNER)
    eo = rel_rms(fo, ro)
    ei = rel_rms(fi, ri)
    rms_o = np.sqrt(np.mean(np.sum(ro * ro, axis=1)))
    mo = float(np.max(np.linalg.norm(fo - ro, axis=1))) / rms_o
    mbead = fi[int(d["n_fluid"] + d["n_wall"]):]
    rms_i = np.sqrt(np.mean(np.sum(ri[int(d["n_fluid"] + d["n_wall"]):] ** 2, axis=1)))
    mi = float(np.max(np.linalg.norm(fi - ri, axis=1))) / rms_i
    sub = _sample(d)
    es = rel_rms(fo[sub], ro[sub])
    print("full-size channel (fp32=%s, k=%d): F_outer rel RMS %.3e over all %d particles (largest per-particle "
          "difference %.3e of the RMS force; edge sample of %d: %.3e), F_inner rel RMS %.3e (largest %.3e)"
          % (fp32, k, eo, d["n"], mo, sub.size, es, ei, mi))
    assert eo <= tol and ei <= tol and es <= tol
    assert mo <= tol_max and mi <= tol_max and mbead.shape[0] == int(d["n_bead"])
    # frozen walls carry no force in either group
    nf, nw = int(d["n_fluid"]), int(d["n_wall"])
    assert np.all(fo[nf:nf + nw] == 0.0) and np.all(fi[nf:nf + nw] == 0.0)
