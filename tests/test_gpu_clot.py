"""Parity on the largest system's code paths, through the C ABI.

  * A reduced clot channel of the largest system's recipe (4,000,000 DPD particles in
    120 x 300 x 37 with walls in y, 30 level-5 platelets pre-packed with Morse bonds and
    4 free ones; 348,228 beads): 2.66 M bins, so the exclusive scans take their
    three-launch path (more than 1,024 tiles of 2,048 entries), and 348 k beads, so the
    inner force kernel runs its largest grid of 8,192 fluid-member blocks.  Both force
    groups on every particle.
  * The largest system itself (102,560,500 particles, 66.6 M bins), where slot offsets
    come closest to the 32-bit limit: the outer force on a sample (random fluid particles
    and those next to the walls, the periodic faces and every platelet), the inner force
    on every particle.

float64 forces to a relative RMS error of 1e-10 and float32 pair forces to 1e-5,
both with the bead-bead skin of the benchmark's legs.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

DT = 0.00125  # the level-5 platelets' inner step
K = 8


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


def _edge_sample(d, n_random, n_edge, seed):
    rng = np.random.default_rng(seed)
    nf = int(d["n_fluid"])
    x = d["x"][:nf]
    L = np.asarray(d["box_L"])
    p = d["params"]
    picks = [rng.choice(nf, n_random, replace=False),
             np.argsort(x[:, 1] - p["wall_lo"])[:n_edge], np.argsort(p["wall_hi"] - x[:, 1])[:n_edge],
             np.argsort(np.minimum(x[:, 0], L[0] - x[:, 0]))[:n_edge],
             np.argsort(np.minimum(x[:, 2], L[2] - x[:, 2]))[:n_edge]]
    xb = d["x"][nf + int(d["n_wall"]):]
    P = int(d["n_platelet"])
    per = xb.shape[0] // P
    cents = np.array([xb[q * per:(q + 1) * per].mean(axis=0) for q in range(P)])
    # for every platelet, the 40 fluid particles nearest its centre, searched in the slab
    # of x within 4 of the centre (fluid sorted by x once; the slab wraps periodically)
    near = np.zeros(nf, bool)
    order = np.argsort(x[:, 0], kind="stable")
    xs = x[order, 0]
    for c in cents:
        parts = []
        for lo, hi in ((c[0] - 4.0, c[0] + 4.0), (c[0] - 4.0 + L[0], c[0] + 4.0 + L[0]),
                       (c[0] - 4.0 - L[0], c[0] + 4.0 - L[0])):
            a, b = np.searchsorted(xs, [max(lo, 0.0), min(hi, L[0])])
            if b > a:
                parts.append(order[a:b])
        cand = np.concatenate(parts)
        dd = x[cand] - c
        for k in (0, 2):
            dd[:, k] -= L[k] * np.round(dd[:, k] / L[k])
        r2 = np.einsum("ij,ij->i", dd, dd)
        near[cand[np.argpartition(r2, 40)[:40]]] = True
    picks.append(np.nonzero(near)[0])
    return np.unique(np.concatenate(picks))


def _check(A, d, fp32, skin_bead, ro, ri, sub, label):
    counters = (4001, 9003)
    ctx = A.from_workload(d, fp32=fp32, skin=0.5, skin_bead=skin_bead)
    ctx.set_counters(*counters)
    ctx.compute_forces(DT, K)
    fo, fi = ctx.forces()
    ctx.close()
    if sub is None:
        eo = rel_rms(fo, ro)
    else:
        eo = rel_rms(fo[sub], ro[sub])
    ei = rel_rms(fi, ri)
    print("%s (fp32=%s): F_outer rel RMS %.3e over %s particles, F_inner rel RMS %.3e over all"
          % (label, fp32, eo, "all" if sub is None else "%d sampled" % sub.size, ei), flush=True)
    tol = 1e-5 if fp32 else 1e-10
    assert eo <= tol and ei <= tol
    nf, nw = int(d["n_fluid"]), int(d["n_wall"])
    assert np.all(fo[nf:nf + nw] == 0.0) and np.all(fi[nf:nf + nw] == 0.0)


@pytest.fixture(scope="module")
def reduced(oracle_lib):
    d = synth.clot_channel(n_total=4_000_000, L=(120.0, 300.0, 37.0), n_free=4, n_packed=30, packed_grid=(3, 2, 5))
    S = oracle_lib.System(d)
    ro = S.outer_forces(d["x"], d["v"], 4001, K * DT, nthreads=16)
    ri = S.inner_forces(d["x"], d["v"], 9003, DT)
    return d, ro, ri


@pytest.mark.timeout(600)
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_reduced_clot_forces_all_particles(A, reduced, fp32):
    d, ro, ri = reduced
    ncell = int(np.prod(np.floor(d["box_L"])))
    assert 2 * ncell > 1024 * 2048  # three-launch scans
    assert int(d["n_bead"]) // 20 >= 8192  # largest fluid-member grid of the inner kernel
    _check(A, d, fp32, 0.2, ro, ri, None, "reduced clot, %d particles" % d["n"])


@pytest.fixture(scope="module")
def full(oracle_lib):
    print("generating the 102,560,500-particle clot ...", flush=True)
    d = synth.clot_channel()
    sub = _edge_sample(d, 20000, 2000, 5)
    S = oracle_lib.System(d)
    print("oracle forces of the clot ...", flush=True)
    ro = S.outer_forces(d["x"], d["v"], 4001, K * DT, subset=sub, nthreads=16)
    ri = S.inner_forces(d["x"], d["v"], 9003, DT)
    return d, sub, ro, ri


@pytest.mark.timeout(900)
@pytest.mark.parametrize("fp32,skin_bead", [(False, 0.2), (True, 0.3)], ids=["fp64", "fp32"])
def test_full_clot_forces(A, full, fp32, skin_bead):
    d, sub, ro, ri = full
    assert int(d["n"]) == 102_560_500
    _check(A, d, fp32, skin_bead, ro, ri, sub, "clot, %d particles" % d["n"])
