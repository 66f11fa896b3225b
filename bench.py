"""Benchmark of the DPD + CGMD multiple-time-stepping hot path on one MI355X.

Default workload (synthetic, seeded; `synth.clot_channel`): the largest single-GPU
system, a channel of 100,000,000 DPD particles (fluid + frozen wall layers in y) in
3000 x 300 x 37, periodic in x and z, body force 0.02 along x, with 250 level-5
platelets of 10,242 CG beads: 70 free at random positions and orientations and 180
pre-packed on the lower wall, bound by inter-platelet Morse bonds (D = 5, a = 2,
r0 = 1): 102,560,500 particles.  It stands in for the paper's 102-million-particle
clot, whose platelet model is not available.  `--workload channel` runs the
2,010,248-particle Poiseuille channel with 4 level-4 platelets instead.

A "step" is one outer step of the whole hot path: cell-list rebuild (counting sort),
DPD outer forces, k inner steps of the platelet group (bonds, angles, WCA, Morse,
platelet-fluid forces), RESPA kicks and drifts, diagnostics and platelet features,
and the controller's inference whenever its hold runs out.

Legs, all from the same equilibrated state:
  * MTS (the headline `value`): float32 pair forces, float64 state, the learned
    controller choosing the ratio (ratio capped at 8) or, with --fixed, ratio --k.  The
    controller leg runs at least 63 untimed steps first, so that its first decision
    (after 64 feature rows) falls on the first timed step.
  * STS: float64 forces, ratio 1, over the same simulated-time window (same start
    time after the equilibrated state, same span).
The temperature error compares the two legs' peculiar temperatures averaged over the
same simulated time: --t-span outer steps of the MTS leg (its first --steps are the
timed ones) against the STS steps that cover that time.
Reported: particle-(outer)steps/s, simulated time per day, the simulated-time speedup
MTS/STS, the temperature error, the roofline of the DPD outer-force kernel (timed live
with HIP events on the library's stream during the timed steps), the HBM-bound phases
against their algorithmic bytes, and the oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s and simulated-time/day: FP64 STS vs FP32 AI-MTS at equal T error"
DT_INNER = 0.0025
SECONDS_PER_DAY = 86400.0
# VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-slots per second)
VALU_PEAK = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12  # bytes per second
# Algorithmic VALU lane-slots per fluid particle per DPD evaluation (half-shell cell list:
# ~40 distance tests and 6.3 unique pairs per particle at density 3): float32 / float64 pair math
SLOTS_PER_PARTICLE = {True: 1.9e3, False: 2.6e3}
# Algorithmic HBM bytes (each datum read or written once):
#   DPD, per particle: x 24 + v 24 + id 4 read, float32 force 12 written
DPD_BYTES_PER_PARTICLE = 64
#   cell sort, per particle: x read 24, cell id written and read 8, then x, v, id read
#   and written in cell order 52 + 52
SORT_BYTES_PER_PARTICLE = 136
#   outer kicks and the lazy drift, per mobile particle and outer step: one kick (v read
#   and written, float32 force read: 60) and one drift (x read and written: 48)
KICK_BYTES_PER_PARTICLE = 108
# This design's own byte counts (what its kernels read and write):
#   counting sort, per particle: binning 40 (x 24, id 4, bin 4, rank 4), scatter 24 (bin,
#   rank, bin start, id; id and source written), rank and gather 160 (source, id, bin,
#   bin range 16; x, v 48 read; x, v 48, id, source, float copies 32, member index
#   written); per cell (two bins): histogram counts and clears 16, scan 16
DESIGN_SORT_BYTES_PER_PARTICLE, DESIGN_SORT_BYTES_PER_CELL = 224, 32
#   outer kicks and lazy drift, per mobile particle: half kick + k drifts (id 4, v 24 + 24,
#   force 12, member index 4, x 24 + 24) and closing half kick (id 4, v 24 + 24, force 12);
#   a frozen wall particle has its id read twice and its x and v copied into the members'
#   second state buffer (48 + 48)
DESIGN_KICK_BYTES_MOBILE, DESIGN_KICK_BYTES_WALL = 180, 104
TRAFFIC_FILES = {"channel": os.path.join(ROOT, "profiles", "k_dpd_f32_channel2M_traffic.json"),
                 "clot": os.path.join(ROOT, "profiles", "k_dpd_f32_clot100M_traffic.json")}
DPD_SOURCES = ("paper_2205_14121_amd/csrc/dpd.hip", "paper_2205_14121_amd/csrc/common.h")
CONTROLLER_WEIGHTS = os.path.join(ROOT, "paper_2205_14121_amd", "data", "controller.npy")


def dpd_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in DPD_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind):
    """HBM bytes per DPD launch of workload `kind` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy kernel), or None if there is none
    or the kernel source changed since."""
    try:
        with open(TRAFFIC_FILES[kind]) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != dpd_source_hash():
        return None
    return t.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("clot", "channel"), default="clot",
                    help="clot (default): the largest single-GPU system, 100,000,000 DPD particles in "
                         "3000x300x37 with 250 level-5 platelets, 180 of them pre-packed with Morse bonds; "
                         "channel: the 2,000,000-particle Poiseuille channel with 4 level-4 platelets")
    ap.add_argument("--steps", type=int, default=100, help="timed outer steps of the MTS leg")
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed outer steps of the MTS leg before the timed ones (the controller leg "
                         "runs at least 63, so that its first decision falls on the first timed step)")
    ap.add_argument("--t-span", type=int, default=100,
                    help="outer steps of the MTS leg over which the temperature error is averaged "
                         "(the timed steps are its first ones; at least --steps)")
    ap.add_argument("--k", type=int, default=4, help="MTS ratio of a fixed-ratio MTS leg (--fixed)")
    ap.add_argument("--equil", type=int, default=800,
                    help="untimed float32 outer steps from the generated start before both legs "
                         "(ratio 4 for the clot, ratio 1 for the channel)")
    ap.add_argument("--controller", default=CONTROLLER_WEIGHTS if os.path.exists(CONTROLLER_WEIGHTS) else "",
                    help="trained controller weights (.npy) for the AI-MTS leg (default: the package's "
                         "trained weights when present)")
    ap.add_argument("--fixed", action="store_true", help="fixed ratio --k instead of the controller")
    ap.add_argument("--k-if", type=int, default=1,
                    help="MTS leg: three-level scheme with the platelet-fluid interface every K_IF inner steps "
                         "(1 with --k-sub 1: two-group RESPA)")
    ap.add_argument("--skin", type=float, default=None,
                    help="MTS leg: platelet-fluid list skin (default 0.35 for the clot's controller leg, "
                         "0.5 for the channel's, 0.4 at a fixed ratio)")
    ap.add_argument("--skin-bead", type=float, default=None,
                    help="MTS leg: bead-bead list skin (default 0.3 for the clot's controller leg, else 0.2)")
    ap.add_argument("--k-sub", type=int, default=1,
                    help="MTS leg: the flowing platelets' sublevel every K_SUB inner steps (the controller sets "
                         "each platelet's sublevel at its decisions)")
    ap.add_argument("--n-total", type=int, default=2_000_000, help="channel workload: DPD particles")
    ap.add_argument("--skip-sts", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-outer-steps", type=int, default=10,
                    help="channel workload: oracle outer steps timed on the host")
    ap.add_argument("--cpu-subset", type=int, default=1_000_000,
                    help="clot workload: fluid particles of the oracle's timed outer-force sample")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no benchmark: write the DPD traffic summary of --workload from two rocprofv3 --pmc "
                         "counter collections (FETCH_SIZE, WRITE_SIZE) of a run with --copy-calibration-mib")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this many MiB first (reference for HBM counters)")
    return ap.parse_args()


def workload(n_total):
    import synth
    scale = n_total / 2_000_000
    L = (200.0 * scale, 50.0, 66.7) if n_total != 2_000_000 else (200.0, 50.0, 66.7)
    return synth.channel(n_total=n_total, L=L, n_platelet=4, level=4, seed=20220530, g=0.02)


def workload_name(d, kind, schedule):
    if kind == "clot":
        n_free = int(d["n_platelet"]) - 180
        return ("Clot channel, %d DPD particles (fluid + frozen walls) in %.0fx%.0fx%.0f, g=0.02, %d platelets x "
                "10,242 beads (%d free, 180 pre-packed on the lower wall with %d Morse bonds); float32 pair forces, "
                "float64 state; RESPA %s" % (int(d["n_fluid"] + d["n_wall"]), *d["box_L"], int(d["n_platelet"]),
                                             n_free, int(d["morse"].shape[0]), schedule))
    return ("Poiseuille channel, %d DPD particles (fluid + frozen walls) in %.1fx%.1fx%.1f, g=0.02, 4 platelets x "
            "2,562 beads; float32 pair forces, float64 state; RESPA %s"
            % (int(d["n_fluid"] + d["n_wall"]), *d["box_L"], schedule))


def oracle_threads():
    # the host share of one GPU is 16 cores; OMP_NUM_THREADS, when set, says what is available
    return min(16, int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1)


def cpu_baseline_channel(sysd, k, outer_steps):
    """The oracle as it stands (float64, OpenMP over the host cores for the outer group)
    on a bounded sample: `outer_steps` RESPA outer steps of the same workload."""
    import oracle
    S = oracle.System(sysd)
    nthreads = oracle_threads()
    x, v = sysd["x"].copy(), sysd["v"].copy()
    t0 = time.perf_counter()
    fo = S.outer_forces(x, v, 0, k * DT_INNER, nthreads=nthreads)
    fi = S.inner_forces(x, v, 0, DT_INNER)
    t1 = time.perf_counter()
    S.respa(x, v, fo, fi, [1, 1], outer_steps, k * DT_INNER, k, nthreads=nthreads)
    t2 = time.perf_counter()
    n = sysd["n"]
    rate = n * outer_steps / (t2 - t1)
    return {"value": rate, "unit": "particle-steps/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d RESPA outer step(s) at k=%d (float64) of the %d-particle channel, after one "
                      "force evaluation (%.1f s); %.1f s timed" % (outer_steps, k, n, t1 - t0, t2 - t1),
            "tau_per_day": outer_steps * k * DT_INNER / (t2 - t1) * SECONDS_PER_DAY}


class ClotInnerTiming:
    """The oracle's inner-group force evaluation of the whole clot (every bead, its bonds,
    angles, Morse bonds and bead/fluid pairs; single-threaded, as the oracle stands) on a
    host thread of its own, started before the GPU legs and joined before any timed
    region (the C call releases the interpreter lock)."""

    def __init__(self, sysd, dt):
        import threading
        self.seconds = None
        self.error = None

        def run():
            try:
                import oracle
                S = oracle.System(sysd)
                t0 = time.perf_counter()
                S.inner_forces(sysd["x"], sysd["v"], 0, dt)
                self.seconds = time.perf_counter() - t0
            except Exception as e:  # reported with the baseline, never fatal to the GPU legs
                self.error = repr(e)

        self.thread = threading.Thread(target=run, daemon=True)
        self.thread.start()

    def join(self):
        self.thread.join()


def cpu_baseline_clot(sysd, inner, n_sub, k_mean, dt_in):
    """The oracle on a bounded sample of the clot: its outer-group forces (cell list over
    all fluid and wall particles, then the DPD sum) for 1 and for `n_sub` fluid particles
    on the host cores, extrapolated linearly to all fluid particles, plus one inner-group
    evaluation of the whole system (timed by `inner`).  One outer step at the MTS leg's
    mean ratio k costs t_outer + k t_inner; the oracle's kicks and drifts are left out,
    so the rate is an upper bound on the oracle's."""
    import oracle
    S = oracle.System(sysd)
    nthreads = oracle_threads()
    nf = int(sysd["n_fluid"])
    rng = np.random.default_rng(7)
    x, v = sysd["x"], sysd["v"]
    times = []
    for m in (1, n_sub):
        sub = np.sort(rng.choice(nf, m, replace=False)).astype(np.int64)
        t0 = time.perf_counter()
        S.outer_forces(x, v, 0, k_mean * dt_in, subset=sub, nthreads=nthreads)
        times.append(time.perf_counter() - t0)
    t_outer = times[0] + (times[1] - times[0]) * (nf - 1) / (n_sub - 1)
    inner.join()
    if inner.seconds is None:
        return {"value": None, "unit": "particle-steps/s", "cores": nthreads, "kind": "oracle",
                "sample": "inner-group evaluation failed: %s" % inner.error}
    t_step = t_outer + k_mean * inner.seconds
    n = int(sysd["n"])
    return {"value": n / t_step, "unit": "particle-steps/s", "cores": nthreads, "kind": "oracle",
            "sample": "outer-group forces of 1 and of %d sampled fluid particles (%.1f s and %.1f s, cell list "
                      "over all %d fluid and wall particles included; %d threads), extrapolated linearly to all "
                      "%d fluid particles: %.1f s; one inner-group evaluation of every bead (1 thread): %.1f s; "
                      "per outer step at the MTS leg's mean ratio %.2f: t_outer + k t_inner = %.1f s (kicks and "
                      "drifts not counted)" % (n_sub, times[0], times[1], int(sysd["n_fluid"] + sysd["n_wall"]),
                                               nthreads, nf, t_outer, inner.seconds, k_mean, t_step),
            "tau_per_day": k_mean * dt_in / t_step * SECONDS_PER_DAY,
            "extrapolated": True}


def write_traffic(kind, fetch_csv, write_csv, copy_mib):
    """HBM traffic of one DPD launch from counter collections: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) of the DPD kernel, each scaled by the ratio of the known bytes of
    the plain copy of `copy_mib` MiB to what the same counter reads for it."""
    import csv

    def per_kernel(path, counter):
        dpd, copies = [], []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                val = float(r["Counter_Value"])
                if "k_dpd" in r["Kernel_Name"]:
                    dpd.append(val)
                elif "elementwise" in r["Kernel_Name"].lower():
                    copies.append(val)
        return dpd, copies

    known_kib = copy_mib * 1024.0
    run = ("python3 bench.py --workload %s --fixed --steps 5 --warmup 1 --equil %d --skip-sts --skip-cpu "
           "--copy-calibration-mib %d" % (kind, 4 if kind == "clot" else 200, copy_mib))
    names = {"channel": "channel, 2,010,248 particles", "clot": "clot channel, 102,560,500 particles"}
    out = {"kernel": "k_dpd<float>", "workload": names[kind], "copy_calibration_mib": copy_mib,
           "source_hash": dpd_source_hash(),
           "commands": ["rocprofv3 --pmc %s --kernel-include-regex 'k_dpd|elementwise' --output-format csv "
                        "-d pmc_out/pmc_%s -o run -- %s" % (c, c.split("_")[0].lower(), run)
                        for c in ("FETCH_SIZE", "WRITE_SIZE")]
           + ["python3 bench.py --workload %s --write-traffic pmc_out/pmc_fetch/run_counter_collection.csv "
              "pmc_out/pmc_write/run_counter_collection.csv --copy-calibration-mib %d" % (kind, copy_mib)]}
    total = 0.0
    for name, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        dpd, copies = per_kernel(path, counter)
        # the calibration kernel is the largest elementwise dispatch of the run
        ref = max(copies)
        factor = known_kib / ref
        kib = sum(dpd) / len(dpd)
        out[name] = {"counter": counter, "kib_per_launch_raw": kib, "copy_kib_raw": ref,
                     "scale": factor, "bytes_per_launch": kib * factor * 1024.0, "launches": len(dpd)}
        total += kib * factor * 1024.0
    out["bytes_per_launch"] = total
    with open(TRAFFIC_FILES[kind], "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args.workload, args.write_traffic[0], args.write_traffic[1], args.copy_calibration_mib)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path (the sharding design is "
              "described in DESIGN.md); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2205_14121_amd.aimts as A
    from paper_2205_14121_amd.controller import time_average

    def note(msg):
        print(msg, file=sys.stderr, flush=True)

    clot = args.workload == "clot"
    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        # an elementwise kernel that reads and writes exactly copy_calibration_mib MiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    t_gen = time.perf_counter()
    if clot:
        import synth
        note("generating the 100,000,000-particle clot channel ...")
        d = synth.clot_channel()
    else:
        d = workload(args.n_total)
    t_gen = time.perf_counter() - t_gen
    note("workload ready (%.1f s)" % t_gen)
    N = int(d["n"])
    # the level-5 platelets of the clot have modes twice as fast as level-4 ones: half the step
    dt_in = 0.5 * DT_INNER if clot else DT_INNER
    use_ctrl = bool(args.controller) and not args.fixed
    k = args.k
    warm = max(args.warmup, 63) if use_ctrl else args.warmup
    span = max(args.steps, args.t_span)
    n_phase = min(args.steps, 20)
    # the oracle's inner-group evaluation of the clot runs on a host thread during the
    # untimed equilibration (joined before the timed steps)
    inner_cpu = None
    if clot and not args.skip_cpu:
        inner_cpu = ClotInnerTiming(d, dt_in)

    # --- equilibration from the uniform random start (untimed) ---
    # the clot's packed layers face each other across 1.0 with beads 0.1 apart: a short
    # bead-bead skin keeps their pair lists at the beads that can interact
    skin_bead = 0.2 if clot else 0.0
    # the platelet-fluid list skin bounds a bead's plus a fluid particle's displacement in
    # one outer step; the clot's outer step is half the channel's at equal ratio (its
    # inner step is), so its legs list fluid partners to a shorter skin
    skin_eq = 0.3 if clot else 0.4
    skin_sts = 0.25 if clot else 0.4
    eq = A.from_workload(d, fp32=True, skin=skin_eq, skin_bead=skin_bead)
    k_eq = 4 if clot else 1
    eq.compute_forces(dt_in, k_eq)
    # the clot's level-5 meshes hit the rare angle-collapse spikes even at ratio 4: every
    # leg of that workload runs in checkpointed segments (a failed segment is rerun at
    # half its ratio, or at ratio 1 with fresh random numbers)
    seg_clot = 8 if clot else 0
    eq.step(args.equil, dt_in, k_eq, rollback=seg_clot)
    x_eq, v_eq = eq.state()
    cnt_eq = eq.counters()
    eq.close()
    del eq
    note("equilibrated (%d outer steps)" % args.equil)

    # --- MTS leg (headline) ---
    # the controller's ratio is capped at 8, and the platelet-fluid list skin (0.5 on the
    # channel, 0.35 on the clot) is such that one outer step at that ratio stays within it
    # even when a bead is briefly kicked to several times its thermal speed (skins change
    # list sizes, not results)
    k_max = 8 if use_ctrl else 0
    # The controller leg runs in checkpointed segments of outer steps (32; 8 for the
    # clot): a segment whose stability checks fail (a bead of a nearly collapsed surface
    # triangle can be thrown to ten times its thermal speed for a few inner steps) is
    # restored and run again at the fallback ratio 4 inside the timed region.
    rollback = (8 if clot else 32) if use_ctrl else seg_clot
    # the clot's controller leg lists bead pairs to 0.3 beyond the cutoff: at ratio 8 the
    # angle-collapse spikes exceed 0.2 several times per 100 steps (each a rolled-back
    # segment), while 0.4 lists so many facing-layer beads that every step slows more
    skin_bead_mts = 0.3 if clot else skin_bead
    if args.skin_bead is not None:
        skin_bead_mts = args.skin_bead
    three = args.k_if > 1 or args.k_sub > 1
    skin_mts = (0.35 if clot else 0.5) if use_ctrl else (0.3 if clot else 0.4)
    if args.skin is not None:
        skin_mts = args.skin
    mts = A.from_workload(d, fp32=True, skin=skin_mts, series_capacity=warm + span + n_phase + 8,
                          ctrl_max_batch=max(8, int(d["n_platelet"])), skin_bead=skin_bead_mts, three_level=three)
    if three:
        mts.set_levels(args.k_if, args.k_sub)  # every platelet at the finest sublevel until a decision
    mode = 0
    if use_ctrl:
        mts.ctrl_set_weights(np.load(args.controller).astype(np.float32))
        mode = 1
    mts.set_state(x_eq, v_eq)
    mts.set_counters(*cnt_eq)
    mts.compute_forces(dt_in, k)
    mts.step(warm, dt_in, k, mode=mode, diag_every=1, k_max=k_max, rollback=rollback)
    if inner_cpu is not None:
        inner_cpu.join()
    d0 = mts.diag()
    mts.profile(1)  # HIP events around the DPD kernel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mts.step(args.steps, dt_in, k, mode=mode, diag_every=1, k_max=k_max, rollback=rollback)
    torch.cuda.synchronize()
    t_mts = time.perf_counter() - t0
    d1 = mts.diag()
    note("MTS leg timed (%d steps, %.2f s)" % (args.steps, t_mts))
    prof_ms, prof_n = mts.get_profile()
    mts.profile(0)
    # the rest of the temperature span, untimed
    t0 = time.perf_counter()
    if span > args.steps:
        mts.step(span - args.steps, dt_in, k, mode=mode, diag_every=1, k_max=k_max, rollback=rollback)
    torch.cuda.synchronize()
    t_rest = time.perf_counter() - t0
    d2 = mts.diag()
    rows = mts.series()
    # the cell sort, the outer kicks, the inner loop and the platelet lists are timed in a
    # short untimed segment afterwards (events break the back-to-back kernel stream, so
    # the timed steps carry only the DPD pair of events)
    mts.profile(2 | 4 | 8 | 32)
    mts.step(n_phase, dt_in, k, mode=mode, diag_every=0, k_max=k_max, rollback=rollback)
    torch.cuda.synchronize()
    phase_ms, phase_n = mts.get_profile()
    t_start = float(rows[warm - 1, 0]) if warm > 0 else 0.0
    timed = rows[warm:warm + args.steps]
    spanr = rows[warm:warm + span]
    sim_mts = float(timed[-1, 0]) - t_start
    sim_span = float(spanr[-1, 0]) - t_start
    Tpec_mts = time_average(spanr, 3)  # over simulated time (rows of a varying k)
    mean_k = time_average(timed, 7)
    mean_k_span = time_average(spanr, 7)
    value = N * args.steps / t_mts
    inferences_timed = int(d1.inferences - d0.inferences)
    mts.close()

    # --- STS leg: float64, ratio 1, the same simulated-time window from the same state ---
    sts = None
    if not args.skip_sts:
        n_pre = int(round(t_start / dt_in))
        n_sts = int(round(sim_span / dt_in))
        ctx = A.from_workload(d, fp32=False, skin=skin_sts, series_capacity=n_sts + 8, skin_bead=skin_bead)
        ctx.set_state(x_eq, v_eq)
        ctx.set_counters(*cnt_eq)
        ctx.compute_forces(dt_in, 1)
        if n_pre:
            ctx.step(n_pre, dt_in, 1, rollback=seg_clot)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(n_sts, dt_in, 1, diag_every=1, rollback=seg_clot)
        torch.cuda.synchronize()
        t_sts = time.perf_counter() - t0
        note("STS leg timed (%d steps after %d untimed, %.1f s)" % (n_sts, n_pre, t_sts))
        srows = ctx.series()
        Tpec_sts = float(np.mean(srows[:, 3]))
        sts = {"particle_steps_per_s": N * n_sts / t_sts, "steps": n_sts, "untimed_steps_before": n_pre,
               "ms_per_step": 1e3 * t_sts / n_sts, "tau_per_day": n_sts * dt_in / t_sts * SECONDS_PER_DAY,
               "T_pec": Tpec_sts, "rollbacks": int(ctx.diag().rollbacks), "skin": skin_sts, "skin_bead": skin_bead}
        ctx.close()

    # --- roofline of the dominant kernel (DPD outer forces, float32) ---
    dpd_ms = prof_ms[0] / max(prof_n[0], 1)
    n_fluid = int(d["n_fluid"])
    slots = n_fluid * SLOTS_PER_PARTICLE[True]
    achieved = slots / (dpd_ms * 1e-3) / 1e12
    dpd_bytes = n_fluid * DPD_BYTES_PER_PARTICLE
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK / 1e12, 3),
                "unit": "T lane-slots/s", "frac": round(achieved * 1e12 / VALU_PEAK, 4),
                "traffic": measured_traffic(args.workload),
                "kernel": "k_dpd<float>", "avg_ms": round(dpd_ms, 4),
                "launches": int(prof_n[0]), "algorithmic_slots_per_launch": slots,
                "algorithmic_bytes_per_launch": dpd_bytes,
                "hbm_gbs": round(dpd_bytes / (dpd_ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(dpd_bytes / (dpd_ms * 1e-3) / HBM_PEAK, 4)}
    # the HBM-bound phases of the step against their algorithmic bytes (this design's own
    # byte counts beside them), and the latency/throughput-bound platelet phases
    n_wall = int(d["n_wall"])
    ncell = int(np.prod(np.floor(np.asarray(d["box_L"]) / 1.0)))
    hbm = {}
    for name, q, alg, design in (
            ("cell_sort", 2, N * SORT_BYTES_PER_PARTICLE,
             N * DESIGN_SORT_BYTES_PER_PARTICLE + ncell * DESIGN_SORT_BYTES_PER_CELL),
            ("outer_kicks", 3, (N - n_wall) * KICK_BYTES_PER_PARTICLE,
             (N - n_wall) * DESIGN_KICK_BYTES_MOBILE + n_wall * DESIGN_KICK_BYTES_WALL)):
        ms = phase_ms[q] / max(n_phase, 1)
        hbm[name] = {"ms_per_step": round(ms, 4), "algorithmic_bytes": int(alg),
                     "gbs": round(alg / (ms * 1e-3) / 1e9, 1), "frac": round(alg / (ms * 1e-3) / HBM_PEAK, 4),
                     "design_bytes": int(design), "design_frac": round(design / (ms * 1e-3) / HBM_PEAK, 4)}
    other = {"inner_loop_ms_per_step": round(phase_ms[1] / max(n_phase, 1), 4),
             "platelet_lists_ms_per_step": round(phase_ms[5] / max(n_phase, 1), 4)}

    schedule = ("learned controller (ratio capped at %d; %d decision(s) in the timed steps)" % (k_max, inferences_timed)
                if mode else "fixed k=%d" % k)
    if three:
        schedule = ("three-level (interface every %d, flowing sublevel every %d inner steps), " % (args.k_if, args.k_sub)
                    + schedule)
    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": warm, "ms_per_step": 1e3 * t_mts / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-pair-forces/f64-state", "data": "synthetic",
        "config": {"workload": workload_name(d, args.workload, schedule),
                   "particles": N, "k": k if not mode else "controller", "mean_k": mean_k, "dt_inner": dt_in},
        "mts": {"tau_per_day": sim_mts / t_mts * SECONDS_PER_DAY, "mean_k": mean_k,
                "controller_inferences_timed": inferences_timed, "controller_inferences": int(d2.inferences),
                "fallbacks": int(d2.fallbacks), "rollbacks_timed": int(d1.rollbacks - d0.rollbacks),
                "rollbacks": int(d2.rollbacks),
                "inner_members": int(d2.inner_members), "inner_pair_entries": int(d2.inner_pairs),
                "skin": skin_mts, "skin_bead": skin_bead_mts,
                "t_span_steps": span, "t_span_tau": sim_span, "T_pec_span": Tpec_mts, "mean_k_span": mean_k_span,
                "span_tau_per_day": sim_span / (t_mts + t_rest) * SECONDS_PER_DAY},
        "sts_fp64": sts,
        "roofline": roofline,
        "hbm_phases": hbm,
        "platelet_phases": other,
    }
    if sts:
        out["simtime_speedup_vs_sts"] = out["mts"]["tau_per_day"] / sts["tau_per_day"]
        out["T_error_vs_sts"] = abs(Tpec_mts - sts["T_pec"]) / sts["T_pec"]
    if not args.skip_cpu:
        if clot:
            out["cpu_baseline"] = cpu_baseline_clot(d, inner_cpu, args.cpu_subset, mean_k_span, dt_in)
        else:
            out["cpu_baseline"] = cpu_baseline_channel(d, k, args.cpu_outer_steps)
    out["workload_generation_s"] = t_gen
    print(json.dumps(out), flush=True)
    if mode and inferences_timed == 0:
        note("the controller made no decision inside the timed steps")
        sys.exit(3)


if __name__ == "__main__":
    main()
