"""Benchmark of the DPD + CGMD multiple-time-stepping hot path on one MI355X.

Workload (synthetic, seeded): Poiseuille channel of 2,000,000 DPD particles (fluid +
frozen wall layers) in a 200 x 50 x 66.7 box, periodic in x and z, body force 0.02
along x, with 4 randomly placed platelets of 2,562 CG beads (level-4 icosphere on a
(3, 1, 3) oblate ellipsoid): 2,010,248 particles in all.  It stands in for the paper's
102-million-particle clot, whose platelet model is not available.

A "step" is one outer step of the whole hot path: cell-list rebuild (counting sort),
DPD outer forces, k inner steps of the platelet group (bonds, angles, WCA, platelet-
fluid forces), RESPA kicks/drifts, diagnostics and platelet features.

Legs, all from the same equilibrated state:
  * MTS (the headline `value`): float32 pair forces, float64 state, fixed ratio k
    (default 4, the controller's fallback) or the learned controller (--controller).
  * STS: float64 forces, ratio 1, run over the same simulated time.
Reported: particle-(outer)steps/s, simulated time per day, the simulated-time speedup
MTS/STS, and the relative difference of their time-averaged peculiar temperatures.
The roofline figure is for the dominant kernel (the DPD outer-force kernel), timed
live with HIP events on the library's stream during the MTS leg.
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
# Algorithmic HBM bytes (each array element read or written once):
#   DPD, per particle: x 24 + v 24 + id 4 + float4 position copy 16 read, float32 force 12 written
DPD_BYTES_PER_PARTICLE = 80
#   outer kicks and lazy drift, per mobile particle: half kick + k drifts (id 4, v 24 + 24,
#   force 12, member index 4, x 24 + 24) and closing half kick (id 4, v 24 + 24, force 12);
#   a frozen wall particle has its id read twice and its x and v copied into the members'
#   second state buffer (48 + 48)
KICK_BYTES_MOBILE, KICK_BYTES_WALL = 180, 104
#   counting sort, per particle: binning 40 (x 24, id 4, bin 4, rank 4), scatter 24 (bin,
#   rank, bin start, id; id and source written), rank and gather 160 (source, id, bin,
#   bin range 16; x, v 48 read; x, v 48, id, source, float copies 32, member index
#   written); per cell (two bins): histogram counts and clears 16, scan 16
SORT_BYTES_PER_PARTICLE, SORT_BYTES_PER_CELL = 224, 32
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_dpd_f32_channel2M_traffic.json")
DPD_SOURCES = ("paper_2205_14121_amd/csrc/dpd.hip", "paper_2205_14121_amd/csrc/common.h")
CONTROLLER_WEIGHTS = os.path.join(ROOT, "paper_2205_14121_amd", "data", "controller.npy")


def dpd_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in DPD_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per DPD launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy kernel), or None if the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != dpd_source_hash():
        return None
    return t.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed outer steps of the MTS leg")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--k", type=int, default=4, help="MTS ratio of the MTS leg")
    ap.add_argument("--equil", type=int, default=800, help="untimed float32 steps before both legs (STS; 800 at ratio 4 for the clot)")
    ap.add_argument("--controller", default=CONTROLLER_WEIGHTS if os.path.exists(CONTROLLER_WEIGHTS) else "",
                    help="trained controller weights (.npy) for the AI-MTS leg (default: the package's "
                         "trained weights when present)")
    ap.add_argument("--fixed", action="store_true", help="fixed ratio --k instead of the controller")
    ap.add_argument("--n-total", type=int, default=2_000_000)
    ap.add_argument("--workload", choices=("channel", "clot"), default="channel",
                    help="channel: the 2,000,000-particle Poiseuille channel with 4 platelets (headline); "
                         "clot: the largest single-GPU system, 100,000,000 particles in 3000x300x37 with "
                         "250 level-5 platelets, 180 of them pre-packed with Morse bonds (defaults then: "
                         "--steps 100 --warmup 64 --equil 400 at ratio 4, no host baseline)")
    ap.add_argument("--skip-sts", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-outer-steps", type=int, default=10, help="oracle outer steps timed on the host")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no benchmark: write the DPD traffic summary from two rocprofv3 --pmc counter "
                         "collections (FETCH_SIZE, WRITE_SIZE) of a run with --copy-calibration-mib")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this many MiB first (reference for HBM counters)")
    args = ap.parse_args()
    if args.workload == "clot":
        given = set(a.split("=")[0] for a in sys.argv[1:])
        if "--steps" not in given:
            args.steps = 100
        if "--warmup" not in given:
            args.warmup = 64  # the controller needs 64 feature rows before its first decision
        if "--equil" not in given:
            args.equil = 800  # outer steps at ratio 4 (4 time units) from the generated start
        args.skip_cpu = True
    return args


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


def cpu_baseline(sysd, k, outer_steps):
    """The oracle as it stands (float64, OpenMP over the host cores for the outer group)
    on a bounded sample: `outer_steps` RESPA outer steps of the same workload."""
    import oracle
    S = oracle.System(sysd)
    # the host share of one GPU is 16 cores; OMP_NUM_THREADS, when set, says what is available
    nthreads = min(16, int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1)
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


def write_traffic(fetch_csv, write_csv, copy_mib):
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
    run = ("python3 bench.py --fixed --steps 5 --warmup 1 --equil 200 --skip-sts --skip-cpu "
           "--copy-calibration-mib %d" % copy_mib)
    out = {"kernel": "k_dpd<float>", "workload": "channel, 2,010,248 particles", "copy_calibration_mib": copy_mib,
           "source_hash": dpd_source_hash(),
           "commands": ["rocprofv3 --pmc %s --kernel-include-regex 'k_dpd|elementwise' --output-format csv "
                        "-d gpurun_out/pmc_%s -o run -- %s" % (c, c.split("_")[0].lower(), run)
                        for c in ("FETCH_SIZE", "WRITE_SIZE")]
           + ["python3 bench.py --write-traffic gpurun_out/pmc_fetch/run_counter_collection.csv "
              "gpurun_out/pmc_write/run_counter_collection.csv --copy-calibration-mib %d" % copy_mib]}
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
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.copy_calibration_mib)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the sharding design is "
              "described in DESIGN.md); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2205_14121_amd.aimts as A

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
    if args.workload == "clot":
        import synth
        print("generating the 100,000,000-particle clot channel ...", file=sys.stderr, flush=True)
        d = synth.clot_channel()
    else:
        d = workload(args.n_total)
    t_gen = time.perf_counter() - t_gen
    print("workload ready (%.1f s)" % t_gen, file=sys.stderr, flush=True)
    N = int(d["n"])
    k = args.k
    # the level-5 platelets of the clot have modes twice as fast as level-4 ones: half the step
    dt_in = DT_INNER if args.workload == "channel" else 0.5 * DT_INNER
    series_cap = args.steps + args.warmup + 8

    # --- equilibration from the uniform random start (untimed) ---
    # the clot's packed layers face each other across 1.0 with beads 0.1 apart: a short
    # bead-bead skin keeps their pair lists at the beads that can interact
    skin_bead = 0.0 if args.workload == "channel" else 0.2
    eq = A.from_workload(d, fp32=True, skin=0.4, skin_bead=skin_bead)
    k_eq = 1 if args.workload == "channel" else 4
    eq.compute_forces(dt_in, k_eq)
    # the clot's level-5 meshes hit the rare angle-collapse spikes even at ratio 4: every
    # leg of that workload runs in checkpointed segments (a failed segment is rerun at
    # half its ratio, or at ratio 1 with fresh random numbers)
    seg_clot = 8 if args.workload == "clot" else 0
    eq.step(args.equil, dt_in, k_eq, rollback=seg_clot)
    x_eq, v_eq = eq.state()
    cnt_eq = eq.counters()
    eq.close()
    del eq
    print("equilibrated (%d steps)" % args.equil, file=sys.stderr, flush=True)

    # --- MTS leg (headline) ---
    use_ctrl = bool(args.controller) and not args.fixed
    # the controller's ratio is capped at 8, and the platelet-list skin is 0.5 so that one
    # outer step at that ratio stays within it even when a bead is briefly kicked to
    # several times its thermal speed (skins change list sizes, not results)
    k_max = 8 if use_ctrl else 0
    # The controller leg runs in checkpointed segments of outer steps (32; 8 for the
    # clot's short timed run): a segment whose stability checks fail (a bead of a nearly
    # collapsed surface triangle can be thrown to ten times its thermal speed for a few
    # inner steps) is restored and run again at the fallback ratio 4 inside the timed
    # region.
    rollback = (32 if args.workload == "channel" else 8) if use_ctrl else 0
    # the clot's controller leg lists bead pairs to 0.3 beyond the cutoff: at ratio 8 the
    # angle-collapse spikes exceed 0.2 several times per 100 steps (each a rolled-back
    # segment), while 0.4 lists so many facing-layer beads that every step slows more
    skin_bead_mts = 0.3 if args.workload == "clot" else skin_bead
    mts = A.from_workload(d, fp32=True, skin=0.5 if use_ctrl else 0.4, series_capacity=series_cap,
                          ctrl_max_batch=max(8, int(d["n_platelet"])), skin_bead=skin_bead_mts)
    mode = 0
    if use_ctrl:
        mts.ctrl_set_weights(np.load(args.controller).astype(np.float32))
        mode = 1
    mts.set_state(x_eq, v_eq)
    mts.set_counters(*cnt_eq)
    mts.compute_forces(dt_in, k)
    mts.step(args.warmup, dt_in, k, mode=mode, diag_every=1, k_max=k_max, rollback=rollback)
    mts.profile(1)  # HIP events around the DPD kernel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mts.step(args.steps, dt_in, k, mode=mode, diag_every=1, k_max=k_max, rollback=rollback)
    torch.cuda.synchronize()
    t_mts = time.perf_counter() - t0
    print("MTS leg timed (%.1f s)" % t_mts, file=sys.stderr, flush=True)
    prof_ms, prof_n = mts.get_profile()
    rows = mts.series()
    diag = mts.diag()
    # the cell sort and the outer kicks are timed in a short untimed segment afterwards
    # (events break the back-to-back kernel stream, so the timed steps carry only the
    # DPD pair of events)
    n_phase = min(args.steps, 50)
    mts.profile(4 | 8)
    mts.step(n_phase, dt_in, k, mode=mode, diag_every=0, k_max=k_max, rollback=rollback)
    torch.cuda.synchronize()
    phase_ms, _ = mts.get_profile()
    sim_mts = float(rows[-1, 0] - rows[args.warmup - 1, 0]) if args.warmup > 0 else float(rows[-1, 0])
    from paper_2205_14121_amd.controller import time_average
    Tpec_mts = time_average(rows[args.warmup:], 3)  # over simulated time (rows of a varying k)
    mean_k = time_average(rows[args.warmup:], 7)
    value = N * args.steps / t_mts

    # --- STS leg: float64, ratio 1, same simulated time from the same state ---
    sts = None
    if not args.skip_sts:
        n_sts = int(round(sim_mts / dt_in))
        ctx = A.from_workload(d, fp32=False, skin=0.4, series_capacity=n_sts + 8, skin_bead=skin_bead)
        ctx.set_state(x_eq, v_eq)
        ctx.set_counters(*cnt_eq)
        ctx.compute_forces(dt_in, 1)
        ctx.step(args.warmup, dt_in, 1, rollback=seg_clot)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(n_sts, dt_in, 1, diag_every=1, rollback=seg_clot)
        torch.cuda.synchronize()
        t_sts = time.perf_counter() - t0
        print("STS leg timed (%d steps, %.1f s)" % (n_sts, t_sts), file=sys.stderr, flush=True)
        srows = ctx.series()
        Tpec_sts = float(np.mean(srows[:, 3]))
        sts = {"particle_steps_per_s": N * n_sts / t_sts, "steps": n_sts, "ms_per_step": 1e3 * t_sts / n_sts,
               "tau_per_day": n_sts * dt_in / t_sts * SECONDS_PER_DAY, "T_pec": Tpec_sts,
               "rollbacks": int(ctx.diag().rollbacks)}
        ctx.close()

    # --- roofline of the dominant kernel (DPD outer forces, float32) ---
    dpd_ms = prof_ms[0] / max(prof_n[0], 1)
    n_fluid = int(d["n_fluid"])
    slots = n_fluid * SLOTS_PER_PARTICLE[True]
    achieved = slots / (dpd_ms * 1e-3) / 1e12
    dpd_bytes = N * DPD_BYTES_PER_PARTICLE
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK / 1e12, 3),
                "unit": "T lane-slots/s", "frac": round(achieved * 1e12 / VALU_PEAK, 4),
                # the committed counter summary is for the channel workload's DPD launch
                "traffic": measured_traffic() if args.workload == "channel" else None,
                "kernel": "k_dpd<float>", "avg_ms": round(dpd_ms, 4),
                "launches": int(prof_n[0]), "algorithmic_slots_per_launch": slots,
                "algorithmic_bytes_per_launch": dpd_bytes,
                "hbm_gbs": round(dpd_bytes / (dpd_ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(dpd_bytes / (dpd_ms * 1e-3) / HBM_PEAK, 4)}
    # the HBM-bound phases of the step, timed the same way
    n_wall = int(d["n_wall"])
    ncell = int(np.prod(np.floor(np.asarray(d["box_L"]) / 1.0)))
    hbm = {}
    for name, q, nbytes in (("cell_sort", 2, N * SORT_BYTES_PER_PARTICLE + ncell * SORT_BYTES_PER_CELL),
                            ("outer_kicks", 3, (N - n_wall) * KICK_BYTES_MOBILE + n_wall * KICK_BYTES_WALL)):
        ms = phase_ms[q] / max(n_phase, 1)
        hbm[name] = {"ms_per_step": round(ms, 4), "algorithmic_bytes": int(nbytes),
                     "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1), "frac": round(nbytes / (ms * 1e-3) / HBM_PEAK, 4)}

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_mts / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-pair-forces/f64-state", "data": "synthetic",
        "config": {"workload": workload_name(d, args.workload, "learned controller" if mode else "fixed k=%d" % k),
                   "particles": N, "k": k if not mode else "controller", "mean_k": mean_k, "dt_inner": dt_in},
        "mts": {"tau_per_day": sim_mts / t_mts * SECONDS_PER_DAY, "T_pec": Tpec_mts, "mean_k": mean_k,
                "controller_inferences": int(diag.inferences), "fallbacks": int(diag.fallbacks),
                "rollbacks": int(diag.rollbacks)},
        "sts_fp64": sts,
        "roofline": roofline,
        "hbm_phases": hbm,
    }
    if sts:
        out["simtime_speedup_vs_sts"] = out["mts"]["tau_per_day"] / sts["tau_per_day"]
        out["T_error_vs_sts"] = abs(Tpec_mts - sts["T_pec"]) / sts["T_pec"]
    if not args.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(d, k, args.cpu_outer_steps)
    out["workload_generation_s"] = t_gen
    print(json.dumps(out))


if __name__ == "__main__":
    main()
