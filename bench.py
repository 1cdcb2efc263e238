#!/usr/bin/env python
"""Benchmark of the docking hot path on one MI355X.

Headline: the screening stream -- 100,000 (ligand, pocket) jobs in seeded
random order over the 16 pockets (20..30 A boxes, all maps resident in HBM)
of an 8,000-atom receptor; ligands of 8..80 atoms and 0..20 torsions; 16
Monte Carlo chains x 300 steps per job, every step a RILC-BFGS local
optimisation (<= 30 iterations).  One bench step is 1/--steps of the stream
(a contiguous slice of the seeded order) docked by the batched persistent
launches (one per ligand size class, hipGraph-replayed), so --steps steps
cover the whole stream; warm-up steps replay the first slices before the
timed region.  Inputs are seeded and synthetic and stay resident in HBM.

Prints one JSON line: docks/s of the whole stream (value), score+grad
evaluations/s, the per-job service time p50/p99, the roofline of the dominant
kernel (HIP events on the stream the kernels run on), the oracle timed on the
host on the first 64 jobs of the stream, and the secondary legs (the other
workloads, the plain per-job launch path, the differentiation form).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12   # MI355X vector FP32, FLOP/s
PEAK_HBM = 8.0e12             # MI355X HBM3E, B/s
MAP_BYTES_PER_ATOM = 32       # 8 trilinear corners x 4 B, per atom and evaluation
METRIC = "ligand-pocket docks/s and score+grad evals/s, batched vs plain on 1 MI355X"

# Algorithmic work of one score+grad evaluation, the planning count of the
# method's operations: 70 flops per intra pair (distance, the five terms and
# their derivative, the forces on both atoms), 90 per atom (frame transform,
# trilinear value and gradient, force and torque accumulation) and 60 per
# torsion (local rotation, frame composition, torsion derivative); its
# transcendentals count as one flop each.  Every evaluation counts in full,
# line-search trials included.  A second figure, the work performed, takes
# out the pair work of the trials the kernel decides from their map energy
# and the intra lower bound, which skip their pair loop.
FLOP_PAIR, FLOP_ATOM, FLOP_TORS = 70, 90, 60


def log(msg):
    """Progress on stderr (stdout carries the one JSON line)."""
    print("[bench %7.1fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def flops_per_eval(n_pairs, n_atoms, n_tors):
    return FLOP_PAIR * np.asarray(n_pairs, np.float64) + FLOP_ATOM * np.asarray(n_atoms, np.float64) + \
        FLOP_TORS * np.asarray(n_tors, np.float64)


def flops_of(n_evals, n_pairs, n_atoms, n_tors):
    """Planning-count flops of evaluations, each counted in full; per job, or
    per element of arrays of jobs."""
    return np.asarray(n_evals, np.float64) * flops_per_eval(n_pairs, n_atoms, n_tors)


def flops_performed(n_evals, n_bounded, n_pairs, n_atoms, n_tors):
    """The planning count less the pair work of the n_bounded trials decided
    by the intra bound, which run no pair loop."""
    return flops_of(n_evals, n_pairs, n_atoms, n_tors) - \
        np.asarray(n_bounded, np.float64) * FLOP_PAIR * np.asarray(n_pairs, np.float64)


# A lighter count, from the operations the kernel must perform once the
# method is fixed: per intra pair tested 8 flops, per pair inside the cutoff
# the terms (20) and with the gradient the derivative and both forces (16);
# per atom the frame transform and trilinear value (48) and with the gradient
# the trilinear gradient and force/torque accumulation (43); per torsion the
# local rotation and frame composition (109) and with the gradient the
# torsion derivative (32); per evaluation the root frame and the BFGS vector
# work.  A line-search trial above the sufficient-decrease bound needs only
# the energy, so the gradient part counts once per evaluation that computed
# it.  Reported beside the headline count.
def flops_light(n_evals, n_grads, pairs_in, n_atoms, n_tors, n_pairs, n_bounded=0, m=5):
    n_evals = np.asarray(n_evals, np.float64)
    n_grads = np.asarray(n_grads, np.float64)
    energy = 8 * n_pairs + 48 * n_atoms + 109 * n_tors + 50 + (4 * m + 10) * (6 + n_tors)
    grad = 43 * n_atoms + 32 * n_tors
    share = np.where(n_evals > 0, n_grads / np.maximum(n_evals, 1), 0.0)
    pair_test = 8 * np.asarray(n_bounded, np.float64) * n_pairs   # trials decided by the bound test no pair
    return float(np.sum(n_evals * energy - pair_test + n_grads * grad +
                        np.asarray(pairs_in, np.float64) * (20 + share * 16)))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4, help="timed steps; each docks 1/steps of the stream")
    ap.add_argument("--warmup", type=int, default=1, help="untimed steps (replays of the first slices)")
    ap.add_argument("--stream-jobs", type=int, default=100000, help="jobs of the screening stream (a prefix)")
    ap.add_argument("--workers", type=int, default=16, help="processes generating the synthetic ligands")
    ap.add_argument("--job-order", choices=["stream", "box"], default="box",
                    help="order in which a batched launch hands out the slice's jobs: the stream's, or grouped "
                         "by pocket (outputs are identical)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-score", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip every secondary leg (the headline, its oracle and the peaks only)")
    ap.add_argument("--batch-ligands", type=int, default=4096,
                    help="ligands of the uneven batch (x 5 pockets = jobs)")
    ap.add_argument("--plain-jobs", type=int, default=20, help="jobs of the uneven batch run one launch each")
    ap.add_argument("--stream-plain-jobs", type=int, default=48,
                    help="jobs of the stream run one launch each (and batched) for the plain comparison")
    ap.add_argument("--cpu-jobs", type=int, default=64, help="stream jobs the oracle docks on all host cores")
    ap.add_argument("--chains", type=int, default=256, help="chains per pocket of the multi-pocket leg")
    ap.add_argument("--mc-steps", type=int, default=1000, help="MC steps of the multi-pocket leg")
    ap.add_argument("--sweep-steps", type=int, default=1000, help="MC steps per chain in the box-size sweep")
    ap.add_argument("--leg", choices=["tiny", "multi_pocket", "score", "local_opt", "batching", "stream_plain",
                                      "box_sweep", "surface"], default=None,
                    help="run only this secondary leg and print its JSON (for profiling it alone)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (calibrates the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; --gpus %d is not supported "
              "(across GPUs the work would shard by pocket, each GPU building only its pockets' maps)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": 4 * n}), flush=True)
        return

    from paper_2506_20043_amd import synth as S
    workers = max(1, min(args.workers, len(os.sched_getaffinity(0))))
    # synthetic inputs first, with forked workers, before the GPU is touched
    need_batch = args.leg == "batching" or (args.leg is None and not args.no_extra)
    need_stream = args.leg in (None, "stream_plain")
    cfg5 = S.CONFIGS["screening"]
    inputs = {}
    t_gen = time.perf_counter()
    if need_stream:
        jobs5 = S.make_jobs(cfg5)[:args.stream_jobs]
        used = np.unique(jobs5[:, 0])
        mols5 = S.make_ligands_parallel("screening", int(used.max()) + 1, 0, workers)
        inputs["stream"] = (S.make_receptor(cfg5), mols5, jobs5)
    if need_batch:
        inputs["batch"] = S.make_ligands_parallel("uneven_batch", args.batch_ligands, 0, workers)
    gen_s = time.perf_counter() - t_gen
    log("synthetic inputs generated in %.1f s" % gen_s)

    import paper_2506_20043_amd as pv

    ctx = pv.Context(0)
    stream = torch.cuda.current_stream()
    if args.leg:
        legs = {"tiny": lambda: bench_tiny(pv, S, ctx, stream, args),
                "multi_pocket": lambda: bench_multi_pocket(pv, S, ctx, stream, args),
                "score": lambda: bench_score(pv, S, ctx, stream),
                "local_opt": lambda: bench_local_opt(pv, S, ctx, stream),
                "batching": lambda: bench_batching(pv, S, ctx, stream, args, inputs["batch"]),
                "stream_plain": lambda: bench_stream_plain(pv, S, ctx, stream, args, inputs["stream"]),
                "box_sweep": lambda: bench_box_sweep(pv, S, ctx, stream, args),
                "surface": lambda: bench_surface(pv, S, ctx, stream)}
        print(json.dumps({"leg": args.leg, "result": legs[args.leg]()}), flush=True)
        return

    log("headline: screening stream, %d jobs in %d steps after %d warm-up steps"
        % (len(inputs["stream"][2]), args.steps, args.warmup))
    result, head = bench_stream(pv, S, ctx, stream, args, inputs["stream"])
    log("headline: %.1f docks/s" % result["value"])
    result["input_generation_s"] = gen_s

    def leg(name, fn):
        log("leg %s" % name)
        return fn()

    if not args.no_extra:
        result["stream_plain"] = leg("stream_plain", lambda: bench_stream_plain(pv, S, ctx, stream, args,
                                                                                inputs["stream"]))
        result["batched_over_plain"] = result["value"] / result["stream_plain"]["plain"]["docks_per_s"]
        result["tiny"] = leg("tiny", lambda: bench_tiny(pv, S, ctx, stream, args))
        result["multi_pocket"] = leg("multi_pocket", lambda: bench_multi_pocket(pv, S, ctx, stream, args))
        result["batching"] = leg("batching", lambda: bench_batching(pv, S, ctx, stream, args, inputs["batch"]))
        if not args.no_score:
            result["score_grad"] = leg("score", lambda: bench_score(pv, S, ctx, stream))
            result["local_opt"] = leg("local_opt", lambda: bench_local_opt(pv, S, ctx, stream))
        result["box_sweep"] = leg("box_sweep", lambda: bench_box_sweep(pv, S, ctx, stream, args))
        result["surface"] = leg("surface", lambda: bench_surface(pv, S, ctx, stream))
    result["measured_peaks"] = leg("measured_peaks", lambda: measure_peaks(pv, ctx, stream))
    if not args.no_cpu:
        result["cpu_baseline"] = leg("cpu_baseline (oracle)", lambda: cpu_baseline_stream(S, inputs["stream"], head,
                                                                                         args))
        if not args.no_extra:
            result["tiny"]["oracle"] = leg("tiny oracle", lambda: cpu_oracle_tiny(S, args))
            result["batching"]["oracle"] = leg("batch oracle", lambda: cpu_oracle_batch(S, inputs["batch"], args))
    log("done")
    print(json.dumps(result), flush=True)


def _jobs_info(ligs, jobs):
    """Per job: atoms, torsions and intra pairs of its ligand."""
    inf = ligs.infos[np.asarray(jobs)[:, 0]]
    return inf[:, 0].astype(np.int64), inf[:, 2].astype(np.int64), inf[:, 3].astype(np.int64)


def bench_stream(pv, S, ctx, stream, args, inp):
    """The headline: the screening stream in --steps slices of its seeded
    order, each docked by one persistent launch per ligand size class
    (ligands of at most 64 atoms, larger ones) with device timestamps."""
    import torch
    (rx, rt, bxs), mols, jobs = inp
    cfg = S.CONFIGS["screening"]
    n = len(jobs)
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=10.0)
    torch.cuda.synchronize()
    grid_ms = min(_timed(stream, grids.rebuild) for _ in range(3))
    ligs = pv.Ligands(ctx, mols)
    N, T, P = _jobs_info(ligs, jobs)
    big = N > 64
    order = pv.PV_DOCK_BOX_ORDER if args.job_order == "box" else 0
    params = pv.dock_params(chains=cfg.chains, steps=cfg.steps, seed=S.philox_seed(cfg),
                            flags=pv.PV_DOCK_GRAPH | pv.PV_DOCK_TIMESTAMPS | order)
    K = args.steps
    bounds = np.linspace(0, n, K + 1).astype(np.int64)
    steps = []
    for k in range(K):
        sl = np.arange(bounds[k], bounds[k + 1])
        cls = []
        for c in (0, 1):
            idx = sl[big[sl] == bool(c)]
            cls.append((pv.Plan(ctx, grids, ligs, jobs[idx], params), idx) if len(idx) else None)
        steps.append(cls)

    def run_step(k, evs=None):
        for c in (0, 1):
            if evs is not None:
                evs[c].record(stream)
            if steps[k][c] is not None:
                steps[k][c][0].run()
        if evs is not None:
            evs[2].record(stream)

    for w in range(args.warmup):
        run_step(w % K)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        run_step(k, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # outputs per job, in stream order
    ev = np.zeros(n, np.int64)
    grads = np.zeros(n, np.int64)
    bnd = np.zeros(n, np.int64)
    pin = np.zeros(n, np.int64)
    tstart = np.zeros(n, np.int64)
    tend = np.zeros(n, np.int64)
    status = np.zeros(n, np.int32)
    best = np.zeros(n, np.float32)
    ms_cls = np.zeros((K, 2))
    sched = [None, None]
    for k in range(K):
        for c in (0, 1):
            ms_cls[k, c] = evs[k][c].elapsed_time(evs[k][c + 1])
            if steps[k][c] is None:
                continue
            plan, idx = steps[k][c]
            o = plan.outputs()
            ch = plan.params.chains
            ev[idx] = o["job_evals"].cpu().numpy()
            grads[idx] = o["chain_grads"].cpu().numpy().reshape(-1, ch).sum(axis=1)
            bnd[idx] = o["chain_bounded"].cpu().numpy().reshape(-1, ch).sum(axis=1)
            pin[idx] = o["chain_pairs"].cpu().numpy().reshape(-1, ch).sum(axis=1)
            tstart[idx] = o["job_t_start"].cpu().numpy()
            tend[idx] = o["job_t_end"].cpu().numpy()
            status[idx] = o["job_status"].cpu().numpy()
            best[idx] = o["job_best_e"].cpu().numpy()
            if sched[c] is None:
                sc = plan.schedule(0)
                sched[c] = {"variant": VARIANTS[sc["variant"]], "workgroups": sc["workgroups"],
                            "lds_bytes": sc["lds_bytes"], "per_cu": sc["per_cu"]}
            plan.close()
    svc = (tend - tstart) / 100.0                 # device clock, 100 MHz -> us
    fl = flops_of(ev, P, N, T)
    dock_ms = float(ms_cls.sum())
    cls_stats = []
    for c in (0, 1):
        m = big == bool(c)
        ms_c = float(ms_cls[:, c].sum())
        launches = int(sum(1 for k in range(K) if steps[k][c] is not None))
        cls_stats.append({
            "class": "ligands of at most 64 atoms" if c == 0 else "ligands of more than 64 atoms",
            "kernel": kernel_name(sched[c]["variant"], params.bfgs_m) if sched[c] else None, "schedule": sched[c],
            "jobs": int(m.sum()), "launches": launches, "launch_ms_mean": ms_c / max(launches, 1),
            "evals": int(ev[m].sum()), "evals_per_s": float(ev[m].sum() / (ms_c * 1e-3)) if ms_c else 0.0,
            "tflops": float(fl[m].sum() / (ms_c * 1e-3) / 1e12) if ms_c else 0.0})
    dom = cls_stats[0]
    dom_fl = float(fl[~big].sum())
    achieved = dom_fl / (float(ms_cls[:, 0].sum()) * 1e-3)
    light = flops_light(ev[~big], grads[~big], pin[~big], N[~big], T[~big], P[~big], bnd[~big])
    performed = float(flops_performed(ev, bnd, P, N, T)[~big].sum())
    gather_b = float((ev * MAP_BYTES_PER_ATOM * N)[~big].sum())
    map_mb = sum(8 * int(np.prod(grids.info(b)[0])) * 4 for b in range(len(bxs))) / 1e6
    result = {
        "metric": METRIC,
        "value": n / wall,
        "unit": "docks/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded receptor, pockets, ligands and job order; no datasets)",
        "config": {
            "workload": "screening stream: %d (ligand, pocket) jobs in seeded random order; 8,000-atom receptor "
                        "in a 60 A cube, 16 pockets of 20..30 A at 0.375 A (%.0f MB of FP32 maps resident in HBM); "
                        "%d ligands of 8..80 atoms / 0..20 torsions; 16 chains x 300 MC steps per job, BFGS <= 30 "
                        "iterations; batched persistent launches (hipGraph), one per ligand size class; "
                        "step = 1/%d of the stream" % (n, map_mb, len(mols), K),
            "jobs": n, "chains": cfg.chains, "mc_steps": cfg.steps, "job_order": args.job_order,
            "parallelism": "single GPU",
        },
        "evals_per_s": float(ev.sum() / wall),
        "evals": int(ev.sum()),
        "evals_decided_by_bound": int(bnd.sum()),
        "dock_ms": dock_ms,
        "docks_per_s_with_grid_build": n / (wall + grid_ms * 1e-3),
        "grid_build_ms_16_pockets": grid_ms,
        "service_us_p50": float(np.percentile(svc, 50)),
        "service_us_p99": float(np.percentile(svc, 99)),
        "service_us_max": float(svc.max()),
        "jobs_status": {"nonfinite": int(np.sum((status & 1) != 0)), "budget": int(np.sum((status & 2) != 0)),
                        "best_pose_outside_box": int(np.sum((status & 4) != 0))},
        "best_e_median": float(np.median(best)),
        "classes": cls_stats,
        "roofline": {
            "bound": "alu",
            "kernel": dom["kernel"] + " (persistent MC + BFGS, ligands of at most 64 atoms)",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR,
            "traffic": recorded_traffic(args.job_order),
            "flops_per_launch": dom_fl / max(dom["launches"], 1),
            "flops_per_eval_mean": dom_fl / max(dom["evals"], 1),
            "launch_ms": dom["launch_ms_mean"],
            # the same count less the pair work of the trials decided by the
            # intra bound, which skip their pair loop
            "work_performed": {"tflops": performed / (float(ms_cls[:, 0].sum()) * 1e-3) / 1e12,
                               "frac": performed / (float(ms_cls[:, 0].sum()) * 1e-3) / PEAK_FP32_VECTOR},
            "flops_light": {"tflops": light / (float(ms_cls[:, 0].sum()) * 1e-3) / 1e12,
                            "frac": light / (float(ms_cls[:, 0].sum()) * 1e-3) / PEAK_FP32_VECTOR},
            "map_gather": {"bytes_per_launch": gather_b / max(dom["launches"], 1),
                           "achieved_GBps": gather_b / (float(ms_cls[:, 0].sum()) * 1e-3) / 1e9,
                           "peak_GBps": PEAK_HBM / 1e9,
                           "frac": gather_b / (float(ms_cls[:, 0].sum()) * 1e-3) / PEAK_HBM},
        },
    }
    head = {"jobs": jobs, "ev": ev, "wall": wall, "n": n}
    return result, head


def native_source_hash():
    """SHA-256 of the native sources (kernels, launch planning, ligand
    layout) in file-name order, with comments and runs of white space
    removed: an edit to a comment keeps the counter record valid, any change
    to the code does not."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2506_20043_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".h")):
            txt = open(os.path.join(csrc, f), encoding="utf-8").read()
            txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
            txt = re.sub(r"//[^\n]*", " ", txt)
            h.update(re.sub(r"\s+", " ", txt).encode())
    return h.hexdigest()


def kernel_name(variant, m):
    """The dock kernel instantiation a schedule runs: its variant's atoms per
    lane and slot layout, and the history capacity (5 when m <= 5, else 8)."""
    a, sl = {"slots": (1, "true"), "gather": (1, "false"), "gather2": (2, "false")}[variant]
    return "dock_kernel<%d, %s, %d>" % (a, sl, 5 if m <= 5 else 8)


def recorded_traffic(job_order):
    """HBM bytes per launch of the dominant dock kernel from the committed
    rocprofv3 counter record, or None when the native sources changed since
    the counters were taken or they were taken under another job order."""
    prof = os.path.join(ROOT, "profiles", "dock_kernel_screening_stream.md")
    if not os.path.exists(prof):
        return None
    rec = None
    for line in open(prof):
        if line.startswith("traffic_record: "):
            rec = json.loads(line[len("traffic_record: "):])
    if rec is None or rec.get("job_order") != job_order:
        return None
    if native_source_hash() != rec.get("native_source_sha256"):
        return None
    return rec["dock_traffic_bytes_per_launch"]


def plan_workgroups(plan):
    return int(plan.params.workgroups) if plan.params.workgroups else None


def bench_multi_pocket(pv, S, ctx, stream, args):
    """The multi-pocket single ligand: 5,000-atom receptor, 5 pockets of
    24 A, one 35-atom / 8-torsion ligand, --chains chains x --mc-steps MC
    steps per pocket as one persistent hipGraph launch (schedule from the
    autotuner), against the plain path (one launch per pocket); then the
    same dock gated by the consistency check, and the output stage."""
    import torch
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    mols = S.make_ligands(cfg)
    seed = S.philox_seed(cfg)
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=10.0)
    torch.cuda.synchronize()
    grid_ms = min(_timed(stream, grids.rebuild) for _ in range(3))
    ligs = pv.Ligands(ctx, mols)
    n_atoms, n_frag, n_tors, n_pairs = ligs.info(0)[:4]
    jobs = [(0, b) for b in range(len(bxs))]
    params = pv.dock_params(chains=args.chains, steps=args.mc_steps, seed=seed, flags=pv.PV_DOCK_GRAPH)
    plan = pv.Plan(ctx, grids, ligs, jobs, params)
    tuning = tune(plan, stream)
    plan.run()
    torch.cuda.synchronize()
    ms = min(_timed(stream, plan.run) for _ in range(2))
    out = plan.outputs()
    n_evals = int(out["job_evals"].sum().item())
    n_bnd = int(out["chain_bounded"].sum().item())
    fl = float(flops_of(n_evals, n_pairs, n_atoms, n_tors))
    fl_done = float(flops_performed(n_evals, n_bnd, n_pairs, n_atoms, n_tors))
    res = {"workload": "multi-pocket single ligand: 5,000-atom receptor in a 50 A cube, 5 pockets of 24 A "
                       "(65^3 x 8 FP32 maps each), one %d-atom ligand with %d torsions (%d intra pairs), %d chains "
                       "x %d MC steps per pocket" % (n_atoms, n_tors, n_pairs, args.chains, args.mc_steps),
           "dock_ms": ms, "docks_per_s": len(jobs) / (ms * 1e-3), "evals_per_s": n_evals / (ms * 1e-3),
           "evals": n_evals, "grid_ms": grid_ms,
           "docks_per_s_with_grid_build": len(jobs) / ((ms + grid_ms) * 1e-3),
           "tflops": fl / (ms * 1e-3) / 1e12, "frac_fp32": fl / (ms * 1e-3) / PEAK_FP32_VECTOR,
           "tflops_work_performed": fl_done / (ms * 1e-3) / 1e12, "autotune": tuning}
    if not args.no_plain:
        plan.run(plain=True)
        torch.cuda.synchronize()
        plain_ms = _timed(stream, lambda: plan.run(plain=True))
        res["plain"] = {"docks_per_s": len(jobs) / (plain_ms * 1e-3), "evals_per_s": n_evals / (plain_ms * 1e-3),
                        "dock_ms": plain_ms}
        res["batched_over_plain"] = plain_ms / ms
    res["output_stage"] = bench_output(pv, plan, stream)
    res["consistency_check"] = bench_consistency(pv, ctx, grids, ligs, jobs, args, seed, stream, n_evals, ms,
                                                 plan.outputs())
    plan.close()
    return res


def bench_tiny(pv, S, ctx, stream, args):
    """The tiny configuration: 2,000-atom receptor, one 20 A pocket, one
    20-atom / 4-torsion ligand, 8 chains x 200 MC steps, batched and plain."""
    import torch
    cfg = S.CONFIGS["tiny"]
    rx, rt, bxs = S.make_receptor(cfg)
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=10.0)
    torch.cuda.synchronize()
    grid_ms = min(_timed(stream, grids.rebuild) for _ in range(3))
    ligs = pv.Ligands(ctx, S.make_ligands(cfg))
    params = pv.dock_params(chains=cfg.chains, steps=cfg.steps, seed=S.philox_seed(cfg), flags=pv.PV_DOCK_GRAPH)
    plan = pv.Plan(ctx, grids, ligs, [(0, 0)], params)
    plan.run()
    torch.cuda.synchronize()
    ms = min(_timed(stream, plan.run) for _ in range(3))
    ms_plain = min(_timed(stream, lambda: plan.run(plain=True)) for _ in range(3))
    out = plan.outputs()
    ev = int(out["job_evals"].sum().item())
    best = float(out["job_best_e"][0].item())
    plan.close()
    return {"workload": "tiny: 2,000-atom receptor in a 30 A cube, one 20 A pocket (55^3 x 8 maps), one 20-atom "
                        "ligand with 4 torsions, 8 chains x 200 MC steps",
            "grid_ms": grid_ms, "dock_ms": ms, "docks_per_s": 1.0 / (ms * 1e-3), "evals": ev,
            "evals_per_s": ev / (ms * 1e-3), "plain_dock_ms": ms_plain, "job_best_e": best}


def bench_score(pv, S, ctx, stream):
    """score+grad of the differentiation workload: 16,384 poses of 64
    ligands (40 atoms, 10 torsions) in one 24 A pocket: 5 runs of 200 calls
    (1,000 in all), the median run's time per call."""
    import torch
    cfg = S.CONFIGS["differentiation"]
    rx, rt, bxs = S.make_receptor(cfg)
    mols = S.make_ligands(cfg)
    grids = pv.build_grids(ctx, rx, rt, bxs[:1], penalty_slope=10.0)
    ligs = pv.Ligands(ctx, mols)
    dims, org = grids.info(0)
    lo, hi = org.astype(np.float64), org + 0.375 * (dims - 1)
    dof = torch.tensor(S.poses(S.rng(cfg.index, S.STREAM_POSES), cfg.n_poses, lo, hi, 10), device="cuda")
    lig = torch.tensor(np.repeat(np.arange(64, dtype=np.int32), 256), device="cuda")
    box = torch.zeros(cfg.n_poses, dtype=torch.int32, device="cuda")
    for _ in range(3):
        pv.score_grad(ctx, grids, ligs, lig, box, dof)
    torch.cuda.synchronize()
    reps, runs = 200, []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            pv.score_grad(ctx, grids, ligs, lig, box, dof)
        b.record(stream)
        torch.cuda.synchronize()
        runs.append(a.elapsed_time(b) / reps)
    ms = float(np.median(runs))
    return {"workload": "16,384 poses, 64 ligands of 40 atoms / 10 torsions, one 24 A pocket",
            "ms_per_call": ms, "evals_per_s": cfg.n_poses / (ms * 1e-3), "calls": 5 * reps,
            "ms_per_call_runs": runs}


def bench_local_opt(pv, S, ctx, stream):
    """RILC-BFGS alone (pv_local_opt, at most 30 iterations) from the
    differentiation workload's 16,384 poses: 5 timed calls, the median."""
    import torch
    cfg = S.CONFIGS["differentiation"]
    rx, rt, bxs = S.make_receptor(cfg)
    grids = pv.build_grids(ctx, rx, rt, bxs[:1], penalty_slope=10.0)
    ligs = pv.Ligands(ctx, S.make_ligands(cfg))
    dims, org = grids.info(0)
    lo, hi = org.astype(np.float64), org + 0.375 * (dims - 1)
    dof = torch.tensor(S.poses(S.rng(cfg.index, S.STREAM_POSES), cfg.n_poses, lo, hi, 10), device="cuda")
    lig = torch.tensor(np.repeat(np.arange(64, dtype=np.int32), 256), device="cuda")
    box = torch.zeros(cfg.n_poses, dtype=torch.int32, device="cuda")
    params = pv.dock_params()
    pv.local_opt(ctx, grids, ligs, lig, box, dof, params)
    torch.cuda.synchronize()
    runs = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        _, e, ne = pv.local_opt(ctx, grids, ligs, lig, box, dof, params)
        b.record(stream)
        torch.cuda.synchronize()
        runs.append(a.elapsed_time(b))
    ms = float(np.median(runs))
    evals = int(ne.sum().item())
    e0 = pv.score_grad(ctx, grids, ligs, lig, box, dof, grad=False)["energy"]
    return {"workload": "BFGS (<= 30 iterations) from 16,384 poses of 64 ligands of 40 atoms / 10 torsions",
            "ms": ms, "poses_per_s": cfg.n_poses / (ms * 1e-3), "evals": evals,
            "evals_per_s": evals / (ms * 1e-3), "mean_energy_start": float(e0.mean().item()),
            "mean_energy_end": float(e.mean().item())}


def bench_consistency(pv, ctx, grids, ligs, jobs, args, seed, stream, evals_off, ms_off, out_off):
    """The same multi-pocket dock with the first-order consistency check
    gating every step's BFGS: evaluations saved and the change of the chain
    bests against the run without it."""
    import torch
    params = pv.dock_params(chains=args.chains, steps=args.mc_steps, seed=seed, flags=pv.PV_DOCK_GRAPH,
                            consistency=1)
    plan = pv.Plan(ctx, grids, ligs, jobs, params)
    tune(plan, stream)
    plan.run()
    torch.cuda.synchronize()
    ms = _timed(stream, plan.run)
    out = plan.outputs()
    ev = int(out["job_evals"].sum().item())
    on_best = out["chain_best_e"].cpu().numpy()
    off_best = out_off["chain_best_e"].cpu().numpy()
    res = {"dock_ms": ms, "docks_per_s": len(jobs) / (ms * 1e-3), "evals_per_s": ev / (ms * 1e-3),
           "evals_per_dock": ev / len(jobs), "evals_per_dock_without": evals_off / len(jobs),
           "evals_saved_frac": 1.0 - ev / evals_off, "speedup_over_without": ms_off / ms,
           "mean_chain_best": float(on_best.mean()), "mean_chain_best_without": float(off_best.mean()),
           "job_best": [float(v) for v in out["job_best_e"].cpu().numpy()],
           "job_best_without": [float(v) for v in out_off["job_best_e"].cpu().numpy()]}
    plan.close()
    return res


def bench_output(pv, plan, stream):
    """The output stage over a dock plan's last chain bests: clustering at
    1 A, up to 20 modes per job, 30 BFGS iterations of refinement each,
    rescoring, r.m.s.d. filter and sort."""
    import torch
    out = plan.outputs()
    res = pv.output_stage(plan, out["chain_best_e"], out["chain_best_dof"])
    torch.cuda.synchronize()
    ms = _timed(stream, lambda: pv.output_stage(plan, out["chain_best_e"], out["chain_best_dof"]))
    n = res["n_modes"].cpu().numpy()
    return {"ms": ms, "jobs": int(plan.n_jobs), "jobs_per_s": plan.n_jobs / (ms * 1e-3),
            "modes_per_job_mean": float(n.mean()), "best_affinity": float(res["mode_affinity"][:, 0].min().item())}


VARIANTS = ["slots", "gather", "gather2"]


def tune(plan, stream, steps=20):
    """Runs the library's autotuner on the plan (outside every timed region)
    and reports the schedules it set."""
    t = time.perf_counter()
    res = plan.autotune(steps=steps, repeats=2, stream=stream)
    dt = time.perf_counter() - t
    sched = []
    for g in range(plan.groups()):
        sc = plan.schedule(g)
        sched.append({"variant": VARIANTS[sc["variant"]], "workgroups": sc["workgroups"],
                      "lds_bytes": sc["lds_bytes"], "per_cu": sc["per_cu"], "jobs": sc["n_jobs"]})
    return {"schedules": sched, "candidates_timed": sum(1 for r in res if not r["cached"]),
            "tune_steps": steps, "tune_s": dt}


def _timed(stream, fn):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def bench_batching(pv, S, ctx, stream, args, mols):
    """Batched vs plain on the uneven batch: --batch-ligands ligands of
    10..60 atoms and 0..15 torsions (4,096: the whole batch), each docked into
    the 5 pockets of the multi-pocket receptor, 32 chains x 500 MC steps per
    job, as one persistent hipGraph launch whose schedule the autotuner
    picks, handing out the most costly ligands' chains first; the plain form
    runs the first --plain-jobs jobs one launch each, and the same jobs are
    also run batched."""
    import torch
    cfg = S.CONFIGS["uneven_batch"]
    rx, rt, bxs = S.make_receptor(cfg)
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=10.0)
    ligs = pv.Ligands(ctx, mols)
    jobs = S.make_jobs(cfg)[:len(mols) * len(bxs)]
    params = pv.dock_params(chains=cfg.chains, steps=cfg.steps, seed=S.philox_seed(cfg),
                            flags=pv.PV_DOCK_GRAPH | pv.PV_DOCK_LARGEST_FIRST)
    plan = pv.Plan(ctx, grids, ligs, jobs, params)
    tuning = tune(plan, stream, steps=10)
    torch.cuda.synchronize()
    ms = _timed(stream, plan.run)
    out = plan.outputs()
    ev = int(out["job_evals"].sum().item())
    N, T, P = _jobs_info(ligs, jobs)
    bnd_j = out["chain_bounded"].cpu().numpy().reshape(len(jobs), -1).sum(axis=1)
    fl = float(flops_of(out["job_evals"].cpu().numpy(), P, N, T).sum())
    fl_done = float(flops_performed(out["job_evals"].cpu().numpy(), bnd_j, P, N, T).sum())
    variant = plan.schedule(0)["variant"]
    output = bench_output(pv, plan, stream)
    plan.close()
    few = jobs[:args.plain_jobs]
    pplan = pv.Plan(ctx, grids, ligs, few, params)
    pplan.run()
    torch.cuda.synchronize()
    ms_same = _timed(stream, pplan.run)
    ms_plain = _timed(stream, lambda: pplan.run(plain=True))
    ev_plain = int(pplan.outputs()["job_evals"].sum().item())
    pplan.close()
    return {
        "workload": "uneven batch: %d ligands of 10..60 atoms / 0..15 torsions x 5 pockets of 24 A (%d jobs), "
                    "32 chains x 500 MC steps per job" % (len(mols), len(jobs)),
        "batched": {"jobs": len(jobs), "docks_per_s": len(jobs) / (ms * 1e-3), "evals_per_s": ev / (ms * 1e-3),
                    "ms": ms, "variant": VARIANTS[variant], "tflops": fl / (ms * 1e-3) / 1e12,
                    "frac_fp32": fl / (ms * 1e-3) / PEAK_FP32_VECTOR,
                    "tflops_work_performed": fl_done / (ms * 1e-3) / 1e12, "autotune": tuning},
        "plain": {"jobs": len(few), "docks_per_s": len(few) / (ms_plain * 1e-3),
                  "evals_per_s": ev_plain / (ms_plain * 1e-3), "ms": ms_plain},
        "batched_same_jobs": {"jobs": len(few), "docks_per_s": len(few) / (ms_same * 1e-3), "ms": ms_same},
        "batched_over_plain": (len(jobs) / ms) / (len(few) / ms_plain),
        "output_stage": output,
    }


def bench_stream_plain(pv, S, ctx, stream, args, inp):
    """Plain against batched on the same jobs of the screening stream: its
    first --stream-plain-jobs jobs, one launch per job in order (the
    per-ligand loop of the paper's engine), then as one batched launch."""
    import torch
    (rx, rt, bxs), mols, jobs = inp
    cfg = S.CONFIGS["screening"]
    few = jobs[:args.stream_plain_jobs]
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=10.0)
    ligs = pv.Ligands(ctx, [mols[i] for i in few[:, 0]])
    jl = np.stack([np.arange(len(few), dtype=np.int32), few[:, 1]], axis=1)
    params = pv.dock_params(chains=cfg.chains, steps=cfg.steps, seed=S.philox_seed(cfg), flags=pv.PV_DOCK_GRAPH)
    plan = pv.Plan(ctx, grids, ligs, jl, params)
    plan.run()
    torch.cuda.synchronize()
    ms = _timed(stream, plan.run)
    ms_plain = _timed(stream, lambda: plan.run(plain=True))
    ev = int(plan.outputs()["job_evals"].sum().item())
    plan.close()
    return {"workload": "screening stream, its first %d jobs" % len(few),
            "batched": {"docks_per_s": len(few) / (ms * 1e-3), "evals_per_s": ev / (ms * 1e-3), "ms": ms},
            "plain": {"docks_per_s": len(few) / (ms_plain * 1e-3), "evals_per_s": ev / (ms_plain * 1e-3),
                      "ms": ms_plain},
            "batched_over_plain_same_jobs": ms_plain / ms}


def bench_box_sweep(pv, S, ctx, stream, args):
    """The box-size sweep: the 5 pockets of the multi-pocket receptor with
    cubic boxes of 15..30 A in 1 A steps (80 boxes) built in one grid-map
    launch, then the 35-atom ligand docked into every box (64 chains x
    --sweep-steps MC steps) as one persistent launch.  Reports the grid build
    rate and the mean best energy per box edge."""
    import torch
    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    edges = list(range(15, 31))
    sweep = S.box_sweep(bxs, edges)
    grids = pv.build_grids(ctx, rx, rt, sweep, penalty_slope=10.0)
    torch.cuda.synchronize()
    grid_ms = min(_timed(stream, grids.rebuild) for _ in range(3))
    points = sum(int(np.prod(grids.info(b)[0])) for b in range(len(sweep)))
    ligs = pv.Ligands(ctx, S.make_ligands(cfg))
    jobs = [(0, b) for b in range(len(sweep))]
    params = pv.dock_params(chains=64, steps=args.sweep_steps, seed=S.philox_seed(cfg), flags=pv.PV_DOCK_GRAPH)
    plan = pv.Plan(ctx, grids, ligs, jobs, params)
    tune(plan, stream)
    plan.run()
    torch.cuda.synchronize()
    ms = _timed(stream, plan.run)
    out = plan.outputs()
    best = out["job_best_e"].cpu().numpy().reshape(len(bxs), len(edges))
    ev = int(out["job_evals"].sum().item())
    plan.close()
    return {
        "workload": "box-size sweep: 5 pockets x edges 15..30 A (80 boxes, %.0f MB of maps); 35-atom ligand, "
                    "64 chains x %d MC steps per box" % (points * 32 / 1e6, args.sweep_steps),
        "grid_ms": grid_ms, "grid_points_per_s": points / (grid_ms * 1e-3),
        "dock_ms": ms, "docks_per_s": len(jobs) / (ms * 1e-3), "evals_per_s": ev / (ms * 1e-3),
        "edges_A": edges, "mean_best_e_by_edge": [float(v) for v in best.mean(axis=0)],
    }


def bench_surface(pv, S, ctx, stream):
    """The step before the path: solvent-accessible surface points of the
    screening receptor (8,000 atoms, 30 directions per atom, 1.6 A probe)
    and their Eq. prank_eq_1 features."""
    import torch
    rx, rt, _ = S.make_receptor(S.CONFIGS["screening"])
    dirs = S.sphere_directions(30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sas = pv.SurfacePoints(ctx, rx, rt, dirs, 1.6)
    build_ms = (time.perf_counter() - t0) * 1e3
    feat = sas.features()
    torch.cuda.synchronize()
    feat_ms = min(_timed(stream, lambda: sas.features(out=feat)) for _ in range(3))
    n = sas.n_points
    sas.close()
    return {"workload": "8,000-atom receptor, 30 directions per atom, probe 1.6 A",
            "candidates": len(rt) * len(dirs), "points": n, "build_ms_host_wall": build_ms,
            "features_ms": feat_ms, "point_atom_pairs_per_s": n * len(rt) / (feat_ms * 1e-3)}


def _oracle_grids(O, rx, rt, bxs, which):
    return {int(b): O.Grid.build(rx, rt, bxs[b].center.astype(np.float64), bxs[b].size.astype(np.float64),
                                 bxs[b].spacing, kappa=10.0) for b in which}


def _oracle_dock(O, mols, grids, jobs, cfg, seed, threads):
    """The oracle's dock of jobs (ligand, box); returns (seconds,
    evaluations)."""
    ligs = {}
    for l in np.unique(jobs[:, 0]):
        m = mols[l]
        ligs[int(l)] = O.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    lk = sorted(ligs)
    gk = sorted(grids)
    oj = [(lk.index(int(l)), gk.index(int(b))) for l, b in jobs]
    P = O.mc_params(cfg.chains, cfg.steps, seed)
    t0 = time.perf_counter()
    res = O.dock([ligs[k] for k in lk], [grids[k] for k in gk], oj, P, n_threads=threads)
    return time.perf_counter() - t0, int(res["chain_evals"].sum())


def cpu_baseline_stream(S, inp, head, args):
    """The FP64 oracle on the host, on the first --cpu-jobs jobs of the
    screening stream (all host cores, OpenMP over chains), and on the first
    job alone on one core; both scaled to docks/s."""
    import oracle as O
    (rx, rt, bxs), mols, jobs = inp
    cfg = S.CONFIGS["screening"]
    seed = S.philox_seed(cfg)
    few = jobs[:args.cpu_jobs]
    grids = _oracle_grids(O, rx, rt, bxs, np.unique(few[:, 1]))
    threads = len(os.sched_getaffinity(0))
    dt, ev = _oracle_dock(O, mols, grids, few, cfg, seed, threads)
    d1, ev1 = _oracle_dock(O, mols, grids, few[:1], cfg, seed, 1)
    return {"value": len(few) / dt, "unit": "docks/s", "cores": threads, "kind": "oracle",
            "sample": "screening stream, its first %d jobs (16 chains x 300 MC steps each), %.1f s wall"
                      % (len(few), dt),
            "evals_per_s": ev / dt, "evals": ev, "cpu": cpu_model(),
            "single_core": {"docks_per_s": 1.0 / d1, "evals_per_s": ev1 / d1,
                            "sample": "the stream's first job on one core, %.1f s" % d1}}


def cpu_oracle_tiny(S, args):
    """The oracle docking the whole tiny configuration on all host cores."""
    import oracle as O
    cfg = S.CONFIGS["tiny"]
    rx, rt, bxs = S.make_receptor(cfg)
    mols = S.make_ligands(cfg)
    grids = _oracle_grids(O, rx, rt, bxs, [0])
    threads = len(os.sched_getaffinity(0))
    dt, ev = _oracle_dock(O, mols, grids, np.array([[0, 0]]), cfg, S.philox_seed(cfg), threads)
    return {"docks_per_s": 1.0 / dt, "evals_per_s": ev / dt, "s": dt, "cores": threads, "sample": "in full"}


def cpu_oracle_batch(S, mols, args):
    """The oracle on the first 16 jobs of the uneven batch (all host cores)."""
    import oracle as O
    cfg = S.CONFIGS["uneven_batch"]
    rx, rt, bxs = S.make_receptor(cfg)
    jobs = S.make_jobs(cfg)[:16]
    grids = _oracle_grids(O, rx, rt, bxs, np.unique(jobs[:, 1]))
    threads = len(os.sched_getaffinity(0))
    dt, ev = _oracle_dock(O, mols, grids, jobs, cfg, S.philox_seed(cfg), threads)
    return {"docks_per_s": len(jobs) / dt, "evals_per_s": ev / dt, "s": dt, "cores": threads,
            "sample": "the first %d jobs of the batch" % len(jobs)}


def measure_peaks(pv, ctx, stream):
    """The device's FP32 multiply-add rate reached by code built here (16
    independent FMA chains per thread, packed FP32 off) and a 256 MiB
    device-to-device copy's bandwidth: measured context for the published
    peaks the roofline is priced at (best of 10 launches each)."""
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    out = torch.empty(n_cu * 2048, dtype=torch.float32, device="cuda")
    iters = 4096
    pv.fma_peak(ctx, iters, out)
    torch.cuda.synchronize()
    best = None
    for _ in range(10):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        flops = pv.fma_peak(ctx, iters, out)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    n = 64 << 20
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    cbest = None
    for _ in range(10):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        cbest = ms if cbest is None else min(cbest, ms)
    return {"fp32_fma_TFLOPs": flops / (best * 1e-3) / 1e12, "fp32_fma_ms": best,
            "published_fp32_vector_TFLOPs": PEAK_FP32_VECTOR / 1e12,
            "copy_GBps": 2 * 4 * n / (cbest * 1e-3) / 1e9, "copy_ms": cbest,
            "published_hbm_GBps": PEAK_HBM / 1e9}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
