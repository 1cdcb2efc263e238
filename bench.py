#!/usr/bin/env python
"""Benchmark of the docking hot path on one MI355X.

One step = one pass of the whole hot path over the multi-pocket workload:
grid maps of 5 pockets rebuilt (the grid-map kernel), then Monte Carlo +
RILC-BFGS docking of one 35-atom, 8-torsion ligand into every pocket, 256
chains x 1,000 MC steps each, as one persistent hipGraph-replayed launch.
Inputs are seeded and synthetic and stay resident in HBM.

Prints one JSON line: docks/s (value), score+grad evaluations/s, the plain
per-job launch path, the roofline of the dominant kernel (measured with HIP
events on the stream the kernels run on) and the oracle timed on the host.
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

# Algorithmic work of one evaluation, counted from the operations the method
# needs, energy part and gradient part: per intra pair tested (difference,
# squared distance); per pair inside the cutoff, the terms (20) and with the
# gradient the derivative and the force on both atoms (16); per atom, the
# frame transform and the trilinear value (48) and with the gradient the
# trilinear gradient and the force/torque accumulation (43); per torsion, the
# local rotation and the frame composition (109) and with the gradient the
# torsion derivative (32); per evaluation the root frame and the BFGS vector
# work.  A line-search trial above the sufficient-decrease bound needs only
# the energy (the kernel stops there), so the gradient part counts once per
# evaluation that computed it.
FLOP_PAIR_TEST = 8
FLOP_PAIR_IN, FLOP_PAIR_IN_GRAD = 20, 16
FLOP_ATOM, FLOP_ATOM_GRAD = 48, 43
FLOP_TORS, FLOP_TORS_GRAD = 109, 32
FLOP_EVAL = 50


def flops_per_launch(n_evals, n_grads, pairs_in, n_atoms, n_tors, n_pairs, m=5):
    energy = FLOP_PAIR_TEST * n_pairs + FLOP_ATOM * n_atoms + FLOP_TORS * n_tors + FLOP_EVAL
    energy += (4 * m + 10) * (6 + n_tors)
    grad = FLOP_ATOM_GRAD * n_atoms + FLOP_TORS_GRAD * n_tors
    # pairs inside the cutoff are counted over all evaluations; their gradient
    # share follows the share of evaluations with a gradient
    share = n_grads / n_evals if n_evals else 0.0
    return (float(n_evals) * energy + float(n_grads) * grad +
            float(pairs_in) * (FLOP_PAIR_IN + share * FLOP_PAIR_IN_GRAD))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chains", type=int, default=256)
    ap.add_argument("--mc-steps", type=int, default=1000)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-score", action="store_true")
    ap.add_argument("--cpu-chains", type=int, default=128)
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the uneven-batch (batched vs plain) and screening-stream legs")
    ap.add_argument("--batch-ligands", type=int, default=256,
                    help="ligands of the uneven batch (x 5 pockets = jobs)")
    ap.add_argument("--plain-jobs", type=int, default=20, help="jobs of the uneven batch run one launch each")
    ap.add_argument("--stream-jobs", type=int, default=2048, help="jobs taken from the screening stream")
    ap.add_argument("--sweep-steps", type=int, default=1000, help="MC steps per chain in the box-size sweep")
    ap.add_argument("--leg", choices=["score", "local_opt", "batching", "screening", "box_sweep", "surface"], default=None,
                    help="run only this secondary leg and print its JSON (for profiling it alone)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (calibrates the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; --gpus %d is not supported "
              "(across GPUs the work would shard by pocket, each GPU building only its pockets' maps)"
              % args.gpus, file=sys.stderr)
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

    import paper_2506_20043_amd as pv
    from paper_2506_20043_amd import synth as S

    if args.leg:
        ctx = pv.Context(0)
        stream = torch.cuda.current_stream()
        legs = {"score": lambda: bench_score(pv, S, ctx, stream),
                "local_opt": lambda: bench_local_opt(pv, S, ctx, stream),
                "batching": lambda: bench_batching(pv, S, ctx, stream, args),
                "screening": lambda: bench_screening(pv, S, ctx, stream, args),
                "box_sweep": lambda: bench_box_sweep(pv, S, ctx, stream, args),
                "surface": lambda: bench_surface(pv, S, ctx, stream)}
        print(json.dumps({"leg": args.leg, "result": legs[args.leg]()}), flush=True)
        return

    cfg = S.CONFIGS["multi_pocket"]
    rx, rt, bxs = S.make_receptor(cfg)
    mols = S.make_ligands(cfg)
    seed = S.philox_seed(cfg)
    ctx = pv.Context(0)
    stream = torch.cuda.current_stream()
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=10.0)
    ligs = pv.Ligands(ctx, mols)
    n_atoms, n_frag, n_tors, n_pairs = ligs.info(0)[:4]
    jobs = [(0, b) for b in range(len(bxs))]
    params = pv.dock_params(chains=args.chains, steps=args.mc_steps, seed=seed,
                            flags=pv.PV_DOCK_GRAPH, workgroups=args.workgroups)
    plan = pv.Plan(ctx, grids, ligs, jobs, params)
    tuning = tune(plan, stream)
    torch.cuda.synchronize()

    def step():
        grids.rebuild()
        plan.run()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        grids.rebuild()
        ev[k][1].record(stream)
        plan.run()
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = plan.outputs()
    n_evals = int(out["job_evals"].sum().item())
    pairs_in = int(out["chain_pairs"].sum().item())
    n_grads = int(out["chain_grads"].sum().item())
    grid_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    dock_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    ms_per_step = wall * 1e3 / args.steps
    docks = len(jobs) * args.steps
    docks_per_s = docks / wall
    evals_per_s = n_evals * args.steps / wall
    flops = flops_per_launch(n_evals, n_grads, pairs_in, n_atoms, n_tors, n_pairs)
    achieved = flops / (dock_ms * 1e-3)
    result = {
        "metric": "ligand-pocket docks/s and score+grad evals/s, batched vs plain on 1 MI355X",
        "value": docks_per_s,
        "unit": "docks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded receptor, pockets and ligand; no datasets)",
        "config": {
            "workload": "multi-pocket single ligand: 5,000-atom receptor in a 50 A cube, 5 pockets of 24 A "
                        "at 0.375 A (65^3 x 8 FP32 maps each), one %d-atom ligand with %d torsions "
                        "(%d intra pairs), %d chains x %d MC steps per pocket, BFGS <= 30 iterations; "
                        "step = grid-map rebuild + batched persistent dock (hipGraph)"
                        % (n_atoms, n_tors, n_pairs, args.chains, args.mc_steps),
            "jobs": len(jobs), "chains": args.chains, "mc_steps": args.mc_steps,
            "parallelism": "single GPU",
        },
        "evals_per_s": evals_per_s,
        "evals_per_step": n_evals,
        "gradient_evals_per_step": n_grads,
        "grid_ms": grid_ms,
        "dock_ms": dock_ms,
        "docks_per_s_without_grid_build": len(jobs) / (dock_ms * 1e-3),
        "workgroups": plan_workgroups(plan),
        "autotune": tuning,
    }
    # plain path: one launch per job, same kernel and draws
    if not args.no_plain:
        plan.run(plain=True)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.run(plain=True)
        b.record(stream)
        torch.cuda.synchronize()
        plain_ms = a.elapsed_time(b)
        result["plain"] = {"docks_per_s": len(jobs) / (plain_ms * 1e-3),
                           "evals_per_s": n_evals / (plain_ms * 1e-3), "dock_ms": plain_ms}
        result["batched_over_plain"] = plain_ms / dock_ms
    result["roofline"] = {
        "bound": "alu",
        "kernel": "dock_kernel (persistent MC + BFGS)",
        "achieved": achieved / 1e12,
        "peak": PEAK_FP32_VECTOR / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_VECTOR,
        "traffic": recorded_traffic(),
        "flops_per_launch": flops,
        "launch_ms": dock_ms,
        # the second ceiling: every evaluation reads 8 corners x 4 B per atom
        # from the maps (L2 / Infinity Cache hits mostly), priced at HBM's peak
        "map_gather": {"bytes_per_launch": MAP_BYTES_PER_ATOM * n_atoms * n_evals,
                       "achieved_GBps": MAP_BYTES_PER_ATOM * n_atoms * n_evals / (dock_ms * 1e-3) / 1e9,
                       "peak_GBps": PEAK_HBM / 1e9,
                       "frac": MAP_BYTES_PER_ATOM * n_atoms * n_evals / (dock_ms * 1e-3) / PEAK_HBM},
    }
    result["output_stage"] = bench_output(pv, plan, stream)
    if not args.no_extra:
        result["consistency_check"] = bench_consistency(pv, ctx, grids, ligs, jobs, args, seed, stream,
                                                        n_evals, dock_ms, plan.outputs())
    if not args.no_score:
        result["score_grad"] = bench_score(pv, S, ctx, stream)
        result["local_opt"] = bench_local_opt(pv, S, ctx, stream)
    if not args.no_extra:
        result["batching"] = bench_batching(pv, S, ctx, stream, args)
        result["screening"] = bench_screening(pv, S, ctx, stream, args)
        result["box_sweep"] = bench_box_sweep(pv, S, ctx, stream, args)
        result["surface"] = bench_surface(pv, S, ctx, stream)
    result["measured_peaks"] = measure_peaks(pv, ctx, stream)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(S, cfg, rx, rt, bxs, mols, seed, args)
    print(json.dumps(result), flush=True)


def recorded_traffic():
    """HBM bytes per dock launch from the committed rocprofv3 counter record,
    or None when the kernel sources changed since the counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "dock_kernel_multipocket.md")
    if not os.path.exists(prof):
        return None
    rec = None
    for line in open(prof):
        if line.startswith("traffic_record: "):
            rec = json.loads(line[len("traffic_record: "):])
    if rec is None:
        return None
    csrc = os.path.join(ROOT, "paper_2506_20043_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("pv_kernels.hip", "pv_internal.h"))
    if hashlib.sha256(src).hexdigest() != rec["kernel_source_sha256"]:
        return None
    return rec["dock_traffic_bytes_per_launch"]


def plan_workgroups(plan):
    return int(plan.params.workgroups) if plan.params.workgroups else None


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


def bench_batching(pv, S, ctx, stream, args):
    """Batched vs plain on the uneven batch: ligands of 10..60 atoms and
    0..15 torsions, each docked into the 5 pockets of the multi-pocket
    receptor, 32 chains x 500 MC steps per job.  The batched form runs the
    first --batch-ligands x 5 jobs as one persistent hipGraph launch, handing
    out the most costly ligands' chains first (PV_DOCK_LARGEST_FIRST); the
    plain form runs the first --plain-jobs jobs one launch each, and the same
    jobs are also run batched."""
    import torch
    cfg = S.CONFIGS["uneven_batch"]
    rx, rt, bxs = S.make_receptor(cfg)
    mols = S.make_ligands(cfg, args.batch_ligands)
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=10.0)
    ligs = pv.Ligands(ctx, mols)
    jobs = S.make_jobs(cfg)[:args.batch_ligands * len(bxs)]
    params = pv.dock_params(chains=cfg.chains, steps=cfg.steps, seed=S.philox_seed(cfg),
                            flags=pv.PV_DOCK_GRAPH | pv.PV_DOCK_LARGEST_FIRST)
    plan = pv.Plan(ctx, grids, ligs, jobs, params)
    tuning = tune(plan, stream, steps=10)
    plan.run()
    torch.cuda.synchronize()
    ms = _timed(stream, plan.run)
    ev = int(plan.outputs()["job_evals"].sum().item())
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
    names = ["slots", "gather", "gather2"]
    return {
        "workload": "uneven batch: ligands of 10..60 atoms / 0..15 torsions x 5 pockets of 24 A, "
                    "32 chains x 500 MC steps per job",
        "batched": {"jobs": len(jobs), "docks_per_s": len(jobs) / (ms * 1e-3), "evals_per_s": ev / (ms * 1e-3),
                    "ms": ms, "variant": names[variant], "autotune": tuning},
        "plain": {"jobs": len(few), "docks_per_s": len(few) / (ms_plain * 1e-3),
                  "evals_per_s": ev_plain / (ms_plain * 1e-3), "ms": ms_plain},
        "batched_same_jobs": {"jobs": len(few), "docks_per_s": len(few) / (ms_same * 1e-3), "ms": ms_same},
        "batched_over_plain": (len(jobs) / ms) / (len(few) / ms_plain),
        "output_stage": output,
    }


def bench_screening(pv, S, ctx, stream, args):
    """The screening stream: an 8,000-atom receptor with 16 pockets of
    20..30 A (all maps resident), ligands of 8..80 atoms / 0..20 torsions,
    16 chains x 300 MC steps per job, jobs in the stream's seeded order.  The
    first --stream-jobs jobs run as one persistent launch with per-job device
    timestamps: service time = last chain done - first chain dequeued."""
    import torch
    cfg = S.CONFIGS["screening"]
    rx, rt, bxs = S.make_receptor(cfg)
    jobs = S.make_jobs(cfg)[:args.stream_jobs]
    uniq, local = np.unique(jobs[:, 0], return_inverse=True)
    mols = [S.make_ligands(cfg, 1, int(i))[0] for i in uniq]
    grids = pv.build_grids(ctx, rx, rt, bxs, penalty_slope=10.0)
    torch.cuda.synchronize()
    grid_ms = _timed(stream, grids.rebuild)
    ligs = pv.Ligands(ctx, mols)
    jl = np.stack([local.astype(np.int32), jobs[:, 1]], axis=1)
    params = pv.dock_params(chains=cfg.chains, steps=cfg.steps, seed=S.philox_seed(cfg),
                            flags=pv.PV_DOCK_GRAPH | pv.PV_DOCK_TIMESTAMPS)
    plan = pv.Plan(ctx, grids, ligs, jl, params)
    tuning = tune(plan, stream, steps=10)
    plan.run()
    torch.cuda.synchronize()
    ms = _timed(stream, plan.run)
    out = plan.outputs()
    t0 = out["job_t_start"].cpu().numpy().astype(np.int64)
    t1 = out["job_t_end"].cpu().numpy().astype(np.int64)
    ev = int(out["job_evals"].sum().item())
    plan.close()
    svc = (t1 - t0) / 100.0          # device clock ticks at 100 MHz -> us
    span = (t1.max() - t0.min()) / 100.0
    map_mb = sum(8 * int(np.prod(grids.info(b)[0])) * 4 for b in range(len(bxs))) / 1e6
    return {
        "workload": "screening stream: 8,000-atom receptor, 16 pockets of 20..30 A (%.0f MB of maps), "
                    "ligands of 8..80 atoms / 0..20 torsions, 16 chains x 300 MC steps, first %d jobs "
                    "of the seeded order" % (map_mb, len(jobs)),
        "jobs": len(jobs), "ms": ms, "docks_per_s": len(jobs) / (ms * 1e-3), "evals_per_s": ev / (ms * 1e-3),
        "service_us_p50": float(np.percentile(svc, 50)), "service_us_p99": float(np.percentile(svc, 99)),
        "service_us_max": float(svc.max()), "makespan_us": float(span), "grid_build_ms_16_pockets": grid_ms,
        "autotune": tuning,
    }


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


def cpu_baseline(S, cfg, rx, rt, bxs, mols, seed, args):
    """The FP64 oracle on the host: a bounded sample of the same dock (the
    first --cpu-chains chains of pocket 0, all MC steps), scaled to docks/s."""
    import oracle as O
    b = bxs[0]
    G = O.Grid.build(rx, rt, b.center.astype(np.float64), b.size.astype(np.float64), b.spacing, kappa=10.0)
    m = mols[0]
    L = O.Ligand(m.xyz, m.types, m.bonds, m.rotatable)
    P = O.mc_params(args.cpu_chains, args.mc_steps, seed)
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    res = O.dock([L], [G], [(0, 0)], P, n_threads=threads)
    dt = time.perf_counter() - t0
    evals = int(res["chain_evals"].sum())
    frac = args.cpu_chains / args.chains
    # one core: the first 4 chains of the same sample
    P1 = O.mc_params(4, args.mc_steps, seed)
    t1 = time.perf_counter()
    r1 = O.dock([L], [G], [(0, 0)], P1, n_threads=1)
    d1 = time.perf_counter() - t1
    return {"value": frac / dt, "unit": "docks/s", "cores": threads, "kind": "oracle",
            "sample": "pocket 0, %d of %d chains x %d MC steps (%.3f of one dock), %.1f s wall"
                      % (args.cpu_chains, args.chains, args.mc_steps, frac, dt),
            "evals_per_s": evals / dt, "cpu": cpu_model(),
            "single_core": {"evals_per_s": int(r1["chain_evals"].sum()) / d1,
                            "docks_per_s": (4 / args.chains) / d1,
                            "sample": "pocket 0, 4 chains x %d MC steps, %.1f s" % (args.mc_steps, d1)}}


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
