#!/usr/bin/env python
"""Throughput of the particle hot path on one MI355X.

Workload (default, --workload shear3d): the 3D3V shearing box, 256^3 Yee cells, 8 particles
per cell per species (e+ and e-, 268,435,456 particles), Maxwell-Juttner theta = 0.3, skin depth
4 cells, weak B0 along z with sigma = 0.05, Keplerian shear q = 1.5, Omega0/omega_c = 0.05,
dt = 0.45, FP32 particles (int32 cell + FP32 offset) with FP64 shear offset.  Synthetic seeded
inputs.  --workload expand3d / leaky2d: the 128x128x512 expanding box and the 2048^2 leaky box
(recipes in paper_2602_15939_amd/workloads.py); the full default run (no --workload, CPU baseline
on) also times these two after the shearing box, and a 128-run sample of the served batch, and
reports them under "other_workloads"; --serve: the served batch of 2D boxes.

One step = tile sort + fused gather/push/deposit + current fold with the J' transport +
implicit-midpoint Maxwell (fixed-point sweeps) + guard fills, i.e. the whole hot path.
value = particles x steps / wall time of the timed steps (particle-steps/s).
The fused push kernel is timed with HIP events on the box stream for the roofline line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
COPY_CAL_BYTES = 1 << 30  # plain device copy used to calibrate the FETCH/WRITE counters
DR_COMPONENTS = 2  # displacement components the fused kernel reads and writes (in-plane test)
GPD_SOURCES = ("paper_2602_15939_amd/csrc/gpd.hip", "paper_2602_15939_amd/csrc/pic_internal.h")


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in GPD_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3 counter record,
    only if it was taken on the current kernel source and workload; else None."""
    path = os.path.join(ROOT, "profiles", "gpd_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("workload") != workload:
        return None
    return rec.get("traffic_bytes_per_launch")


def workload_shear3d(n=256, ppc=8):
    from paper_2602_15939_amd import workloads

    return workloads.shear3d(n, ppc)


def make_box(w, seed, device="cuda"):
    from paper_2602_15939_amd import workloads

    return workloads.make_box(w, seed, device=device)


def algorithmic_bytes(w, nparticles):
    """Bytes the method must move per launch of the fused gather/push/deposit: the particle
    state read and written (int32 cell + dim FP32 offsets + 3 FP32 momenta: 28 B each way in
    3D, 24 B in 2D), the leaky box's particle id read for its Philox counter (4 B) and, in the
    displacement mode, the tracked in-plane displacement read and written (2 x 8 B); per cell
    the six field components read once (24 B) and the current read and written (24 B)."""
    ncell = math.prod(w["n"])
    per = 2 * (4 + 4 * w["dim"] + 12)
    if w["kind"] == "leaky":
        per += 4
    if w.get("escape") == "displacement":
        per += 2 * 4 * DR_COMPONENTS  # the tracked displacement of the escape test (Sec. 4.1)
    return nparticles * per + ncell * (24 + 24)


def implementation_bytes(w, nparticles):
    """Traffic of this implementation beyond the algorithmic bytes, per launch: the read of the
    sort permutation (4 B per particle), and the particle id written in sorted order where ids
    are carried (4 B)."""
    return nparticles * (4 + (4 if w["kind"] == "leaky" else 0))


def one_step_plain(L, h):
    """One untimed step: sort, fused push, current fold, Maxwell."""
    L.pic_tile_sort(h)
    L.pic_gather_push(h, L.FUSE_DEPOSIT)
    L.pic_shear_remap(h, L.REMAP_CURRENT)
    L.pic_maxwell_step(h)


def frame_params(w):
    """The physical parameters of a workload for the bench line."""
    import math as m

    wp = 0.25  # skin depth 4 cells
    sigma = round((w["B0"] / wp) ** 2, 6)
    p = dict(theta=w["theta"], sigma=sigma, dt=w["dt"])
    if w["kind"] == "shear":
        p.update(q=w["shear_s"], omega0_over_wc=round(w["omega0"] / w["B0"], 6),
                 maxwell_iters=w["maxwell_iters"])
    elif w["kind"] == "expand":
        p.update(adot_over_wp=round(w["adot"] / wp, 9), dB_over_B0=w["dB"], spectrum_slope_3d=-5 / 3)
    elif w.get("escape") == "displacement":
        p.update(dB_over_B0=w["dB"], l_esc=w["l_esc"], theta_inj=w["theta"],
                 escape="displacement (Sec. 4.1), Maxwell-Juttner re-draw in place")
    else:
        p.update(dB_over_B0=w["dB"], gamma_thr=w["gamma_thr"], t_esc_over_L=w["t_esc"] / w["n"][0],
                 escape="probabilistic, Philox keyed by id and step")
        if "shell_gamma" in w:
            p.update(shell_gamma=w["shell_gamma"], t_esc_over_dt=w["t_esc"] / w["dt"])
    return p


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(seconds=12.0, n=64, w=None, steps=None):
    """The FP64 oracle, unchanged, on the host cores: an n^3 sample of the 3D shearing-box
    workload (same ppc, theta, sigma, shear), or the workload w itself when given, one untimed
    step, then timed steps until ~seconds have elapsed (at least 3), or exactly `steps`."""
    import numpy as np

    import oracle
    from paper_2602_15939_amd import synth

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    sample = w is None
    if sample:
        w = workload_shear3d(n=n)
    dim = w["dim"]
    parts = synth.pair_plasma(w["n"], w["ppc"], w["theta"], 99, device="cpu")
    box = oracle.make_box(dim, w["n"], dt=w["dt"], frame=oracle.SHEAR, shear_s=w["shear_s"],
                          omega0=w["omega0"], maxwell_iters=w["maxwell_iters"])
    E, B = synth.uniform_field(w["n"], 2, w["B0"])
    J = np.zeros_like(E)
    sp = []
    for s, p in enumerate(parts):
        c = p["cell"].numpy().astype(np.int64)
        off = p["off"].numpy().astype(np.float64)
        n = w["n"]
        x = c % n[0] + off[0]
        y = (c // n[0]) % n[1] + off[1]
        z = c // (n[0] * n[1]) + off[2] if dim == 3 else None
        u = p["u"].numpy().astype(np.float64)
        qm = (-1.0, 1.0)[s]
        sp.append(oracle.SpeciesState(x, y, z, u[0], u[1], u[2], qm, qm * w["q"]))
    npart = sum(len(s.x) for s in sp)
    oracle.step(box, E, B, J, sp, nthreads=cores)  # warm-up (page faults of the buffers)
    done, t0 = 0, time.perf_counter()
    while True:
        oracle.step(box, E, B, J, sp, nthreads=cores)
        done += 1
        el = time.perf_counter() - t0
        if steps is not None:
            if done >= steps:
                break
        elif (el > seconds and done >= 3) or done >= 200:
            break
    what = (f"{w['n'][0]}^3 shearing box of the same recipe, {w['ppc']} ppc/species" if sample
            else f"the same {w['name']} box, {w['ppc']} ppc/species")
    return dict(value=npart * done / el, unit="particle-steps/s", cores=cores, kind="oracle",
                cpu_model=cpu_model(), threads=cores,
                sample=f"{what} ({npart} particles), 1 untimed + {done} timed full steps in "
                       f"{el:.1f} s, OpenMP over particles")


def serve_bench(args, runs=None, run_steps=None, baseline_runs=None):
    """The served batch: 512 independent 2D box runs of 500 steps (see serve.py for the
    recipe; runs / run_steps / baseline_runs override the command line for a smaller sample).  (1) capacity: all runs queued at t = 0, admitted by HBM footprint, stepped together
    by the batched step, eagerly and replayed as HIP graphs (the faster mode serves the rest);
    (2) Poisson arrivals at 0.8 x capacity: p50/p99 run latency and aggregate particle-steps/s;
    (3) one box at a time (per-box launches) on the first runs of the same list; (4) runs sampled
    from the mix re-run alone: final energies within 1%."""
    import numpy as np
    import torch

    from paper_2602_15939_amd import serve

    runs = args.runs if runs is None else runs
    run_steps = args.run_steps if run_steps is None else run_steps
    baseline_runs = args.baseline_runs if baseline_runs is None else baseline_runs
    budget = int(args.budget_gb * 2**30)
    tiles = serve.tune_tiles(log=lambda m: print(m, file=sys.stderr, flush=True))
    # warm-up (module loads, allocator pools): a few runs each way, not timed
    warm = serve.make_specs(6, 5, seed=1)
    serve.serve(warm, budget, batched=True)
    serve.serve(warm, budget, batched=True, graph=True)
    serve.serve(warm[:2], 0, batched=False)
    specs = serve.make_specs(runs, run_steps)
    print(f"[serve] capacity run: {len(specs)} runs queued at t=0", file=sys.stderr, flush=True)
    res, wall = serve.serve(specs, budget, batched=True)
    cap_eager = serve.summarize(res, wall)
    print("[serve] capacity run, batched step replayed as HIP graphs", file=sys.stderr, flush=True)
    res, wall = serve.serve(serve.make_specs(runs, run_steps), budget, batched=True, graph=True)
    cap_graph = serve.summarize(res, wall)
    graph = cap_graph["particle_steps_per_s"] > cap_eager["particle_steps_per_s"]
    cap = cap_graph if graph else cap_eager
    rate = 0.8 * cap["runs_per_s"]
    specs = serve.poisson_arrivals(serve.make_specs(runs, run_steps), rate)
    print(f"[serve] Poisson run at {rate:.2f} runs/s (graph={graph})", file=sys.stderr, flush=True)
    res, wall = serve.serve(specs, budget, batched=True, keep_energies=True, graph=graph)
    mix = serve.summarize(res, wall)
    base_specs = serve.make_specs(runs, run_steps)[: baseline_runs]
    print(f"[serve] one box at a time: {len(base_specs)} runs", file=sys.stderr, flush=True)
    bres, bwall = serve.serve(base_specs, 0, batched=False)
    base = serve.summarize(bres, bwall)
    # consistency: sampled runs alone vs in the mix
    rng = np.random.default_rng(3)
    by_id = {r.spec.rid: r for r in res}
    sample = [by_id[int(i)] for i in rng.choice(sorted(by_id), size=min(16, len(by_id)), replace=False)]
    worst = 0.0
    for r in sample:
        sp = serve.RunSpec(**{k: getattr(r.spec, k) for k in ("rid", "n", "ppc", "kind", "theta",
                                                                "param", "steps", "seed")})
        alone, _ = serve.serve([sp], 0, batched=False, keep_energies=True)
        ef_m, ek_m, n_m = r.energies
        ef_a, ek_a, n_a = alone[0].energies
        worst = max(worst, abs(ef_m - ef_a) / abs(ef_a), abs(ek_m - ek_a) / abs(ek_a))
        assert n_m == n_a, (r.spec.rid, n_m, n_a)
    torch.cuda.synchronize()
    out = {
        "metric": "served batch: aggregate particle-steps/s (batched) & p50/p99 run latency",
        "value": mix["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": run_steps,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"served_2d_{runs}runs_{run_steps}steps",
                   "runs": runs, "steps_per_run": run_steps,
                   "budget_gb": args.budget_gb, "arrival_rate_runs_per_s": rate,
                   "tiles": {f"{n}^2 ppc{serve.PPC_CLASSES[k][0]}-{serve.PPC_CLASSES[k][1]}":
                             "x".join(map(str, t[:2])) for (n, k), t in sorted(tiles.items())},
                   "capacity": cap, "capacity_eager_batched": cap_eager,
                   "capacity_graph_batched": cap_graph, "graph": graph,
                   "poisson": mix, "one_at_a_time": base,
                   "batched_over_one_at_a_time": mix["particle_steps_per_s"] / base["particle_steps_per_s"],
                   "capacity_over_one_at_a_time": cap["particle_steps_per_s"] / base["particle_steps_per_s"],
                   "alone_vs_mix_max_rel_energy_diff": worst, "alone_vs_mix_runs": len(sample)},
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None,
                    choices=["shear3d", "shear2d_parity", "expand3d", "leaky2d", "leaky2d_stress",
                             "leaky2d_paper", "leaky2d_paper_stress"],
                    help="shear3d: 256^3 shearing box (the default line); shear2d_parity: the "
                         "64^2 parity configuration (time it over 200 steps: the oracle runs "
                         "the same steps beside it); expand3d: 128x128x512 "
                         "expanding box; leaky2d: 2048^2 leaky box (probabilistic escape); "
                         "leaky2d_paper: the same box with the displacement escape of the paper; "
                         "*_stress: the escape path under load.  Without it: shear3d, and in "
                         "the full default run (with the CPU baseline) also expand3d and leaky2d")
    ap.add_argument("--n", type=int, default=None, help="shear3d only: cells per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="default run only: skip timing the expanding and leaky boxes after it")
    ap.add_argument("--seed", type=int, default=20260216)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration for profiles)")
    ap.add_argument("--settle", type=int, default=30,
                    help="untimed steps before the tile autotuner and the warmup")
    ap.add_argument("--serial-sort", action="store_true",
                    help="queue the tile sort on the box stream before each push instead of "
                         "overlapping it with the current fold and the Maxwell step")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shape instead of pic_autotune's choice")
    ap.add_argument("--serve", action="store_true",
                    help="the served batch of independent 2D boxes instead of the 3D box")
    ap.add_argument("--runs", type=int, default=512)
    ap.add_argument("--run-steps", type=int, default=500)
    ap.add_argument("--baseline-runs", type=int, default=512)
    ap.add_argument("--budget-gb", type=float, default=160.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: every box of this library lives on a single MI355X; "
              "--gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        print(json.dumps(serve_bench(args)), flush=True)
        return
    from paper_2602_15939_amd import workloads

    full = args.workload is None and args.n is None and not args.no_cpu_baseline
    if args.workload in (None, "shear3d"):
        w = workload_shear3d(n=args.n or 256)
    else:
        w = workloads.WORKLOADS[args.workload]()
    out = measure(args, w)
    if full and not args.no_other_workloads:
        # the full default run: the paper's other two frames at their benchmark sizes, timed in
        # the same process after the line's workload (their lines alone: --workload expand3d /
        # leaky2d); the profiling runs (--no-cpu-baseline) time the shearing box only
        out["other_workloads"] = []
        for name in ("expand3d", "leaky2d"):
            o = measure(args, workloads.WORKLOADS[name]())
            out["other_workloads"].append({
                "workload": o["config"]["workload"], "value": o["value"], "unit": o["unit"],
                "ms_per_step": o["ms_per_step"], "steps": o["steps"],
                "particles": o["config"]["particles"], "gpd_ms": o["config"]["gpd_ms"],
                "roofline_frac": o["roofline"]["frac"], "autotune_tile": (o["config"]["autotune"] or {}).get("tile")})
        # a sample of the served batch (its full line: --serve): 128 runs of 250 steps, the
        # one-box-at-a-time baseline over all of them
        o = serve_bench(args, runs=128, run_steps=250, baseline_runs=128)
        c = o["config"]
        out["other_workloads"].append({
            "workload": c["workload"], "value": o["value"], "unit": o["unit"],
            "metric": o["metric"], "p50_latency_s": c["poisson"]["p50_latency_s"],
            "p99_latency_s": c["poisson"]["p99_latency_s"], "capacity": c["capacity"]["particle_steps_per_s"],
            "graph": c["graph"], "one_at_a_time": c["one_at_a_time"]["particle_steps_per_s"],
            "batched_over_one_at_a_time": c["batched_over_one_at_a_time"],
            "capacity_over_one_at_a_time": c["capacity_over_one_at_a_time"],
            "alone_vs_mix_max_rel_energy_diff": c["alone_vs_mix_max_rel_energy_diff"]})
    if not args.no_cpu_baseline and w["kind"] == "shear":  # the oracle sample is a shearing box
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        if w["dim"] == 2:  # the small parity box: the oracle runs the timed steps in full
            out["cpu_baseline"] = cpu_baseline(w=w, steps=args.steps)
        else:
            out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def measure(args, w):
    """Build the workload's box on the GPU, settle, optionally autotune, time args.steps steps;
    the bench line of that workload (without the CPU baseline)."""
    import torch

    from paper_2602_15939_amd import _lib as L

    print(f"[bench] building {w['name']}", file=sys.stderr, flush=True)
    graph_steps = w["dim"] == 2 and w["kind"] == "shear"
    if graph_steps:  # a captured graph needs a stream other than the legacy default one
        torch.cuda.set_stream(torch.cuda.Stream())
    box, npart = make_box(w, args.seed)
    h = [box.h]
    st = torch.cuda.current_stream()
    tuned = None
    # the kernel's speed depends on how the particles of a tile are ordered in memory: the
    # loader's cell-by-cell order is not the order the step keeps (particles moving inside a
    # tile keep their slots, arrivals are appended), so the tile shape is chosen and the steps
    # are timed after the order has settled
    for _ in range(args.settle):
        one_step_plain(L, h)
    if not args.no_autotune:
        tile, ms = box.autotune(trials=2)
        tuned = {"tile": list(tile), "fused_kernel_ms": {"x".join(map(str, k)): v for k, v in ms.items()}}
        print(f"[bench] autotuned tile {tile}: {tuned['fused_kernel_ms']}", file=sys.stderr, flush=True)

    # one step: the push (through the sort of the previous step), then the sort for the next
    # step on the box's second stream, overlapping the current fold and the Maxwell step
    def one_step(ev=None):
        if args.serial_sort:
            L.pic_tile_sort(h)
        if ev is not None:
            ev[0].record(st)
        L.pic_gather_push(h, L.FUSE_DEPOSIT)
        if ev is not None:
            ev[1].record(st)
        if not args.serial_sort:
            L.pic_tile_sort(h, L.SORT_OVERLAP)
        L.pic_shear_remap(h, L.REMAP_CURRENT)
        L.pic_maxwell_step(h)  # also fills the field guard cells at t^{n+1}

    if not args.serial_sort:
        L.pic_tile_sort(h)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done, timing {args.steps} steps", file=sys.stderr, flush=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    live0 = box.count(0) + box.count(1)
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(evs[k])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpd_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    graph_el = None
    if graph_steps:
        # the small parity box is bound by launches: the same steps replayed as one captured
        # HIP graph per step (the batched step of one box), the way such a box is run
        from paper_2602_15939_amd.box import step_many

        for _ in range(3):
            step_many([box], batched=True, graph=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step_many([box], batched=True, graph=True)
        torch.cuda.synchronize()
        graph_el = time.perf_counter() - t1
    if args.copy_calibration:
        src = torch.empty(COPY_CAL_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        L.pic_device_copy(dst.data_ptr(), src.data_ptr(), COPY_CAL_BYTES, st.cuda_stream)
        torch.cuda.synchronize()
        del src, dst
    info = box.info()
    assert info.errors & ~L.DERR_ORDER == 0, f"device error bits {info.errors}"
    # particle-steps of the timed steps: with escapes the live count decays geometrically
    # (a constant escape probability per step) from live0 to live1
    live1 = int(info.n_particles[0] + info.n_particles[1])
    if live1 < live0:
        r = (live1 / live0) ** (1.0 / args.steps)
        psteps = live0 * (1.0 - r ** args.steps) / (1.0 - r)
    else:
        psteps = float(live0 * args.steps)
    eager_el = el
    if graph_el is not None and graph_el < el:
        el = graph_el
    value = psteps / el
    n_avg = psteps / args.steps  # live particles per timed step (npart without escapes)
    nbytes = algorithmic_bytes(w, n_avg)
    ibytes = implementation_bytes(w, n_avg)
    achieved = nbytes / (gpd_ms * 1e-3) / 1e9
    traffic = measured_traffic(w["name"])
    out = {
        "metric": "particle-steps/s (gather+push+deposit) & HBM %peak",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "particles": npart,
                   "live_particles_first_last": [live0, live1],
                   "frame": {"shear": "shearing box", "expand": "expanding box",
                             "leaky": "leaky box"}[w["kind"]],
                   **frame_params(w),
                   "gpd_ms": gpd_ms, "gpd_particle_steps_per_s": n_avg / (gpd_ms * 1e-3),
                   "gpd_algorithmic_bytes": nbytes, "gpd_implementation_bytes": ibytes,
                   "slow_path_particles": int(info.n_slow),
                   "kernel_source_hash": kernel_source_hash(), "settle_steps": args.settle,
                   "sort": "serial" if args.serial_sort else "overlapped",
                   "step_mode": "graph replay" if el is not eager_el else "eager",
                   "eager_ms_per_step": eager_el * 1e3 / args.steps,
                   "graph_ms_per_step": None if graph_el is None else graph_el * 1e3 / args.steps,
                   "autotune": tuned},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
    }
    box.close()
    del box
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
