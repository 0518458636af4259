"""Throughput of the MMAS hot path on one MI355X.

One step is one iteration of Alg. 1 on the n = 1002 clustered workload
(1002 ants, candidate lists of 32, alpha 1, beta 2, rho 0.02): choice_info
(folded into the previous update), tour construction for every ant, iteration
and global best with the trail limits, evaporation + deposit + clamp. The
metric is tours constructed per second; inputs are resident in HBM before the
timed region starts.

Prints one JSON line with, besides the contract fields, the roofline of the
construction kernel (algorithmic bytes per launch / its average duration,
measured with HIP events on the library's stream) and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_clustered1002.json")


def construct_source_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("construct.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2003_11902_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per construction launch from the committed counter record, or
    None when there is none for this workload or the kernel source changed
    since the counters were taken."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("source_sha256") != construct_source_sha256():
        return None
    return rec.get("construct_hbm_bytes")


def algorithmic_bytes(n: int, cl: int, ants: int, fallback_nodes: float) -> float:
    """Bytes one construction launch must move: per step the candidate row
    (cl ids of 2 B and cl choice_info values of 4 B), per tour the tour itself
    (2 B per city) and its edge lengths (4 B per city), and 4 B of
    choice_info per city enumerated in the all-node fallback."""
    per_tour = (n - 1) * cl * 6 + 2 * n + 4 * n
    return ants * per_tour + 4.0 * fallback_nodes


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_bandwidth_gbs(torch, mib: int = 1024, reps: int = 10) -> float:
    """Measured device-to-device copy rate (read + write bytes per second) of
    a plain torch copy, as a practical ceiling beside the published peak."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    return 2.0 * (mib << 20) / sec / 1e9


def cpu_baseline(dist, w, seed, budget_s):
    from oracle import oracle as O

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 16))
    o = O.Colony(dist, w["ants"], cand_len=w["cand_len"], alpha=w["alpha"], beta=w["beta"],
                 rho=w["rho"], seed=seed, problem=w.get("problem", "tsp"))
    t0 = time.perf_counter()
    it = 0
    while True:
        o.iterate(it, threads)
        it += 1
        el = time.perf_counter() - t0
        if el >= budget_s or it >= 200:
            break
    # and one thread, as the paper's CPU runs: a few iterations of a fresh colony
    o1 = O.Colony(dist, w["ants"], cand_len=w["cand_len"], alpha=w["alpha"], beta=w["beta"],
                  rho=w["rho"], seed=seed, problem=w.get("problem", "tsp"))
    t1 = time.perf_counter()
    it1 = 0
    while True:
        o1.iterate(it1, 1)
        it1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= budget_s / 3 or it1 >= 50:
            break
    return {"value": w["ants"] * it / el, "unit": "tours/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{it} full iterations (choice, construction of {w['ants']} tours, update) of the same "
                      f"workload, OpenMP over ants, {el:.1f} s",
            "value_1_core": w["ants"] * it1 / el1,
            "sample_1_core": f"{it1} iterations of a fresh colony on one thread, {el1:.1f} s"}


def run_batched(args):
    """Many instances per step (mmas_batch_*): autotuned launch shape, one
    captured graph per step."""
    import torch

    from paper_2003_11902_amd import instances as I
    from paper_2003_11902_amd import mmas as M

    t0 = time.perf_counter()
    if args.batch_of:
        # K colonies of one named workload, seeds 1..K (the same instance)
        _, d0, w = I.workload_instance(args.batch_of)
        dists = [d0] * args.batch_count
        params = [M.make_params(w["n"], w["ants"], cand_len=w["cand_len"], alpha=w["alpha"], beta=w["beta"],
                                rho=w["rho"], seed=1 + k, tabu=args.tabu, pher=w["pher"], problem=w["problem"])
                  for k in range(args.batch_count)]
        workload = f"{args.batch_of} x {args.batch_count} colonies"
    else:
        insts = I.batch_instances(args.batch_count)
        dists = [d for _, d in insts]
        params = [M.make_params(d.shape[0], d.shape[0], cand_len=32, rho=0.02, seed=1 + k, tabu=args.tabu)
                  for k, d in enumerate(dists)]
        workload = f"batched{args.batch_count}"
    b = M.Batch(dists, params)
    setup_s = time.perf_counter() - t0
    apb, tb, lanes, tuned_tabu = b.tune()
    if not args.no_graph:
        b.capture()
    for _ in range(args.warmup):
        b.step()
    b.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        b.step()
    b.synchronize()
    elapsed = time.perf_counter() - t1
    print(f"[bench] batched: set-up {setup_s:.1f} s, {args.steps} steps in {elapsed:.3f} s", file=sys.stderr,
          flush=True)
    total_ants = sum(int(p.ants) for p in params)
    # algorithmic bytes of one construction step over all instances, with the
    # fallback enumeration counts of the last step
    nbytes = 0.0
    for k, (d, p) in enumerate(zip(dists, params)):
        n = d.shape[0]
        fb = b.instance(k).fallback()[1].sum()
        nbytes += algorithmic_bytes(n, min(int(p.cand_len), n - 1), int(p.ants), float(fb))
    ms = elapsed / args.steps * 1e3
    achieved = nbytes / (ms * 1e-3) / 1e9
    out = {
        "metric": ("tours constructed/sec, batched instances (1 GPU)" if not args.batch_of
                   else f"tours constructed/sec at n={dists[0].shape[0]}, {args.batch_count} colonies batched (1 GPU)"),
        "value": total_ants * args.steps / elapsed, "unit": "tours/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "instances": args.batch_count,
                   "n_range": [int(min(d.shape[0] for d in dists)), int(max(d.shape[0] for d in dists))],
                   "ants": "n per instance" if not args.batch_of else int(params[0].ants),
                   "cand_len": int(params[0].cand_len), "rho": float(params[0].rho),
                   "tabu": {0: "bitmask", 1: "compact", 2: "list"}[tuned_tabu], "graph": not args.no_graph, "ants_per_block": apb, "table_bytes": tb, "lanes_per_ant": lanes,
                   "total_ants": total_ants},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole step (construction + update)", "bytes_per_step": nbytes},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="clustered1002")
    ap.add_argument("--tabu", default="bitmask", choices=["bitmask", "compact", "list"])
    ap.add_argument("--select", default="wrs", choices=["wrs", "prwm"],
                    help="node selection: weighted reservoir sampling or the parallel roulette wheel")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--ants", type=int, default=0, help="override the workload's ant count")
    ap.add_argument("--ants-per-block", type=int, default=0)
    ap.add_argument("--table-rows", type=int, default=-1)
    ap.add_argument("--lanes-per-ant", type=int, default=64, choices=(32, 64))
    ap.add_argument("--cand-len", type=int, default=None,
                    help="override the workload's candidate-list length (0: no list, every step is a fallback)")
    ap.add_argument("--waves-per-ant", type=int, default=0, choices=(0, 1, 2, 4, 8, 16),
                    help="construction waves per ant (0: from the ant count)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="time the batched workload (256 instances, n in [100, 2000], ants = n) "
                         "instead of the single colony")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-of", default=None,
                    help="with --batched: that many colonies of this named workload (seeds 1..K) instead of "
                         "the mixed 256-instance batch")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (3 times) and exit; "
                         "its FETCH_SIZE / WRITE_SIZE calibrate the HBM traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the method's "
              "multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2003_11902_amd import instances as I
    from paper_2003_11902_amd import mmas as M

    torch.cuda.set_device(0)
    if args.calibrate_copy_mib:
        src = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": src.numel() * 4}), flush=True)
        return
    if args.batched:
        return run_batched(args)
    xy, dist, w = I.workload_instance(args.workload)
    if args.ants:
        w["ants"] = args.ants
    if args.cand_len is not None:
        w["cand_len"] = args.cand_len
    n = w["n"]
    col = M.Colony(dist, w["ants"], cand_len=w["cand_len"], alpha=w["alpha"], beta=w["beta"],
                   rho=w["rho"], seed=args.seed, tabu=args.tabu, pher=w["pher"], ls_nn=w["ls_nn"],
                   problem=w["problem"])
    col.set_launch(args.ants_per_block, args.table_rows, args.lanes_per_ant, args.waves_per_ant)
    if args.select != "wrs":
        col.set_selection(args.select)
    stream = col.stream

    def step(it):
        col.prepare_choice_info()
        col.construct(it)
        if w["ls_nn"]:
            col.two_opt()
        col.update_pheromone()

    it = 0
    for _ in range(args.warmup):
        step(it)
        it += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(it)
        it += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    # per-kernel pass: HIP events around the construction launch on its stream
    kp = min(args.steps, 50)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(kp)]
    fb_nodes, fb_steps, curve = [], [], []
    for k in range(kp):
        col.prepare_choice_info()
        ev[k][0].record(stream)
        col.construct(it)
        ev[k][1].record(stream)
        col.update_pheromone()
        fbs, fbn = col.fallback()
        fb_nodes.append(int(fbn.sum()))
        fb_steps.append(int(fbs.sum()))
        st = col.state()
        curve.append([it, int(st.ib_len), int(st.gb_len)])
        it += 1
    torch.cuda.synchronize()
    cons_all = [a.elapsed_time(b) for a, b in ev]
    cons_ms = float(np.mean(cons_all))
    cons_median_ms = float(np.median(cons_all))
    copy_gbs = copy_bandwidth_gbs(torch)
    nbytes = algorithmic_bytes(n, col.cl, w["ants"], float(np.mean(fb_nodes)))
    achieved = nbytes / (cons_ms * 1e-3) / 1e9

    tours_per_s = w["ants"] * args.steps / elapsed
    out = {
        "metric": f"tours constructed/sec at n={n}" + (" with 2-opt on every tour" if w["ls_nn"] else "") + " (1 GPU)",
        "value": tours_per_s,
        "unit": "tours/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "ants": w["ants"], "cand_len": w["cand_len"],
                   "alpha": w["alpha"], "beta": w["beta"], "rho": w["rho"], "tabu": args.tabu, "select": args.select,
                   "pheromone": w["pher"], "problem": w["problem"],
                   "instance": f"{w['kind']} seed {w['seed']}"
                               + (f", one-way surcharges up to {w['asym']:.0%}" if w.get("asym") else ""),
                   "ants_per_block": args.ants_per_block or 4, "table_rows": args.table_rows,
                   "lanes_per_ant": args.lanes_per_ant, "waves_per_ant": args.waves_per_ant or "auto"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(args.workload)
                                 if args.tabu == "bitmask" and args.select == "wrs" and args.cand_len is None
                                 and not args.ants else None),
                     "kernel": "k_construct" if args.select == "wrs" else "k_construct_prwm", "kernel_ms": cons_ms,
                     "kernel_ms_median": cons_median_ms, "kernel_launches_timed": kp,
                     "copy_measured_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "construct_only_tours_per_s": w["ants"] / (cons_ms * 1e-3),
                     "bytes_per_launch": nbytes},
    }
    out["search"] = {
        "fallback_step_fraction": float(np.mean(fb_steps)) / (w["ants"] * (n - 1)),
        "fallback_nodes_per_ant": float(np.mean(fb_nodes)) / w["ants"],
        "best_lengths": {"iterations": [c[0] for c in curve[::5]], "iteration_best": [c[1] for c in curve[::5]],
                         "global_best": [c[2] for c in curve[::5]]},
        "note": "from the untimed per-kernel pass that follows the timed steps",
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(dist, w, args.seed, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
