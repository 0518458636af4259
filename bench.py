"""Throughput of the MMAS hot path on one MI355X.

One step is one iteration of Alg. 1 on the n = 1002 clustered workload
(1002 ants, candidate lists of 32, alpha 1, beta 2, rho 0.02, bitmask tabu):
choice_info (folded into the previous update), tour construction for every
ant, iteration and global best with the trail limits, evaporation + deposit +
clamp. The metric is tours constructed per second; inputs are resident in HBM
before the timed region starts.

Prints one JSON line with, besides the contract fields:
- `roofline`: the construction kernel's algorithmic bytes per launch over its
  average duration (HIP events on the library's stream);
- `variants`: the same workload with the compact tabu, as K colonies batched
  into one persistent launch per step, and the 256-instance batch (n in
  [100, 2000], ants = n), each with its own roofline;
- `time_to_gap`: the learned heuristic against the plain one (training on
  generated instances, then time to reach plain MMAS's B-iteration length on
  the 3795-city instance);
- `cpu_baseline`: the oracle timed on the host cores on a bounded sample.
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
TABU_NAMES = {0: "bitmask", 1: "compact", 2: "list"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def roofline(nbytes, kernel_ms, kernel, **extra):
    achieved = nbytes / (kernel_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel, "kernel_ms": kernel_ms,
           "bytes_per_launch": nbytes}
    out.update(extra)
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(threads, 16))


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


# ---------------------------------------------------------------------------
# single colony


def run_colony(args, workload, tabu, steps, warmup, kernel_passes=50):
    """One colony: warm-up, `steps` timed iterations, then an untimed pass with
    HIP events around every construction launch. Returns a dict with the
    throughput, the roofline of the construction kernel and the search curve."""
    import torch

    from paper_2003_11902_amd import instances as I
    from paper_2003_11902_amd import mmas as M

    xy, dist, w = I.workload_instance(workload)
    if args.ants:
        w["ants"] = args.ants
    if args.cand_len is not None:
        w["cand_len"] = args.cand_len
    n = w["n"]
    col = M.Colony(dist, w["ants"], cand_len=w["cand_len"], alpha=w["alpha"], beta=w["beta"],
                   rho=w["rho"], seed=args.seed, tabu=tabu, pher=w["pher"], ls_nn=w["ls_nn"],
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
    for _ in range(warmup):
        step(it)
        it += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(it)
        it += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"{workload} {tabu}: timed {steps} steps in {elapsed:.3f} s")

    # per-kernel pass: HIP events around the construction launch on its stream
    kp = min(steps, kernel_passes)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(kp)]
    fb_nodes, fb_steps, curve = [], [], []
    for k in range(kp):
        col.prepare_choice_info()
        ev[k][0].record(stream)
        col.construct(it)
        ev[k][1].record(stream)
        if w["ls_nn"]:
            col.two_opt()
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
    nbytes = algorithmic_bytes(n, col.cl, w["ants"], float(np.mean(fb_nodes)))
    col.close()
    return {
        "workload": workload, "w": w, "n": n, "tabu": tabu, "steps": steps, "warmup": warmup,
        "value": w["ants"] * steps / elapsed, "ms_per_step": elapsed / steps * 1e3,
        "roofline": roofline(nbytes, cons_ms, "k_construct" if args.select == "wrs" else "k_construct_prwm",
                             kernel_ms_median=float(np.median(cons_all)), kernel_launches_timed=kp,
                             construct_only_tours_per_s=w["ants"] / (cons_ms * 1e-3)),
        "search": {
            "fallback_step_fraction": float(np.mean(fb_steps)) / (w["ants"] * (n - 1)),
            "fallback_nodes_per_ant": float(np.mean(fb_nodes)) / w["ants"],
            "best_lengths": {"iterations": [c[0] for c in curve[::5]],
                             "iteration_best": [c[1] for c in curve[::5]],
                             "global_best": [c[2] for c in curve[::5]]},
            "note": "from the untimed per-kernel pass that follows the timed steps",
        },
        "dist": dist,
    }


# ---------------------------------------------------------------------------
# batches


def run_batch(batch_of, count, steps, warmup, tabu="bitmask", graph=True, kernel_passes=10):
    """K colonies of one named workload (seeds 1..K), or the mixed batch of
    `count` instances: autotuned launch shape, one captured graph per step.
    After the timed steps, an untimed pass runs the same step without the
    graph and brackets each construction launch with HIP events."""
    from paper_2003_11902_amd import instances as I
    from paper_2003_11902_amd import mmas as M

    t0 = time.perf_counter()
    if batch_of:
        _, d0, w = I.workload_instance(batch_of)
        dists = [d0] * count
        params = [M.make_params(w["n"], w["ants"], cand_len=w["cand_len"], alpha=w["alpha"], beta=w["beta"],
                                rho=w["rho"], seed=1 + k, tabu=tabu, pher=w["pher"], problem=w["problem"])
                  for k in range(count)]
        workload = f"{batch_of} x {count} colonies"
    else:
        insts = I.batch_instances(count)
        dists = [d for _, d in insts]
        params = [M.make_params(d.shape[0], d.shape[0], cand_len=32, rho=0.02, seed=1 + k, tabu=tabu)
                  for k, d in enumerate(dists)]
        workload = f"batched{count}"
    b = M.Batch(dists, params)
    setup_s = time.perf_counter() - t0
    apb, tb, lanes, tuned_tabu = b.tune()
    if graph:
        b.capture()
    for _ in range(warmup):
        b.step()
    b.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        b.step()
    b.synchronize()
    elapsed = time.perf_counter() - t1
    log(f"{workload}: set-up {setup_s:.1f} s, {steps} steps in {elapsed:.3f} s")
    # construction-kernel pass
    b.set_timing(True)
    fb = np.zeros(len(dists))
    for _ in range(kernel_passes):
        b.step()
        b.synchronize()
        fb += np.array([b.instance(k).fallback()[1].sum() for k in range(len(dists))], dtype=np.float64)
    cons_ms, calls = b.read_timing(reset=True)
    b.set_timing(False)
    cons_ms /= max(calls, 1)
    fb /= kernel_passes
    nbytes = 0.0
    for k, (d, p) in enumerate(zip(dists, params)):
        n = d.shape[0]
        nbytes += algorithmic_bytes(n, min(int(p.cand_len), n - 1), int(p.ants), float(fb[k]))
    total_ants = sum(int(p.ants) for p in params)
    b.close()
    return {
        "value": total_ants * steps / elapsed, "unit": "tours/s", "steps": steps, "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "config": {"workload": workload, "instances": count,
                   "n_range": [int(min(d.shape[0] for d in dists)), int(max(d.shape[0] for d in dists))],
                   "ants": "n per instance" if not batch_of else int(params[0].ants),
                   "cand_len": int(params[0].cand_len), "rho": float(params[0].rho),
                   "tabu": TABU_NAMES[tuned_tabu], "graph": graph, "ants_per_block": apb, "table_bytes": tb,
                   "lanes_per_ant": lanes, "total_ants": total_ants},
        "roofline": roofline(nbytes, cons_ms, "k_batch_construct", kernel_launches_timed=calls,
                             construct_only_tours_per_s=total_ants / (cons_ms * 1e-3),
                             note="construction launches timed in an untimed pass of the same step run "
                                  "without its graph"),
    }


# ---------------------------------------------------------------------------
# learned heuristic


def run_time_to_gap(args):
    """The learned heuristic against the plain one: training data from plain
    MMAS on generated instances, training, then on the 3795-city instance the
    time the learned run needs to reach the length plain MMAS has after B
    iterations, over seeds 1..S; gaps against L_ref, the best tour of a long
    MMAS + 2-opt run on the same instance."""
    import torch

    from paper_2003_11902_amd import instances as I
    from paper_2003_11902_amd import learned as L

    quiet = (lambda m: None) if not args.verbose else log
    t0 = time.perf_counter()
    X, F = L.training_set(args.ttg_count, 200, 1000, R=args.ttg_label_seeds, iterations=args.ttg_label_iterations,
                          ants=64, log=quiet)
    data_s = time.perf_counter() - t0
    log(f"time to gap: training data ({int(X.shape[0])} edges of {args.ttg_count} instances) in {data_s:.1f} s")
    t1 = time.perf_counter()
    params, hist = L.train(X, F, epochs=args.ttg_epochs, log=quiet)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del X, F
    xy, dist, w = I.workload_instance("uniform3795")
    L_ref = L.reference_length(dist, iterations=300, log=quiet)
    recs = L.time_to_gap(params, dist, xy, seeds=range(1, args.ttg_seeds + 1), budget=args.ttg_budget,
                         cand_len=w["cand_len"], rho=w["rho"], log=quiet)
    ratios = [r["ratio"] for r in recs if r["ratio"] is not None]
    total_s = time.perf_counter() - t0
    log(f"time to gap: {len(ratios)}/{len(recs)} seeds reached plain's length, median ratio "
        f"{float(np.median(ratios)) if ratios else float('nan'):.3f}, {total_s:.1f} s in all")
    return {
        "metric": "time-to-gap learned vs plain (wall time of the learned run to reach plain MMAS's "
                  "B-iteration length, over plain's time for B iterations)",
        "value": float(np.median(ratios)) if ratios else None, "unit": "ratio", "higher_is_better": False,
        "reached": len(ratios), "seeds": len(recs), "budget_iterations": args.ttg_budget,
        "eval_instance": "uniform3795 (n = 3795 uniform in [0, 1e4]^2, seed 5), 3795 ants, cl 32, rho 0.02",
        "reference_len": L_ref, "reference": "best of MMAS + 2-opt (8-NN), 64 ants, 300 iterations, seed 1000",
        "median_plain_gap": float(np.median([(r["plain_len"] - L_ref) / L_ref for r in recs])),
        "median_learned_gap": float(np.median([(r["learned_final_len"] - L_ref) / L_ref for r in recs])),
        "median_plain_s": float(np.median([r["plain_s"] for r in recs])),
        "median_learned_s": float(np.median([r["learned_s"] for r in recs])),
        "training": {"instances": args.ttg_count, "n_range": [200, 1000], "label_seeds": args.ttg_label_seeds,
                     "label_iterations": args.ttg_label_iterations, "label_ants": 64, "epochs": args.ttg_epochs,
                     "data_s": data_s, "train_s": train_s, "loss": hist},
        "runs": [{k: r[k] for k in ("seed", "plain_len", "plain_s", "learned_iters", "learned_s",
                                    "learned_final_len", "ratio")} for r in recs],
        "total_s": total_s,
    }


# ---------------------------------------------------------------------------
# CPU baseline


def cpu_baseline(dist, w, seed, budget_s):
    """The oracle, built for this host (-march=native, no contraction), timed
    on whole iterations (OpenMP over ants, all usable cores up to 16) and on
    construction alone, plus one thread as the paper's CPU runs."""
    from oracle import build as OB
    from oracle import oracle as O

    native = True
    try:
        O.use_library(OB.build(native=True))
    except Exception as e:  # noqa: BLE001  (fall back to the portable build, say so)
        log(f"native oracle build failed ({e}); timing the portable build")
        native = False
    threads = host_threads()

    def colony():
        return O.Colony(dist, w["ants"], cand_len=w["cand_len"], alpha=w["alpha"], beta=w["beta"],
                        rho=w["rho"], seed=seed, problem=w.get("problem", "tsp"))

    o = colony()
    t0 = time.perf_counter()
    it = 0
    cons_s = 0.0
    while True:
        o.prepare_choice()
        c0 = time.perf_counter()
        o.construct(it, threads)
        cons_s += time.perf_counter() - c0
        o.update()
        it += 1
        el = time.perf_counter() - t0
        if el >= budget_s or it >= 200:
            break
    o1 = colony()
    t1 = time.perf_counter()
    it1 = 0
    while True:
        o1.iterate(it1, 1)
        it1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= budget_s / 3 or it1 >= 50:
            break
    build = "gcc -O2 -march=native -ffp-contract=off" if native else "gcc -O2 -ffp-contract=off"
    return {"value": w["ants"] * it / el, "unit": "tours/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "build": build,
            "sample": f"{it} full iterations (choice, construction of {w['ants']} tours, update) of the same "
                      f"workload, OpenMP over ants, {el:.1f} s",
            "construct_only_tours_per_s": w["ants"] * it / cons_s,
            "value_1_core": w["ants"] * it1 / el1,
            "sample_1_core": f"{it1} iterations of a fresh colony on one thread, {el1:.1f} s"}


# ---------------------------------------------------------------------------


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
    ap.add_argument("--headline-only", action="store_true",
                    help="only the single colony (no variants, no time to gap)")
    ap.add_argument("--no-time-to-gap", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="time the batched workload (256 instances, n in [100, 2000], ants = n) "
                         "instead of the single colony")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-of", default=None,
                    help="with --batched: that many colonies of this named workload (seeds 1..K) instead of "
                         "the mixed 256-instance batch")
    ap.add_argument("--colonies", type=int, default=8, help="K of the batched-colonies variant")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--ttg-count", type=int, default=2000)
    ap.add_argument("--ttg-label-seeds", type=int, default=8)
    ap.add_argument("--ttg-label-iterations", type=int, default=300)
    ap.add_argument("--ttg-epochs", type=int, default=8)
    ap.add_argument("--ttg-seeds", type=int, default=10)
    ap.add_argument("--ttg-budget", type=int, default=500)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (3 times) and exit; "
                         "its FETCH_SIZE / WRITE_SIZE calibrate the HBM traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the method's "
              "multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)

    import torch

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
        r = run_batch(args.batch_of, args.batch_count, args.steps, args.warmup, tabu=args.tabu,
                      graph=not args.no_graph)
        out = {"metric": ("tours constructed/sec, batched instances (1 GPU)" if not args.batch_of
                          else f"tours constructed/sec, {args.batch_count} colonies batched (1 GPU)"),
               "value": r["value"], "unit": "tours/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f32", "data": "synthetic", "config": r["config"], "roofline": r["roofline"]}
        print(json.dumps(out), flush=True)
        return

    head = run_colony(args, args.workload, args.tabu, args.steps, args.warmup)
    w, n = head["w"], head["n"]
    rf = head["roofline"]
    default_head = (args.tabu == "bitmask" and args.select == "wrs" and args.cand_len is None and not args.ants)
    rf["traffic"] = measured_traffic(args.workload) if default_head else None
    rf["copy_measured_gbs"] = copy_bandwidth_gbs(torch)
    rf["frac_of_copy"] = rf["achieved"] / rf["copy_measured_gbs"]
    out = {
        "metric": f"tours constructed/sec at n={n}" + (" with 2-opt on every tour" if w["ls_nn"] else "") + " (1 GPU)",
        "value": head["value"],
        "unit": "tours/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
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
        "roofline": rf,
        "search": head["search"],
    }
    if not args.headline_only and args.workload == "clustered1002":
        var = {}
        c = run_colony(args, args.workload, "compact", args.steps, args.warmup)
        var["compact_tabu"] = {"value": c["value"], "unit": "tours/s", "steps": args.steps,
                               "ms_per_step": c["ms_per_step"],
                               "config": {"workload": "clustered1002", "tabu": "compact", "ants": w["ants"],
                                          "cand_len": w["cand_len"]},
                               "roofline": c["roofline"]}
        var["colonies_batched"] = run_batch("clustered1002", args.colonies, args.steps, args.warmup)
        var["batched256"] = run_batch(None, 256, args.steps, args.warmup)
        out["variants"] = var
        if not args.no_time_to_gap:
            out["time_to_gap"] = run_time_to_gap(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(head["dist"], w, args.seed, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
