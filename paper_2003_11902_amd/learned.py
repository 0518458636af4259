"""Learned heuristic driver: training data, training loop and evaluation.

Every computation runs in the library's kernels (feature extraction, labels,
MLP forward/backward, Adam, installation, MMAS itself); this module only
sequences the calls and moves arrays. Inputs are the seeded synthetic
instances of `instances`.

Training data: instances with n uniform in [n_lo, n_hi] (uniform and
clustered alternately); each is solved by plain MMAS with R seeds (one batch
for all instances and seeds), and the target of a kNN edge is the share of the
R global-best tours that contain it.

Evaluation (time to gap): on one instance, plain MMAS runs B iterations; its
final global best L_plain(B) and wall time T_plain set the bar. The learned
run (features + inference + installation + MMAS) is timed until its global
best first reaches L_plain(B). Reported: t*/T_plain per seed and the median,
and the gaps of both runs' B-iteration lengths to L_ref, the best tour of a
long MMAS run with 2-opt on the same instance.
"""
from __future__ import annotations

import time

import numpy as np

from . import instances as I
from . import mmas as M

HID = 128


def init_params(seed: int, bias: float = 0.0) -> np.ndarray:
    """Uniform Glorot initialisation; W1 rows 8..15 (zero inputs) stay 0;
    the output bias starts at `bias`."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((16, HID), np.float32)
    a1 = np.sqrt(6.0 / (8 + HID))
    W1[:8] = rng.uniform(-a1, a1, (8, HID))
    a2 = np.sqrt(6.0 / (2 * HID))
    W2 = rng.uniform(-a2, a2, (HID, HID)).astype(np.float32)
    a3 = np.sqrt(6.0 / (HID + 1))
    w3 = rng.uniform(-a3, a3, HID).astype(np.float32) * 0.1
    p = np.concatenate([W1.ravel(), np.zeros(HID, np.float32), W2.ravel(), np.zeros(HID, np.float32), w3,
                        np.array([bias], np.float32)]).astype(np.float32)
    assert p.size == M.mlp_param_count()
    return p


def training_set(count=2000, n_lo=200, n_hi=1000, base_seed=20000, R=4, iterations=100, ants=64, cand_len=32,
                 rho=0.02, colonies_per_batch=2048, log=print):
    """(X uint16 [E,16] bfloat16 bits, targets float32 [E]) on the GPU. The
    colonies (instances x R seeds) are solved in batches of about
    `colonies_per_batch`, so that each batched step keeps the GPU busy."""
    import torch

    rng = np.random.default_rng(base_seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    t0 = time.perf_counter()
    insts = []
    for k in range(count):
        kind = "uniform" if k % 2 == 0 else "clustered"
        xy, d = I.make_instance(kind, int(sizes[k]), seed=base_seed + k)
        insts.append((xy, d))
    log(f"[learned] {count} instances generated in {time.perf_counter() - t0:.1f} s")
    Xs, Fs = [], []
    chunk = max(1, colonies_per_batch // R)  # instances per batch
    for c0 in range(0, count, chunk):
        part = insts[c0:c0 + chunk]
        dists, params = [], []
        for xy, d in part:
            for r in range(R):
                dists.append(d)
                params.append(M.make_params(d.shape[0], ants, cand_len=cand_len, rho=rho, seed=1 + r))
        b = M.Batch(dists, params)
        b.capture()
        for _ in range(iterations):
            b.step()
        b.synchronize()
        for q, (xy, d) in enumerate(part):
            dd = torch.from_numpy(d).cuda()
            knn, X, _ = M.mmas_mlp_features(dd, torch.from_numpy(xy.astype(np.float32)).cuda())
            tours = torch.stack([b.instance(q * R + r).tensor(M.MMAS_BUF_GB_TOUR) for r in range(R)]).contiguous()
            Fs.append(M.mmas_mlp_labels(tours, knn).reshape(-1))
            Xs.append(X)
        b.close()
        del b
        log(f"[learned] labels for {min(count, c0 + chunk)}/{count} instances, "
            f"{time.perf_counter() - t0:.1f} s")
    X = torch.cat(Xs)
    F = torch.cat(Fs)
    torch.cuda.synchronize()
    return X, F


def train(X, F, epochs=4, batch=65536, lr=2e-3, seed=0, groups=256, log=print):
    """Adam on mini-batches of contiguous edge ranges after one fixed shuffle
    of the instances' edge blocks. Returns (params tensor, loss per epoch)."""
    import torch

    E = int(X.shape[0])
    mean = float(F.mean().item())
    bias = float(np.log(max(mean, 1e-4) / max(1 - mean, 1e-4)))
    params = torch.from_numpy(init_params(seed, bias)).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    packed = M.mmas_mlp_pack(params)
    P = M.mlp_param_count()
    partial = torch.empty(groups * (P + 1), dtype=torch.float32, device="cuda")
    grad = torch.empty(P + 1, dtype=torch.float32, device="cuda")
    # one shuffle of 1024-edge blocks (host permutation of block indices)
    blocks = (E + 1023) // 1024
    order = np.random.default_rng(seed).permutation(blocks)
    idx = torch.from_numpy(order).cuda()
    starts = idx * 1024
    rows = (starts[:, None] + torch.arange(1024, device="cuda")[None, :]).reshape(-1)
    rows = rows[rows < E]
    Xs = X.index_select(0, rows)
    Fs = F.index_select(0, rows)
    step = 0
    history = []
    for ep in range(epochs):
        tot = 0.0
        for b0 in range(0, E, batch):
            xb = Xs[b0:b0 + batch]
            fb = Fs[b0:b0 + batch]
            M.mmas_mlp_grad(xb, fb, params, packed, groups=groups, partial=partial, grad=grad)
            step += 1
            M.mmas_mlp_adam(params, grad, m, v, lr, step)
            # refresh the bfloat16 copies in place
            M._check(M.lib.mmas_mlp_pack(M._dptr(params), M._dptr(packed), M._cur_stream()), "mmas_mlp_pack")
            tot += float(grad[P].item())
        history.append(tot / E)
        log(f"[learned] epoch {ep}: mean loss {tot / E:.5f}")
    return params, history


def scores(params, dist, xy):
    """(knn, s [n,16]) of one instance."""
    import torch

    dd = torch.from_numpy(np.ascontiguousarray(dist, np.int32)).cuda()
    knn, X, _ = M.mmas_mlp_features(dd, torch.from_numpy(np.ascontiguousarray(xy, np.float32)).cuda())
    packed = M.mmas_mlp_pack(params)
    s = M.mmas_mlp_forward(X, params, packed)
    return knn, s.reshape(-1, 16)


def time_to_gap(params, dist, xy, seeds=range(1, 11), budget=500, ants=None, cand_len=32, rho=0.02, check_every=5,
                full=True, log=print):
    """Per seed: plain MMAS for `budget` iterations (final best L and wall time
    T); the learned run (inference and installation included) timed until its
    best first reaches L. With `full`, the learned run then continues (untimed)
    to `budget` iterations so that both final lengths can be compared.
    Returns a list of dicts."""
    import torch

    n = dist.shape[0]
    ants = ants or n
    out = []
    for seed in seeds:
        plain = M.Colony(dist, ants, cand_len=cand_len, rho=rho, seed=seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(budget):
            plain.iterate(it)
        _, L_plain = plain.best()
        T_plain = time.perf_counter() - t0
        learned = M.Colony(dist, ants, cand_len=cand_len, rho=rho, seed=seed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        knn, s = scores(params, dist, xy)
        learned.set_learned_heuristic(knn, s)
        reached = None
        t_star = None
        L_learned = None
        it = 0
        while it < budget:
            learned.iterate(it)
            it += 1
            if reached is None and (it % check_every == 0 or it == budget):
                _, L_learned = learned.best()
                if L_learned <= L_plain:
                    reached = it
                    t_star = time.perf_counter() - t1
                    if not full:
                        break
        _, L_final = learned.best()
        if t_star is None:
            t_star = time.perf_counter() - t1
        rec = {"seed": seed, "plain_len": L_plain, "plain_s": T_plain, "learned_iters": reached, "learned_s": t_star,
               "learned_final_len": L_final if full else None, "learned_final_iters": it,
               "ratio": (t_star / T_plain) if reached is not None else None}
        log(f"[learned] seed {seed}: plain {L_plain} in {T_plain:.2f} s; learned "
            f"{'reached it at iteration ' + str(reached) if reached else 'did not reach it'} in {t_star:.2f} s"
            + (f"; learned after {it} iterations: {L_final}" if full else ""))
        out.append(rec)
        plain.close()
        learned.close()
    return out


def reference_length(dist, iterations=300, ants=64, cand_len=32, ls_nn=8, rho=0.02, seed=1000, log=print):
    """L_ref: the best tour of a long plain MMAS run with 2-opt on every tour
    (the yardstick the gaps are quoted against)."""
    col = M.Colony(dist, ants, cand_len=cand_len, rho=rho, seed=seed, ls_nn=ls_nn)
    t0 = time.perf_counter()
    for it in range(iterations):
        col.iterate(it)
    _, L = col.best()
    col.close()
    log(f"[learned] reference: MMAS + 2-opt, {ants} ants, {iterations} iterations: {L} "
        f"({time.perf_counter() - t0:.1f} s)")
    return int(L)


def main(argv=None):
    """Train on generated instances and report the time to gap as one JSON line."""
    import argparse
    import json

    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--n-lo", type=int, default=200)
    ap.add_argument("--n-hi", type=int, default=1000)
    ap.add_argument("--label-seeds", type=int, default=8)
    ap.add_argument("--label-iterations", type=int, default=300)
    ap.add_argument("--label-ants", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--eval-n", type=int, default=3795)
    ap.add_argument("--eval-seeds", type=int, default=10)
    ap.add_argument("--budget", type=int, default=500)
    ap.add_argument("--ref-iterations", type=int, default=300,
                    help="iterations of the MMAS + 2-opt run that gives the reference length")
    ap.add_argument("--eval-cand-len", type=int, default=32,
                    help="candidate-list length of both evaluated runs")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    X, F = training_set(args.count, args.n_lo, args.n_hi, R=args.label_seeds, iterations=args.label_iterations,
                        ants=args.label_ants)
    t_data = time.perf_counter() - t0
    t1 = time.perf_counter()
    params, hist = train(X, F, epochs=args.epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    xy, dist = I.make_instance("uniform", args.eval_n, seed=5)
    L_ref = reference_length(dist, iterations=args.ref_iterations)
    recs = time_to_gap(params, dist, xy, seeds=range(1, args.eval_seeds + 1), budget=args.budget,
                       cand_len=args.eval_cand_len)
    for r in recs:
        r["plain_gap"] = (r["plain_len"] - L_ref) / L_ref
        r["learned_final_gap"] = (r["learned_final_len"] - L_ref) / L_ref if r["learned_final_len"] else None
    ratios = [r["ratio"] for r in recs if r["ratio"] is not None]
    out = {"metric": "time-to-gap learned vs plain", "eval_instance": f"uniform n={args.eval_n} seed 5",
           "budget_iterations": args.budget, "eval_cand_len": args.eval_cand_len, "reached": len(ratios), "seeds": len(recs),
           "median_ratio": float(np.median(ratios)) if ratios else None,
           "reference_len": L_ref,
           "median_plain_gap": float(np.median([r["plain_gap"] for r in recs])),
           "median_learned_final_gap": float(np.median([r["learned_final_gap"] for r in recs])),
           "train_edges": int(X.shape[0]), "train_instances": args.count, "data_s": t_data,
           "train_s": t_train, "loss": hist, "runs": recs}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
