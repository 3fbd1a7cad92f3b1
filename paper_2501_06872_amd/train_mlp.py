"""Train the parameter-choice MLP on timings the autotuner measures.

    python -m paper_2501_06872_amd.train_mlp --out models/gt_mlp.bin --metrics train_metrics.json

1. Seeded synthetic training graphs (the uneven batch distribution: R-MAT,
   uniform and geometric-locality graphs of 2^10..2^22 vertices, plus a few
   large ones); evaluation graphs come from disjoint seeds.
2. For every graph: its sampled features (the plan's sampling pass) and the
   run time of each of the 32 kernel configurations (gt_autotune: median of
   `reps` timed runs).
3. Targets: per graph, log time of each configuration minus the mean over
   configurations.  Loss: mean squared error.  Training runs entirely in the
   library's HIP kernels (gt_mlp_gradient, gt_mlp_adam), full batch.
4. Regret on the evaluation graphs (chosen time / best time) for the MLP and
   for the heuristic, written as JSON.
"""
import argparse
import concurrent.futures
import json
import math
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import gen  # noqa: E402
import paper_2501_06872_amd as gt  # noqa: E402
from paper_2501_06872_amd import mlp_model  # noqa: E402


def log(*a):
    print(*a, flush=True)


def graph_specs(count, seed, large=0):
    specs = gen.batch_specs(count, seed=seed)
    rs = np.random.default_rng(seed)
    for i in range(large):
        fam = int(rs.integers(0, 3))
        n = 1 << int(rs.integers(23, 25))
        spec = dict(n=n, ef=int(rs.choice([8, 16])), family=fam, seed=seed * 1000 + i, payload=bool(i % 2))
        if fam == gen.FAM_RMAT:
            spec.update(probs=gen.RMAT_G500, permute=bool(rs.integers(0, 2)))
        elif fam == gen.FAM_GEOMETRIC:
            spec.update(p_geom=0.01)
        specs.append(spec)
    return specs


def heuristic_config(n, m):
    """Index of the heuristic's choice in the configuration grid."""
    avg = m / max(n, 1)
    fb = int(round(math.log2(8192.0 / max(avg, 1.0))))
    fb = min(max(fb, 6), 9)
    L = max(1, (max(int(n), 2) - 1).bit_length())
    # variant 1; 10-bit digits, or 8-bit ones (the same three passes as the
    # heuristic's 9) when the coarse bits would need two 10-bit passes
    return (fb - 6) * 8 + (0 if L - fb > 18 else 1)


def collect(specs, dev, reps, seed=77, verbose=False):
    X, Tm, sizes = [], [], []
    pool = concurrent.futures.ThreadPoolExecutor(8)  # the generator releases the GIL
    futures = [pool.submit(gen.from_spec, spec) for spec in specs]
    for k, fut in enumerate(futures):
        O, D, P = fut.result()
        futures[k] = None
        g = (torch.from_numpy(O).to(dev), torch.from_numpy(D).to(dev),
             torch.from_numpy(P.view(np.int32)).to(dev) if P is not None else None)
        if verbose:
            log(f"  [graph {k}] n={O.size - 1} m={D.size} spec={specs[k]}")
        feats = gt.Plan([g], gt.make_options(policy=gt.POLICY_HEURISTIC, seed=seed, flags=gt.FLAG_FEATURES)).features()
        ms, _ = gt.autotune(*g, reps=reps)
        X.append(feats)
        Tm.append(ms)
        sizes.append((O.size - 1, D.size))
        if k % 16 == 0:
            log(f"  graph {k}/{len(specs)} n={O.size - 1} m={D.size} best={min(ms):.3f} ms worst={max(ms):.3f} ms")
        del g, O, D, P
        torch.cuda.empty_cache()
    pool.shutdown()
    return np.array(X, dtype=np.float32), np.array(Tm, dtype=np.float64), sizes


def targets(Tm):
    L = np.log(Tm)
    return (L - L.mean(axis=1, keepdims=True)).astype(np.float32)


def init_params(rng):
    """He initialisation: weights ~ N(0, 2 / fan_in), biases zero."""
    F, H, G = mlp_model.INPUTS, mlp_model.HIDDEN, mlp_model.OUTPUTS
    parts = []
    for fan_in, fan_out in ((F, H), (H, H), (H, G)):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / fan_in), size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(X, Y, dev, steps, lr, seed=0):
    rng = np.random.default_rng(seed)
    p = torch.from_numpy(init_params(rng)).to(dev)
    m1 = torch.zeros_like(p)
    m2 = torch.zeros_like(p)
    Xt = torch.from_numpy(X).to(dev)
    Yt = torch.from_numpy(Y).to(dev)
    work = torch.empty(gt.lib().gt_mlp_work_floats(X.shape[0]), dtype=torch.float32, device=dev)
    hist = []
    for step in range(1, steps + 1):
        _, grad, loss = gt.mlp_gradient(p, Xt, Yt, work)
        gt.mlp_adam(p, grad, m1, m2, step, lr)
        if step % 200 == 0 or step == 1:
            hist.append((step, loss.item()))
    return p.cpu().numpy(), hist


def regret(params, X, Tm, sizes, dev):
    y = gt.mlp_forward(torch.from_numpy(params).to(dev), torch.from_numpy(X).to(dev)).cpu().numpy()
    best = Tm.min(axis=1)
    pick = y.argmin(axis=1)
    t_mlp = Tm[np.arange(len(Tm)), pick]
    t_heur = np.array([Tm[i, heuristic_config(n, m)] for i, (n, m) in enumerate(sizes)])
    gm = lambda a: float(np.exp(np.mean(np.log(a))))
    return dict(graphs=len(Tm), regret_mlp_geomean=gm(t_mlp / best), regret_heuristic_geomean=gm(t_heur / best),
                gain_mlp_over_heuristic_geomean=gm(t_heur / t_mlp), total_ms_best=float(best.sum()),
                total_ms_mlp=float(t_mlp.sum()), total_ms_heuristic=float(t_heur.sum()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=mlp_model.DEFAULT_PATH)
    ap.add_argument("--metrics", default=None)
    ap.add_argument("--train-graphs", type=int, default=320)
    ap.add_argument("--eval-graphs", type=int, default=48)
    ap.add_argument("--large", type=int, default=8)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--verbose", action="store_true", help="name every graph before it is timed")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    t0 = time.time()
    log("[train] collecting training timings")
    Xtr, Ttr, Str = collect(graph_specs(args.train_graphs, 1001, args.large), dev, args.reps, verbose=args.verbose)
    log(f"[train] collecting evaluation timings ({time.time() - t0:.0f} s)")
    Xev, Tev, Sev = collect(graph_specs(args.eval_graphs, 2001, args.large // 2), dev, args.reps, verbose=args.verbose)
    log(f"[train] training ({time.time() - t0:.0f} s)")
    params, hist = train(Xtr, targets(Ttr), dev, args.steps, args.lr)
    fmin, fmax = Xtr.min(axis=0), Xtr.max(axis=0)
    mlp_model.save(args.out, params, fmin, fmax)
    res = dict(train=regret(params, Xtr, Ttr, Str, dev), eval=regret(params, Xev, Tev, Sev, dev), loss=hist,
               seconds=time.time() - t0, configs=[gt.config(c) for c in range(gt.num_configs())])
    log(json.dumps({k: v for k, v in res.items() if k in ("train", "eval")}))
    if args.metrics:
        with open(args.metrics, "w") as f:
            json.dump(res, f, indent=1)
        np.savez(os.path.splitext(args.metrics)[0] + "_data.npz", Xtr=Xtr, Ttr=Ttr, Xev=Xev, Tev=Tev,
                 Str=np.array(Str), Sev=np.array(Sev))


if __name__ == "__main__":
    main()
