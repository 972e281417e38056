"""Train the learned column-scale MLP and evaluate it against Jacobi.

Three steps, each resumable on its own:

    # targets of a family of training systems (LSQR solves on the GPU)
    python -m paper_2604_11920_amd.train_scale search --family cfg0 --first 1 --count 160 \
        --out targets_cfg0.npz
    python -m paper_2604_11920_amd.train_scale search --family cfg1 --first 1 --count 24 \
        --out targets_cfg1.npz
    # fit the MLP on the GPU (the library's FP32 forward/backward and Adam)
    python -m paper_2604_11920_amd.train_scale fit targets_cfg0.npz targets_cfg1.npz \
        --out paper_2604_11920_amd/colscale_mlp.npz
    # held-out evaluation: iterations and seconds to eta <= tol, learned vs Jacobi
    python -m paper_2604_11920_amd.train_scale eval --model paper_2604_11920_amd/colscale_mlp.npz \
        --family cfg0 --first 1001 --count 20 --report report.json

Shipped models: colscale_mlp_c17.npz (the benchmark's; fitted on the 200
training systems of the family stated for the learned scale: c17cfg0 seeds
1-160, per-depth targets, three rounds from step 1; c17cfg1 seeds 161-200,
linear-in-depth targets, one round; 16,384 sampled columns per config-1-shape
system):

    python -m paper_2604_11920_amd.train_scale search --family c17cfg0 --first 1 --count 160 \
        --param depth --rounds 3 --step 1.0 --out targets_c17cfg0.npz
    python -m paper_2604_11920_amd.train_scale search --family c17cfg1 --first 161 --count 15 \
        --param linear --rounds 1 --out targets_c17cfg1_a.npz     # and 176 / 15, 191 / 10
    python -m paper_2604_11920_amd.train_scale fit targets_c17cfg0.npz targets_c17cfg1_a.npz \
        targets_c17cfg1_b.npz targets_c17cfg1_c.npz --cols-per-system 16384 \
        --out paper_2604_11920_amd/colscale_mlp_c17.npz
    python -m paper_2604_11920_amd.train_scale eval --model paper_2604_11920_amd/colscale_mlp_c17.npz \
        --family c17cfg1 --first 1001 --count 20 --report report.json

colscale_mlp.npz (fitted on cfg0 and cfg1 targets) and
colscale_mlp_cfg1.npz (fitted on config-1-geometry targets only: cfg1 seeds
1-6, and cfg1large seeds 1-5, depth family, one search round; the benchmark
system itself, seed 0 with 229 stations, is not among them):

    python -m paper_2604_11920_amd.train_scale search --family cfg1 --first 1 --count 6 \
        --param depth --rounds 1 --out targets_cfg1_depth.npz
    python -m paper_2604_11920_amd.train_scale search --family cfg1large --first 1 --count 2 \
        --param depth --rounds 1 --out targets_cfg1large_a.npz
    python -m paper_2604_11920_amd.train_scale search --family cfg1large --first 3 --count 3 \
        --param depth --rounds 1 --out targets_cfg1large_b.npz
    python -m paper_2604_11920_amd.train_scale fit targets_cfg1_depth.npz \
        targets_cfg1large_a.npz targets_cfg1large_b.npz --epochs 40 \
        --out paper_2604_11920_amd/colscale_mlp_cfg1.npz

Families: "cfg0" = config-0 geometry (16x16x9) with 20-60 stations and damping
0.05-0.5; "cfg1" = config-1 geometry (80x80x20) with 30-80 stations and 6-12
periods; "cfg1large" = config-1 geometry with 100-200 stations and 14-20
periods (near the benchmark system).  Each training system's targets come from the iteration-minimising
search of paper_2604_11920_amd.learned.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, flush=True)


def family(name, first, count):
    import synth
    if name == "cfg0":
        return synth.learned_family(first, count)
    if name == "cfg1":
        return synth.learned_family_wide(first, count)
    if name == "cfg1large":
        return synth.learned_family_large(first, count)
    if name in ("c17cfg0", "c17cfg1"):
        return synth.c17_family(name[3:], first, count)
    raise SystemExit(f"unknown family {name}")


def cmd_search(args):
    import synth
    from paper_2604_11920_amd import learned
    t0 = time.perf_counter()
    feats, targets, rows = [], [], []
    for i, cfg in enumerate(family(args.family, args.first, args.count)):
        s = synth.make_system(cfg)
        f, t, theta, kj, kb = learned.search_targets(
            s, tol=args.tol, family=args.param, rounds=args.rounds, step=args.step,
            progress=log if s.nnz > 50_000_000 else None)
        feats.append(f.astype(np.float32))
        targets.append(t.astype(np.float32))
        rows.append({"name": cfg.name, "n": int(s.n), "nnz": int(s.nnz), "jacobi_iters": int(kj),
                     "best_iters": int(kb), "theta": [float(x) for x in theta]})
        log(f"[search {i + 1}/{args.count}] {cfg.name}: jacobi {kj} best {kb} "
            f"({time.perf_counter() - t0:.0f}s)")
        # save after every system, so a cut-off run keeps what it has
        np.savez(args.out, feat=np.concatenate(feats), target=np.concatenate(targets),
                 sizes=np.array([len(x) for x in targets]), meta=np.array(json.dumps(rows)))


def load_blocks(path, cols=0, seed=0):
    """Per-system feature and target blocks of a target file, with each
    system's feature means over all its columns; cols > 0 keeps a seeded
    sample of at most that many columns per system (the means stay those of
    all columns, so centring matches inference)."""
    z = np.load(path, allow_pickle=False)
    cut = np.cumsum(z["sizes"])[:-1]
    feats = np.split(z["feat"].astype(np.float64), cut)
    targets = np.split(z["target"].astype(np.float64), cut)
    rows = json.loads(str(z["meta"]))
    means = list(z["means"]) if "means" in z else [f.mean(axis=0) for f in feats]
    if cols > 0:
        for i, f in enumerate(feats):
            if len(f) > cols:
                keep = np.sort(np.random.default_rng(seed + i).choice(len(f), cols, replace=False))
                feats[i], targets[i] = f[keep], targets[i][keep]
    return feats, targets, means, rows


def cmd_subsample(args):
    feats, targets, means, rows = load_blocks(args.targets, args.cols)
    np.savez(args.out, feat=np.concatenate(feats).astype(np.float32),
             target=np.concatenate(targets).astype(np.float32),
             sizes=np.array([len(x) for x in targets]), means=np.array(means),
             meta=np.array(json.dumps(rows)))
    log(f"[subsample] {len(rows)} systems, {sum(len(x) for x in targets)} columns -> {args.out}")


def cmd_fit(args):
    from paper_2604_11920_amd import learned
    feats, targets, means, rows = [], [], [], []
    for path in args.targets:
        # per-system blocks (features are centred per system)
        f, t, mu, r = load_blocks(path, args.cols_per_system)
        feats += f
        targets += t
        means += mu
        rows += r
    model = learned.train(feats, targets, epochs=args.epochs, log=log, means=means)
    model.meta["train_systems"] = rows
    model.meta["tol"] = args.tol
    model.save(args.out)
    log(f"[fit] {len(rows)} systems, {model.meta['samples']} columns; loss "
        f"{model.meta['loss_history'][-1][1]:.4e} (Jacobi multiplier: {model.meta['loss_at_jacobi']:.4e}); "
        f"saved {args.out}")


def cmd_eval(args):
    import synth
    from paper_2604_11920_amd import learned
    model = learned.ColumnScaleModel.load(args.model)
    ev = []
    for i, cfg in enumerate(family(args.family, args.first, args.count)):
        s = synth.make_system(cfg)
        kj, _ = learned.iterations_to_tol(s, None, args.tol, 20000)
        with learned.Solver.from_system(s, precond="jacobi", check_every=16) as sol:
            tj = time.perf_counter()
            dmj, _, _ = sol.solve(s.dt, 20000, tol=args.tol, history=False)
            tj = time.perf_counter() - tj
        dml, il = learned.solve_learned(s, model, args.tol, k_jacobi=kj)
        rd = float(np.linalg.norm(dml - dmj) / np.linalg.norm(dmj))
        ev.append({"name": cfg.name, "jacobi_iters": int(kj), "learned_iters": int(il["iters"]),
                   "learned_iters_total": int(il["iters_total"]), "learned_istop": il["istop"],
                   "fallback": il["fallback_used"], "jacobi_seconds": tj,
                   "learned_seconds": il["seconds"], "rel_diff": rd})
        log(f"[eval {i + 1}/{args.count}] {cfg.name}: jacobi {kj} learned {il['iters_total']} "
            f"(fallback {il['fallback_used']}) rel diff {rd:.2e}")
    jac = np.array([e["jacobi_iters"] for e in ev], dtype=float)
    lrn = np.array([e["learned_iters_total"] for e in ev], dtype=float)
    summary = {"family": args.family, "heldout": len(ev), "tol": args.tol,
               "mean_jacobi_iters": float(jac.mean()), "mean_learned_iters": float(lrn.mean()),
               "mean_iteration_ratio": float(np.mean(lrn / jac)),
               "systems_improved": int(np.sum(lrn < jac)),
               "fallbacks": int(sum(e["fallback"] for e in ev)),
               "max_rel_diff": max(e["rel_diff"] for e in ev)}
    log(f"[eval] {json.dumps(summary)}")
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"summary": summary, "heldout": ev,
                       "loss_history": model.meta.get("loss_history"),
                       "loss_at_jacobi": model.meta.get("loss_at_jacobi")}, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("search")
    a.add_argument("--family", default="cfg0", choices=["cfg0", "cfg1", "cfg1large", "c17cfg0", "c17cfg1"])
    a.add_argument("--first", type=int, default=1)
    a.add_argument("--count", type=int, default=160)
    a.add_argument("--tol", type=float, default=1e-6)
    a.add_argument("--param", default="depth", choices=["depth", "linear"],
                   help="target family: one log multiplier per depth layer, or linear in depth")
    a.add_argument("--rounds", type=int, default=2, help="coordinate-descent rounds (step halved)")
    a.add_argument("--step", type=float, default=0.5,
                   help="first round's step: candidates base + {-1, -1/2, 1/2, 1} x step")
    a.add_argument("--out", required=True)
    b = sub.add_parser("fit")
    b.add_argument("targets", nargs="+")
    b.add_argument("--epochs", type=int, default=60)
    b.add_argument("--cols-per-system", type=int, default=0,
                   help="fit on a seeded sample of at most this many columns per system")
    b.add_argument("--tol", type=float, default=1e-6)
    b.add_argument("--out", default=os.path.join(ROOT, "paper_2604_11920_amd", "colscale_mlp.npz"))
    c = sub.add_parser("eval")
    c.add_argument("--model", default=os.path.join(ROOT, "paper_2604_11920_amd", "colscale_mlp.npz"))
    c.add_argument("--family", default="cfg0", choices=["cfg0", "cfg1", "cfg1large", "c17cfg0", "c17cfg1"])
    c.add_argument("--first", type=int, default=1001)
    c.add_argument("--count", type=int, default=20)
    c.add_argument("--tol", type=float, default=1e-6)
    c.add_argument("--report", default=None)
    d = sub.add_parser("subsample")
    d.add_argument("targets")
    d.add_argument("--cols", type=int, required=True)
    d.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "subsample":          # host only
        cmd_subsample(args)
        return
    import torch
    torch.cuda.set_device(0)
    {"search": cmd_search, "fit": cmd_fit, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    main()
