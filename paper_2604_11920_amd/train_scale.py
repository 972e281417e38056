"""Train the learned column-scale MLP and evaluate it against Jacobi.

    python -m paper_2604_11920_amd.train_scale --train 200 --heldout 20 \
        --out paper_2604_11920_amd/colscale_mlp.npz --report report.json

Training systems: config-0 geometry (16x16x9) with 20-60 stations and damping
0.05-0.5 (seeds 1..N); held-out systems: the same family, seeds 1001..  Each
training system's targets come from the iteration-minimising search of
paper_2604_11920_amd.learned; the MLP is then fitted on the GPU.  The report
gives, per held-out system, LSQR iterations and seconds to eta <= 1e-6 with
Jacobi and with the learned scale, and the relative difference of the two
solutions.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--heldout", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2604_11920_amd", "colscale_mlp.npz"))
    ap.add_argument("--report", default=None)
    args = ap.parse_args()

    import torch

    import synth
    from paper_2604_11920_amd import learned

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    feats, targets, rows = [], [], []
    for i, cfg in enumerate(synth.learned_family(1, args.train)):
        s = synth.make_system(cfg)
        f, t, theta, kj, kb = learned.search_targets(s, tol=args.tol)
        feats.append(f)
        targets.append(t)
        rows.append({"name": cfg.name, "jacobi_iters": kj, "best_iters": kb, "theta": theta.tolist()})
        log(f"[train {i + 1}/{args.train}] {cfg.name}: jacobi {kj} best {kb} "
            f"({time.perf_counter() - t0:.0f}s)")
    model = learned.train(feats, targets, epochs=args.epochs, log=log)
    model.meta["train_systems"] = rows
    model.meta["tol"] = args.tol
    model.save(args.out)
    log(f"[train] saved {args.out}")

    ev = []
    for i, cfg in enumerate(synth.learned_family(1001, args.heldout)):
        s = synth.make_system(cfg)
        kj, ij = learned.iterations_to_tol(s, None, args.tol, 20000)
        with learned.Solver.from_system(s, precond="jacobi", check_every=16) as sol:
            tj = time.perf_counter()
            dmj, _, _ = sol.solve(s.dt, 20000, tol=args.tol, history=False)
            tj = time.perf_counter() - tj
        dml, il = learned.solve_learned(s, model, args.tol, k_jacobi=kj)
        rd = float(np.linalg.norm(dml - dmj) / np.linalg.norm(dmj))
        ev.append({"name": cfg.name, "jacobi_iters": kj, "learned_iters": il["iters"],
                   "learned_istop": il["istop"], "fallback": il["fallback_used"],
                   "jacobi_seconds": tj, "learned_seconds": il["seconds"], "rel_diff": rd})
        log(f"[heldout {i + 1}/{args.heldout}] {cfg.name}: jacobi {kj} learned {il['iters']} "
            f"(fallback {il['fallback_used']}) rel diff {rd:.2e}")
    jac = np.array([e["jacobi_iters"] for e in ev], dtype=float)
    lrn = np.array([e["learned_iters"] for e in ev], dtype=float)
    summary = {"heldout": len(ev), "mean_jacobi_iters": float(jac.mean()),
               "mean_learned_iters": float(lrn.mean()),
               "mean_iteration_ratio": float(np.mean(lrn / jac)),
               "systems_improved": int(np.sum(lrn < jac)), "max_rel_diff": max(e["rel_diff"] for e in ev)}
    log(f"[heldout] {json.dumps(summary)}")
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"summary": summary, "heldout": ev, "train": rows,
                       "loss_history": model.meta["loss_history"],
                       "loss_at_jacobi": model.meta["loss_at_jacobi"]}, f, indent=1)


if __name__ == "__main__":
    main()
