"""Write the oracle's converged solutions for selected right-hand sides of the
largest system of the batched workload (config-1 geometry, 229 stations, 20
periods, generator seed 3; right-hand sides from synth.checker_rhs_batch) to
tests/golden/cfg3_largest.npz.

Only oracle/ computes anything here (synth/ supplies the inputs).  For each
selected right-hand side r: LSQR (FP64, Jacobi column scale, Neumaier-
compensated sums) run to eta <= 1e-12, or until eta stops improving for 200
iterations, accepted when the eta <= 1e-11 and final iterates agree to 1e-7.
A fingerprint of the generated system is stored with the results.

Usage: python tests/golden/make_cfg3_golden.py [--threads 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "cfg3_largest.npz")
PICK = (0, 16)          # a 2-cell checkerboard and the first noise draw


def log(msg):
    print(f"[golden3] {msg}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--cap", type=int, default=40000)
    args = ap.parse_args()
    t0 = time.time()
    s = synth.make_system(synth.config3_systems()[-1])
    rhs = synth.checker_rhs_batch(s)
    fp = synth.fingerprint(s)
    log(f"system m={s.m} n={s.n} nnz={s.nnz} fingerprint {fp[:16]} ({time.time() - t0:.0f} s)")
    op = oracle.Operator.from_system(s, nthreads=args.threads)
    d = op.jacobi()
    del op
    opj = oracle.Operator.from_system(s, d=d, compensated=True, nthreads=args.threads)
    arrays, meta = {}, {"picked": list(PICK)}
    for r in PICK:
        t1 = time.time()
        out = opj.lsqr_ref(rhs[:, r], args.cap, 1e-12, 1e-11, stall=200)
        gap = float(np.linalg.norm(out["x"] - out["x_snap"]) / np.linalg.norm(out["x"]))
        acc = bool(out["k_snap"] > 0 and gap <= 1e-7)
        arrays[f"x_star_{r}"] = out["x"]
        meta.update({f"iters_{r}": int(out["iters"]), f"istop_{r}": int(out["istop"]),
                     f"eta_{r}": float(out["hist"][-1, 2]), f"gap_{r}": gap,
                     f"accepted_{r}": acc})
        log(f"rhs {r}: {out['iters']} iterations, istop {out['istop']}, eta "
            f"{out['hist'][-1, 2]:.3e}, gap {gap:.3e}, accepted {acc} ({time.time() - t1:.0f} s)")
    meta.update(fingerprint=fp, m=int(s.m), n=int(s.n), nnz=int(s.nnz), threads=args.threads,
                seconds=round(time.time() - t0, 1))
    np.savez(OUT, meta=np.array(json.dumps(meta)), **arrays)
    log(f"wrote {OUT}: {json.dumps(meta)}")
    if not all(meta[f"accepted_{r}"] for r in PICK):
        sys.exit(1)


if __name__ == "__main__":
    main()
