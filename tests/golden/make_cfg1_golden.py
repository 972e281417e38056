"""Write the oracle's reference results for the paper-shaped system (80x80x20
grid, 229 stations, 26,106 pairs x 20 periods, bent rays, paths of >= 2
wavelengths, generator seed 0) to tests/golden/cfg1_seed0.npz.

Only oracle/ computes anything here (synth/ supplies the inputs):

* the converged reference x*: LSQR (FP64, Jacobi column scale, Neumaier-
  compensated sums) run to eta <= 1e-12, or until eta stops improving for 200
  iterations; it is accepted only if the eta <= 1e-11 and eta <= 1e-12
  iterates agree to 1e-7 (the reference must be far tighter than the 1e-5
  bound the reduced-precision forms are held to);
* the fixed-count iterates: 300 LSQR iterations without column scaling, once
  with plain and once with compensated sums, with their histories.  Their
  distance Delta_self(300) is the oracle's own sensitivity to summation order
  at that count, the envelope any other summation order can be held to.

A fingerprint of the generated system (sizes, row pointer, right-hand side and
a stride of the column indices and values) is stored with the results, so the
tests can check that the generator reproduced the same system.

Usage: python tests/golden/make_cfg1_golden.py [--threads 8]
"""
from __future__ import annotations

import argparse
import hashlib
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

OUT = os.path.join(HERE, "cfg1_seed0.npz")


def fingerprint(s) -> str:
    h = hashlib.sha256()
    h.update(np.array([s.m, s.n, s.nnz], dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(s.row_ptr).tobytes())
    h.update(np.ascontiguousarray(s.dt).tobytes())
    h.update(np.ascontiguousarray(s.col[::997]).tobytes())
    h.update(np.ascontiguousarray(s.val[::997]).tobytes())
    return h.hexdigest()


def log(msg):
    print(f"[golden] {msg}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--cap", type=int, default=40000)
    args = ap.parse_args()
    t0 = time.time()
    s = synth.make_system(synth.config1(seed=0))
    fp = fingerprint(s)
    log(f"system m={s.m} n={s.n} nnz={s.nnz} fingerprint {fp[:16]} ({time.time() - t0:.0f} s)")

    res = {}
    for comp in (False, True):
        t1 = time.time()
        op = oracle.Operator.from_system(s, compensated=comp, nthreads=args.threads)
        r = op.lsqr(s.dt, 300)
        del op
        tag = "comp" if comp else "plain"
        res[f"x300_{tag}"] = r["x"]
        res[f"hist300_{tag}"] = r["hist"]
        log(f"300 iterations, {tag} sums: {time.time() - t1:.0f} s")
    xp, xc = res["x300_plain"], res["x300_comp"]
    delta_self = float(np.linalg.norm(xp - xc) / np.linalg.norm(xc))
    hist_self = float(np.max(np.abs(res["hist300_plain"][:, 0] - res["hist300_comp"][:, 0])
                             / res["hist300_comp"][:, 0]))
    log(f"Delta_self(300) = {delta_self:.3e} in x, {hist_self:.3e} in the residual history")

    t1 = time.time()
    op = oracle.Operator.from_system(s, nthreads=args.threads)
    d = op.jacobi()
    del op
    opj = oracle.Operator.from_system(s, d=d, compensated=True, nthreads=args.threads)
    r = opj.lsqr_ref(s.dt, args.cap, 1e-12, 1e-11, stall=200)
    del opj
    x_star, x11 = r["x"], r["x_snap"]
    gap = float(np.linalg.norm(x_star - x11) / np.linalg.norm(x_star))
    eta_end = float(r["hist"][-1, 2])
    accepted = bool(r["k_snap"] > 0 and gap <= 1e-7)
    log(f"x*: {r['iters']} iterations, istop {r['istop']}, eta {eta_end:.3e}, eta<=1e-11 at "
        f"{r['k_snap']}, gap {gap:.3e}, accepted {accepted} ({time.time() - t1:.0f} s)")

    meta = dict(fingerprint=fp, m=int(s.m), n=int(s.n), nnz=int(s.nnz),
                delta_self_300=delta_self, hist_self_300=hist_self,
                xstar_iters=int(r["iters"]), xstar_istop=int(r["istop"]),
                xstar_eta=eta_end, xstar_k11=int(r["k_snap"]), xstar_gap_11_12=gap,
                xstar_accepted=accepted, threads=args.threads,
                seconds=round(time.time() - t0, 1))
    np.savez(OUT, x_star=x_star, x300_plain=xp, x300_comp=xc,
             hist300_plain=res["hist300_plain"], hist300_comp=res["hist300_comp"],
             xstar_eta_hist=r["hist"][:, 2].copy(), meta=np.array(json.dumps(meta)))
    log(f"wrote {OUT}: {json.dumps(meta)}")
    if not accepted:
        sys.exit(1)


if __name__ == "__main__":
    main()
