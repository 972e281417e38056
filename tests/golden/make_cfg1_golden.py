"""Write the oracle's reference results for the paper-shaped system (80x80x20
grid, 229 stations, 26,106 pairs x 20 periods, bent rays, paths of >= 2
wavelengths, generator seed 0) to tests/golden/cfg1_seed0.npz.

Only oracle/ computes anything here (synth/ supplies the inputs):

* the converged reference x*: LSQR (FP64, Jacobi column scale, Neumaier-
  compensated sums) run to eta <= 1e-12, or until eta stops improving for 200
  iterations; it is accepted only if the eta <= 1e-11 and eta <= 1e-12
  iterates agree to 1e-7 (the reference must be far tighter than the 1e-5
  bound the reduced-precision forms are held to);
* the fixed-count iterates: K = 3, 10, 30, 100 and 300 LSQR iterations
  without column scaling, once with plain and once with compensated sums
  (with the 300-iteration histories).  Their distance Delta_self(K) is the
  oracle's own sensitivity to summation order at that count, the envelope
  any other summation order can be held to.  The compensated iterates are
  stored; the plain ones enter only Delta_self.

A fingerprint of the generated system (sizes, row pointer, right-hand side and
a stride of the column indices and values) is stored with the results, so the
tests can check that the generator reproduced the same system.

Usage: python tests/golden/make_cfg1_golden.py [--threads 8] [--only fixed|xstar]
(--only recomputes one part and keeps the other from the existing file).
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

OUT = os.path.join(HERE, "cfg1_seed0.npz")


fingerprint = synth.fingerprint


def log(msg):
    print(f"[golden] {msg}", flush=True)


KS = (3, 10, 30, 100, 300)


def fixed_counts(s, threads):
    """x_K with plain and compensated sums for K in KS, and Delta_self(K)."""
    res, meta = {}, {}
    for comp in (False, True):
        t1 = time.time()
        op = oracle.Operator.from_system(s, compensated=comp, nthreads=threads)
        tag = "comp" if comp else "plain"
        for K in KS:
            r = op.lsqr(s.dt, K)
            res[f"x{K}_{tag}"] = r["x"]
            if K == KS[-1]:
                res[f"hist{K}_{tag}"] = r["hist"]
        del op
        log(f"fixed counts {KS}, {tag} sums: {time.time() - t1:.0f} s")
    for K in KS:
        xp, xc = res[f"x{K}_plain"], res[f"x{K}_comp"]
        meta[f"delta_self_{K}"] = float(np.linalg.norm(xp - xc) / np.linalg.norm(xc))
    hp, hc = res[f"hist{KS[-1]}_plain"], res[f"hist{KS[-1]}_comp"]
    meta[f"hist_self_{KS[-1]}"] = float(np.max(np.abs(hp[:, 0] - hc[:, 0]) / hc[:, 0]))
    log("Delta_self: " + ", ".join(f"K={K}: {meta[f'delta_self_{K}']:.3e}" for K in KS))
    return res, meta


def explicit_eta(s, x, threads):
    """|Abar^T (bbar - Abar x)| / |Abar^T bbar| with the unscaled oracle operator."""
    op = oracle.Operator.from_system(s, compensated=True, nthreads=threads)
    b = np.concatenate([s.dt, np.zeros(2 * s.n)])
    return float(np.linalg.norm(op.apply_t(b - op.apply(x))) / np.linalg.norm(op.apply_t(b)))


def reference(s, threads, cap):
    """x*: Jacobi-scaled LSQR with compensated sums to eta <= 1e-12 (or
    stagnation), accepted when the eta <= 1e-11 and final iterates agree to
    1e-7; its eta re-checked explicitly with the unscaled oracle operator."""
    t1 = time.time()
    op = oracle.Operator.from_system(s, nthreads=threads)
    d = op.jacobi()
    del op
    opj = oracle.Operator.from_system(s, d=d, compensated=True, nthreads=threads)
    r = opj.lsqr_ref(s.dt, cap, 1e-12, 1e-11, stall=200)
    del opj
    x_star, x11 = r["x"], r["x_snap"]
    gap = float(np.linalg.norm(x_star - x11) / np.linalg.norm(x_star))
    eta_end = float(r["hist"][-1, 2])
    accepted = bool(r["k_snap"] > 0 and gap <= 1e-7)
    eta_true = explicit_eta(s, x_star, threads)
    log(f"x*: {r['iters']} iterations, istop {r['istop']}, eta {eta_end:.3e} (explicit "
        f"{eta_true:.3e}), eta<=1e-11 at {r['k_snap']}, gap {gap:.3e}, accepted {accepted} "
        f"({time.time() - t1:.0f} s)")
    res = dict(x_star=x_star, xstar_eta_hist=r["hist"][:, 2].copy())
    meta = dict(xstar_iters=int(r["iters"]), xstar_istop=int(r["istop"]), xstar_eta=eta_end,
                xstar_eta_explicit=eta_true, xstar_k11=int(r["k_snap"]), xstar_gap_11_12=gap,
                xstar_accepted=accepted)
    return res, meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--cap", type=int, default=40000)
    ap.add_argument("--only", choices=["fixed", "xstar"], default=None)
    args = ap.parse_args()
    t0 = time.time()
    s = synth.make_system(synth.config1(seed=0))
    fp = fingerprint(s)
    log(f"system m={s.m} n={s.n} nnz={s.nnz} fingerprint {fp[:16]} ({time.time() - t0:.0f} s)")
    arrays, meta = {}, {}
    if args.only:
        z = np.load(OUT, allow_pickle=False)
        old = json.loads(str(z["meta"]))
        assert old["fingerprint"] == fp, "the existing file describes another system"
        arrays = {k: z[k] for k in z.files if k != "meta"}
        meta = old
    if args.only in (None, "fixed"):
        a, mt = fixed_counts(s, args.threads)
        arrays.update(a)
        meta.update(mt)
    if args.only in (None, "xstar"):
        a, mt = reference(s, args.threads, args.cap)
        arrays.update(a)
        meta.update(mt)
    elif "xstar_eta_explicit" not in meta:
        meta["xstar_eta_explicit"] = explicit_eta(s, arrays["x_star"], args.threads)
        log(f"x*: explicit eta {meta['xstar_eta_explicit']:.3e}")
    meta.update(fingerprint=fp, m=int(s.m), n=int(s.n), nnz=int(s.nnz), threads=args.threads,
                seconds=round(time.time() - t0, 1))
    # stored: the compensated iterates (the plain ones only enter Delta_self)
    arrays = {k: v for k, v in arrays.items() if not k.endswith("_plain")}
    np.savez(OUT, meta=np.array(json.dumps(meta)), **arrays)
    log(f"wrote {OUT}: {json.dumps(meta)}")
    if not meta.get("xstar_accepted", False):
        sys.exit(1)


if __name__ == "__main__":
    main()
