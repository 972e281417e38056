"""Write the oracle's converged solution of an ill-conditioned variant of the
small system (config 0's geometry and data, damping 1e-3, smoothing weight
0.01) to tests/golden/cfg0_illcond.npz.

Only oracle/ computes anything here (synth/ supplies the inputs): LSQR in
FP64 with the Jacobi column scale and Neumaier-compensated sums, run to
eta <= 1e-12; the result is accepted only if the eta <= 1e-11 solution agrees
with it to 1e-7, so the reference is far tighter than the 1e-5 bar the
reduced-precision forms are held to.  A fingerprint of the generated system
is stored with it, so the test can check that the generator reproduced the
same system.

Usage: python tests/golden/make_illcond_golden.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

DAMP, SMOOTH = 1e-3, 0.01


def system():
    c = synth.config0()
    c.damp, c.smooth = DAMP, SMOOTH
    return synth.make_system(c)


def main():
    s = system()
    op = oracle.Operator.from_system(s)
    scaled = oracle.Operator.from_system(s, d=op.jacobi(), compensated=True)
    r12 = scaled.lsqr(s.dt, 100000, tol=1e-12)
    r11 = scaled.lsqr(s.dt, 100000, tol=1e-11)
    assert r12["istop"] == 1 and r11["istop"] == 1, (r12["istop"], r11["istop"])
    d = np.linalg.norm(r12["x"] - r11["x"]) / np.linalg.norm(r12["x"])
    print(f"x*: {r12['iters']} iterations to eta <= 1e-12; the 1e-11 solution differs by {d:.2e}")
    assert d <= 1e-7
    np.savez(os.path.join(HERE, "cfg0_illcond.npz"), xstar=r12["x"], iters=r12["iters"],
             damp=DAMP, smooth=SMOOTH, fingerprint=synth.fingerprint(s))


if __name__ == "__main__":
    main()
