"""The batched workload's largest system (config-1 geometry, 229 stations, 20
periods, generator seed 3; 565 M stored entries) with its 32 right-hand
sides (16 checkerboards of 2-8 cells, 16 noise draws), solved in one batched
call with FP64 refinement per right-hand side, in the schedule the
autotuner picks: every right-hand side stops at the tolerance, and the
selected ones lie within 1e-5 of the oracle's x* stored in
tests/golden/cfg3_largest.npz (written by tests/golden/make_cfg3_golden.py,
which calls only oracle/: Jacobi-scaled LSQR with compensated sums to
eta <= 1e-12)."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg3_largest.npz")
# two sweeps reach it for every right-hand side (eta 9e-9 .. 2.6e-8); it
# puts x within a few 1e-6 of x*
TOL = 5e-8


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_largest_batched_system_reaches_xstar():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2604_11920_amd import Solver, solve_batched_refined
    z = np.load(GOLDEN, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    s = synth.make_system(synth.config3_systems()[-1])
    assert meta["fingerprint"] == synth.fingerprint(s), "the stored results describe another system"
    rhs = synth.checker_rhs_batch(s)
    print(f"[cfg3-golden] m={s.m} n={s.n} nnz={s.nnz}, {rhs.shape[1]} right-hand sides",
          flush=True)
    with Solver.from_system(s, precond="jacobi") as sol:
        cfg = sol.autotune_batched(rhs.shape[1], probe_iters=8)
        dms, infos = solve_batched_refined([sol], [torch.from_numpy(rhs).cuda()], 4000, TOL,
                                           inner_tol=1e-4, sweeps=8)
    dm = dms[0].cpu().numpy()
    print("[cfg3-golden] istop / sweeps / inner iterations / eta per right-hand side: " +
          " ".join(f"{I['istop']}/{I['sweeps']}/{I['iters']}/{I['eta_final_fp64']:.1e}"
                   for I in infos[0]), flush=True)
    for r, I in enumerate(infos[0]):
        assert I["istop"] == 1 and I["eta_final_fp64"] <= TOL, (r, I)
    for r in meta["picked"]:
        assert meta[f"accepted_{r}"]
        e = rel(dm[:, r], z[f"x_star_{r}"])
        I = infos[0][r]
        print(f"[cfg3-golden] schedule {cfg}; rhs {r}: sweeps {I['sweeps']} inner iters "
              f"{I['iters']} eta {I['eta_final_fp64']:.2e} |x - x*|/|x*| {e:.2e}", flush=True)
        assert e <= 1e-5
