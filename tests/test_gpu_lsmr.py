"""GPU parity of LSMR (the paper's solver, Fong & Saunders 2011) against the
LSMR oracle (oracle/lsmr.py), with the same bars as the LSQR path: early
iterates and histories to 1e-10, converged solutions to 1e-10, the method's
monotone |A^T r| on the GPU, FP32 to 1e-4, and the mixed forms' refinement
with LSMR inner solves reaching the FP64 solution.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle.lsmr import lsmr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def from_sys(s, **k):
    from paper_2604_11920_amd import Solver
    return Solver.from_system(s, method="lsmr", **k)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_system(synth.config0())


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_early_iterates_strict(cfg0, precond):
    s = cfg0
    d = oracle.Operator.from_system(s).jacobi() if precond == "jacobi" else None
    op = oracle.Operator.from_system(s, d=d)
    with from_sys(s, precond=precond) as sol:
        for K in (1, 2, 3, 5, 8):
            ref = lsmr(op, s.dt, K)
            dm, hist, info = sol.solve(s.dt, K)
            assert info["iters"] == K and info["istop"] == 2
            assert rel(dm, ref["x"]) <= 1e-10, (K, rel(dm, ref["x"]))
            assert np.allclose(hist, ref["hist"], rtol=1e-10, atol=0), K


def test_converged_strict(cfg0):
    s = cfg0
    op = oracle.Operator.from_system(s)
    ref = lsmr(op, s.dt, 40000, tol=1e-13)
    xs = oracle.lsqr(s, 40000, tol=1e-13)["x"]
    with from_sys(s) as sol:
        dm, hist, info = sol.solve(s.dt, 40000, tol=1e-13)
    assert info["istop"] == 1 and ref["istop"] == 1 and info["eta"] <= 1e-13
    assert rel(dm, ref["x"]) <= 1e-10
    assert rel(dm, xs) <= 1e-9              # LSQR's and LSMR's common limit
    assert abs(info["iters"] - ref["iters"]) <= 0.1 * ref["iters"] + 2


def test_normal_residual_monotone(cfg0):
    with from_sys(cfg0) as sol:
        dm, hist, info = sol.solve(cfg0.dt, 300)
    assert info["iters"] == 300
    assert np.all(np.diff(hist[:, 1]) <= 1e-12 * hist[0, 1])
    assert np.all(np.diff(hist[:, 0]) <= 1e-12 * hist[0, 0])


def test_ragged_and_small_shapes():
    s = synth.random_system(700, 6, 5, 4, row_len=(0, 60), seed=21)
    for K in (1, 4, 8):
        ref = lsmr(oracle.Operator.from_system(s), s.dt, K)
        with from_sys(s) as sol:
            dm, _, _ = sol.solve(s.dt, K)
        assert rel(dm, ref["x"]) <= 1e-10, K
    for grid in [(1, 1, 1), (1, 1, 3), (3, 2, 1)]:
        s = synth.random_system(25, *grid, row_len=(0, 4), seed=sum(grid))
        ref = lsmr(oracle.Operator.from_system(s), s.dt, 3)
        with from_sys(s) as sol:
            dm, _, info = sol.solve(s.dt, 3)
        assert rel(dm, ref["x"]) <= 1e-10 or info["istop"] in (1, 3), grid


def test_fp32_iterates(cfg0):
    ref = lsmr(oracle.Operator.from_system(cfg0), cfg0.dt, 5)
    with from_sys(cfg0, precision="fp32") as sol:
        dm, hist, info = sol.solve(cfg0.dt, 5)
    assert info["iters"] == 5 and rel(dm, ref["x"]) <= 1e-4


def test_bf16_refinement_with_lsmr_inner_solves(cfg0):
    op = oracle.Operator.from_system(cfg0)
    xs = oracle.Operator.from_system(cfg0, d=op.jacobi(), compensated=True).lsqr(
        cfg0.dt, 40000, tol=1e-12)["x"]
    # LSMR drives |A^T r| down faster than the error in the small singular
    # directions (LSQR's error, not LSMR's, decreases monotonically), so the
    # same error needs a tighter eta than with LSQR inner solves (still above
    # the refinement's FP32 floor of a few 1e-9)
    with from_sys(cfg0, precision="bf16", precond="jacobi", refine_sweeps=10,
                  refine_inner_tol=1e-3) as sol:
        dm, hist, info = sol.solve(cfg0.dt, 3000, tol=1e-8)
    print(f"[bf16/lsmr] sweeps={info['sweeps']} iters={info['iters']} eta={info['eta']:.2e} "
          f"err={rel(dm, xs):.2e}")
    assert info["istop"] in (1, 4) and rel(dm, xs) <= 1e-5


def test_degenerate_right_hand_side(cfg0):
    with from_sys(cfg0) as sol:
        dm, hist, info = sol.solve(np.zeros(cfg0.m), 10)
    assert info["istop"] == 0 and np.all(dm == 0)
