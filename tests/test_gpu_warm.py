"""GPU checks of the warm-started solve (lsqr_solve_x0) against the oracle
(oracle/warm.py): iterates at fixed step counts from a random start and from
a cold solve's iterate (FP64, with and without column scaling; LSMR), the
tolerance stop with eta kept in the original problem's terms, an exact start
that needs no step, device buffers (x0 may be dm), and the BF16 refinement
started from a looser FP64 solution.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import warm as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def from_sys(s, **k):
    from paper_2604_11920_amd import Solver
    return Solver.from_system(s, **k)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_system(synth.config0())


def explicit_eta(s, x):
    op = oracle.Operator.from_system(s)
    b = W.bbar_of(op, s.dt)
    return W.normal_residual(op, b, x) / W.normal_residual(op, b, np.zeros(s.n))


@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("start", ["random", "cold5"])
def test_warm_iterates_follow_oracle(cfg0, precond, start):
    s = cfg0
    d = oracle.Operator.from_system(s).jacobi() if precond == "jacobi" else None
    op = oracle.Operator.from_system(s, d=d)
    if start == "random":
        x0 = 0.05 * np.random.default_rng(4).standard_normal(s.n)
    else:
        x0 = op.lsqr(s.dt, 5)["x"]
    with from_sys(s, precond=precond) as sol:
        for K in (1, 3, 8):
            ref = W.warm(op, s.dt, x0, K)
            dm, hist, info = sol.solve(s.dt, K, x0=x0)
            assert info["iters"] == K and info["istop"] == 2
            assert rel(dm, ref["x"]) <= 1e-10, (K, rel(dm, ref["x"]))


def test_warm_lsmr_iterates_follow_oracle(cfg0):
    s = cfg0
    op = oracle.Operator.from_system(s)
    x0 = op.lsqr(s.dt, 4)["x"]
    with from_sys(s, method="lsmr") as sol:
        for K in (1, 3, 6):
            ref = W.warm(op, s.dt, x0, K, method="lsmr")
            dm, hist, info = sol.solve(s.dt, K, x0=x0)
            assert rel(dm, ref["x"]) <= 1e-10, (K, rel(dm, ref["x"]))


@pytest.mark.parametrize("method", ["lsqr", "lsmr"])
def test_warm_tolerance_stop_keeps_eta_meaning(cfg0, method):
    # a looser solve, then a warm restart to the tighter tolerance: the stop
    # eta is the original problem's, and the restart takes fewer steps than
    # a cold solve to the same tolerance
    s = cfg0
    with from_sys(s, precond="jacobi", method=method) as sol:
        x1, _, i1 = sol.solve(s.dt, 20000, tol=1e-4)
        dm, hist, info = sol.solve(s.dt, 20000, tol=1e-8, x0=x1)
        dc, _, ic = sol.solve(s.dt, 20000, tol=1e-8)
    assert info["istop"] == 1 and info["eta"] <= 1e-8
    if method == "lsqr":
        # LSQR's eta is the unscaled normal-equation residual: re-check it
        assert explicit_eta(s, dm) <= 3e-8
    assert info["iters"] < ic["iters"]
    # both stopped at eta <= 1e-8; their distance is bounded by the
    # conditioning (cond(Abar^T Abar) ~ 1e3 with the Jacobi scale) times eta
    assert rel(dm, dc) <= 1e-4
    print(f"[{method}] cold {ic['iters']} iterations; warm from eta 1e-4: {i1['iters']} + "
          f"{info['iters']}")


def test_exact_start_and_device_aliasing(cfg0):
    s = cfg0
    dt = torch.from_numpy(s.dt).cuda()
    with from_sys(s, precond="jacobi") as sol:
        xs, _, _ = sol.solve(dt, 20000, tol=1e-13)
        # started at the solution: at most one step, same solution
        x2, _, info = sol.solve(dt, 50, tol=1e-10, x0=xs.clone())
        assert info["iters"] <= 1 and info["eta"] <= 1e-10
        assert rel(x2.cpu().numpy(), xs.cpu().numpy()) <= 1e-10
        # x0 and dm the same device buffer
        x0 = 0.01 * torch.ones(s.n, dtype=torch.float64, device="cuda")
        ref, _, _ = sol.solve(dt, 5, x0=x0.clone())
        out, _, _ = sol.solve(dt, 5, dm=x0, x0=x0)
        assert out.data_ptr() == x0.data_ptr()
        assert torch.equal(out, ref)


def test_warm_rejections(cfg0):
    from paper_2604_11920_amd import LsqrError
    with from_sys(cfg0) as sol:
        x0 = np.full(cfg0.n, np.nan)
        with pytest.raises(LsqrError):
            sol.solve(cfg0.dt, 5, x0=x0)


def test_bf16_refinement_from_fp64_start(cfg0):
    s = cfg0
    with from_sys(s, precond="jacobi") as sol:
        x1, _, _ = sol.solve(s.dt, 20000, tol=1e-4)
        xs, _, _ = sol.solve(s.dt, 40000, tol=1e-12)
    with from_sys(s, precision="bf16", precond="jacobi", refine_sweeps=10) as sol:
        dm, _, info = sol.solve(s.dt, 3000, tol=1e-7, x0=x1)
        dc, _, ic = sol.solve(s.dt, 3000, tol=1e-7)
    assert info["istop"] == 1 and info["eta"] <= 1e-7
    assert rel(dm, xs) <= 1e-5
    assert info["iters"] <= ic["iters"]
    print(f"[bf16] cold {ic['iters']} inner iterations ({ic['sweeps']} sweeps); from the "
          f"1e-4 FP64 solution {info['iters']} ({info['sweeps']} sweeps)")


def test_fp32_warm_iterates(cfg0):
    # FP32 vectors and values, FP64 scalars: the early-iterate bar of the FP32
    # form (1e-4), from the FP64 oracle's 4-step iterate
    s = cfg0
    op = oracle.Operator.from_system(s)
    x0 = op.lsqr(s.dt, 4)["x"]
    with from_sys(s, precision="fp32") as sol:
        for K in (1, 3, 5):
            ref = W.warm(op, s.dt, x0, K)
            dm, hist, info = sol.solve(s.dt, K, x0=x0)
            assert info["iters"] == K
            assert rel(dm, ref["x"]) <= 1e-4, (K, rel(dm, ref["x"]))
