"""GPU checks of the batched solve with FP64 refinement per right-hand side
(lsqr_solve_batched_refined): FP32 values and vectors in every sweep's
batched LSQR, the residual, the correction (G - Ghat)^T r_G and the stopping
ratio in FP64.

Expected values: x* of every selected right-hand side from the oracle
(FP64, Jacobi column scale, compensated sums, run to eta <= 1e-12), one
system at a time.  Bar: 1e-5 relative (the reduced-precision forms' bar
after refinement), with istop 1 and the FP64 eta of the returned solution at
the tolerance.  The batched solve without refinement is reported beside it:
FP32 rounding of G alone moves its fixed point well beyond that bar.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-7
PICK = (0, 5, 15, 16, 31)          # checkerboards of 2, 4 and 8 cells, two noise draws


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def systems():
    """Two uneven systems (the small survey and a smaller bent-ray survey on
    another grid), 32 right-hand sides each: 16 checkerboards, 16 noise
    draws."""
    out = []
    for s in (synth.make_system(synth.config0()),
              synth.make_system(synth.small_config(nx=12, ny=11, nz=7, n_stations=24,
                                                   n_periods=6, region=1.1, seed=5))):
        out.append((s, synth.checker_rhs_batch(s)))
    return out


@pytest.fixture(scope="module")
def xstars(systems):
    res = []
    for s, rhs in systems:
        d = oracle.Operator.from_system(s, nthreads=8).jacobi()
        op = oracle.Operator.from_system(s, d=d, compensated=True, nthreads=8)
        xs = {}
        for r in PICK:
            out = op.lsqr(rhs[:, r], 40000, tol=1e-12)
            assert out["istop"] == 1
            xs[r] = out["x"]
        res.append(xs)
    return res


def test_refined_batch_reaches_xstar(systems, xstars):
    from paper_2604_11920_amd import Solver, solve_batched, solve_batched_refined
    sols = [Solver.from_system(s, precond="jacobi") for s, _ in systems]
    try:
        dts = [rhs for _, rhs in systems]
        dms, infos = solve_batched_refined(sols, dts, 3000, TOL, inner_tol=1e-4, sweeps=8)
        plain, _, pinfo = solve_batched(sols, dts, 3000, tol=TOL, history=False)
    finally:
        for so in sols:
            so.close()
    for k, ((s, rhs), xs) in enumerate(zip(systems, xstars)):
        for r in range(rhs.shape[1]):
            I = infos[k][r]
            assert I["istop"] == 1 and I["eta_final_fp64"] <= TOL, (k, r, I)
            assert I["sweeps"] >= 1
        for r in PICK:
            e, ep = rel(dms[k][:, r], xs[r]), rel(plain[k][:, r], xs[r])
            print(f"[batched-refined] system {k} rhs {r}: sweeps {infos[k][r]['sweeps']} inner "
                  f"iters {infos[k][r]['iters']} eta {infos[k][r]['eta_final_fp64']:.2e} "
                  f"|x - x*|/|x*| {e:.2e} (no refinement: {ep:.2e})", flush=True)
            assert e <= 1e-5
            assert e < ep


def test_refined_batch_padding_and_zero_rhs(systems):
    """nrhs not a power of two; a zero right-hand side stops at once with
    x = 0 (istop 0) and leaves the others unchanged."""
    from paper_2604_11920_amd import Solver, solve_batched_refined
    s, rhs = systems[1]
    sub = rhs[:, :5].copy()
    sub[:, 2] = 0.0
    with Solver.from_system(s, precond="jacobi") as so:
        dms, infos = solve_batched_refined([so], [sub], 3000, TOL)
        full, finfo = solve_batched_refined([so], [rhs[:, :5]], 3000, TOL)
    assert infos[0][2]["istop"] == 0 and np.all(dms[0][:, 2] == 0.0)
    for r in (0, 1, 3, 4):
        assert infos[0][r]["istop"] == 1
        assert np.array_equal(dms[0][:, r], full[0][:, r])


def test_refined_batch_rejections(systems):
    from paper_2604_11920_amd import LsqrError, Solver, solve_batched_refined
    s, rhs = systems[1]
    with Solver.from_system(s) as so:
        with pytest.raises(LsqrError):
            solve_batched_refined([so], [rhs[:, :2]], 100, 0.0)
        with pytest.raises(LsqrError):
            solve_batched_refined([so], [rhs[:, :2]], 100, 1e-6, inner_tol=1.5)
        with pytest.raises(LsqrError):
            solve_batched_refined([so], [rhs[:, :2]], 100, 1e-6, sweeps=0)
    with Solver.from_system(s, damp=0.0) as so:
        with pytest.raises(LsqrError):
            solve_batched_refined([so], [rhs[:, :2]], 100, 1e-6)
