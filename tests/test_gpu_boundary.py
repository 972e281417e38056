"""GPU checks of the stopping ratio verified at exit and of the learned-scale
fallback inside the library.

* info.eta_final_fp64 is |Abar^T (bbar - Abar dm)| / |Abar^T bbar| of the
  returned dm in the original variables (the tolerance of the solver
  section's normal-equation stopping rule), recomputed with the FP64
  operator: it equals a SciPy evaluation of the same ratio on the host, for
  LSQR and LSMR with and without column scaling and for the BF16 form; it is
  NaN for fixed iteration counts.
* A user scale that has not converged within opts.fallback_iters iterations
  is replaced by Jacobi inside the solve, which continues from its iterate
  and converges to the same solution; the context keeps the user scale.
"""
import math

import numpy as np
import pytest

import synth
from _helpers import eta_explicit, sparse_abar

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def sysA():
    return synth.make_system(synth.small_config(nx=10, ny=9, nz=7, n_stations=18, n_periods=6,
                                                region=0.9, seed=11))


def from_sys(s, **k):
    from paper_2604_11920_amd import Solver
    return Solver.from_system(s, **k)


@pytest.mark.parametrize("kw", [dict(), dict(precond="jacobi"), dict(method="lsmr"),
                                dict(precond="jacobi", method="lsmr"),
                                dict(precision="fp32", precond="jacobi"),
                                dict(precision="bf16", precond="jacobi")])
def test_eta_final_fp64_is_the_explicit_ratio(sysA, kw):
    s = sysA
    A = sparse_abar(s)
    tol = 1e-5 if kw.get("precision") == "fp32" else 1e-7     # FP32 stalls near 1e-6
    print(f"eta_final: {kw}", flush=True)
    with from_sys(s, **kw) as sol:
        dm, _, info = sol.solve(s.dt, 4000, tol=tol, history=False)
    eta, _ = eta_explicit(s, dm, A)
    assert info["istop"] == 1, info
    assert math.isfinite(info["eta_final_fp64"])
    # the two evaluations differ only by rounding of a ratio that is itself
    # ~tol: relative agreement to ~1e-6 of the ratio
    assert abs(info["eta_final_fp64"] - eta) <= 1e-6 * eta + 1e-15, (info["eta_final_fp64"], eta)
    if kw.get("precision") == "bf16":
        assert info["eta_final_fp64"] == info["eta"]
    if kw.get("method") != "lsmr" and kw.get("precision") != "fp32":
        # LSMR's own eta is in scaled variables; FP32's estimate drifts from
        # the FP64 value by its rounding
        assert info["eta_final_fp64"] <= tol * 1.01


def test_eta_final_fp64_nan_for_fixed_count(sysA):
    with from_sys(sysA) as sol:
        _, _, info = sol.solve(sysA.dt, 20, history=False)
    assert info["istop"] == 2 and math.isnan(info["eta_final_fp64"])


def test_fallback_to_jacobi_inside_the_library(sysA):
    s = sysA
    tol = 1e-8
    with from_sys(s, precond="jacobi") as sol:
        xj, _, ij = sol.solve(s.dt, 20000, tol=tol, history=False)
        djac = sol.scale()
    kj = ij["iters"]
    # a valid but poor scale: Jacobi times factors spread over six decades
    rng = np.random.default_rng(5)
    bad = djac * 10.0 ** rng.uniform(-3, 3, s.n)
    with from_sys(s, precond="user", col_scale=bad, fallback_iters=2 * kj) as sol:
        xb, _, ib = sol.solve(s.dt, 20000, tol=tol, history=False)
        kept = sol.scale()
    print(f"fallback: jacobi {kj} iterations; bad scale with fallback {ib}", flush=True)
    assert ib["fallback_used"] == 1 and ib["istop"] == 1
    assert ib["iters"] > 2 * kj                     # the failed attempt is counted
    assert ib["eta_final_fp64"] <= tol * 1.01
    assert np.array_equal(kept, bad)                # the user scale is restored
    assert np.linalg.norm(xb - xj) / np.linalg.norm(xj) <= 1e-5
    # without a budget the same scale runs on (no fallback)
    with from_sys(s, precond="user", col_scale=bad) as sol:
        _, _, ic = sol.solve(s.dt, 2 * kj, tol=tol, history=False)
    assert ic["fallback_used"] == 0 and ic["istop"] == 2


def test_fallback_not_taken_when_the_scale_converges(sysA):
    s = sysA
    tol = 1e-8
    with from_sys(s, precond="jacobi") as sol:
        _, _, ij = sol.solve(s.dt, 20000, tol=tol, history=False)
        djac = sol.scale()
    with from_sys(s, precond="user", col_scale=djac * 2.0, fallback_iters=2 * ij["iters"]) as sol:
        _, _, iu = sol.solve(s.dt, 20000, tol=tol, history=False)
    assert iu["fallback_used"] == 0 and iu["istop"] == 1
    # a power-of-two factor scales every product exactly: the same iterations
    assert iu["iters"] == ij["iters"]


def test_fallback_bf16_refinement(sysA):
    s = sysA
    tol = 1e-8
    with from_sys(s, precond="jacobi") as sol:
        xj, _, ij = sol.solve(s.dt, 20000, tol=tol, history=False)
        djac = sol.scale()
    rng = np.random.default_rng(6)
    bad = djac * 10.0 ** rng.uniform(-3, 3, s.n)
    with from_sys(s, precision="bf16", precond="user", col_scale=bad, refine_sweeps=12,
                  fallback_iters=ij["iters"]) as sol:
        xb, _, ib = sol.solve(s.dt, 4000, tol=tol, history=False)
    print(f"bf16 fallback: {ib}", flush=True)
    assert ib["fallback_used"] == 1 and ib["istop"] == 1
    assert np.linalg.norm(xb - xj) / np.linalg.norm(xj) <= 1e-5
