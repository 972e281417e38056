"""Pins of the LSMR oracle (oracle/lsmr.py) against what mathematics fixes
(no GPU): the MINRES-on-normal-equations definition by Krylov brute force,
dense least squares at convergence, closed forms, SciPy's LSMR (on the
explicit block operator, and with its own internal damping on [G; w L]), and
the method's invariants — both |r_k| and |A^T r_k| non-increasing, the
estimates equal to the explicit residuals, LSQR's and LSMR's common limit.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle.lsmr import lsmr
from test_oracle_pins import bbar, dense_abar, diag_system, rel


@pytest.fixture(scope="module")
def tiny():
    return synth.random_system(60, 2, 2, 5, row_len=(1, 8), seed=11, damp=0.1, smooth=0.5)


@pytest.fixture(scope="module")
def small_geo():
    return synth.make_system(synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4,
                                                region=0.5))


def run(s, k, tol=0.0, d=None):
    return lsmr(oracle.Operator.from_system(s, d=d), s.dt, k, tol)


def test_minres_on_normal_equations_bruteforce(small_geo):
    # x_k minimises |A^T (b - A x)| over K_k(A^T A, A^T b): an orthonormal
    # Krylov basis (Gram-Schmidt twice) and a dense least-squares solve
    A, b = dense_abar(small_geo), bbar(small_geo)
    M = A.T @ A
    g = A.T @ b
    V = np.zeros((small_geo.n, 0))
    vec = g.copy()
    for k in range(1, 9):
        for _ in range(2):
            vec = vec - V @ (V.T @ vec)
        V = np.hstack([V, (vec / np.linalg.norm(vec))[:, None]])
        c = np.linalg.lstsq(M @ V, g, rcond=None)[0]
        xk = V @ c
        assert rel(run(small_geo, k)["x"], xk) < (1e-11 if k <= 6 else 1e-9), k
        vec = M @ V[:, -1]


def test_converged_matches_dense_least_squares(tiny, small_geo):
    for s in (tiny, small_geo):
        A, b = dense_abar(s), bbar(s)
        xs = np.linalg.lstsq(A, b, rcond=None)[0]
        r = run(s, 20000, tol=1e-14)
        assert r["istop"] == 1
        assert rel(r["x"], xs) < 1e-10


def test_diagonal_closed_form():
    n = 24
    g = np.array([1.0, 2.0, 3.0] * 8)
    b = np.random.default_rng(5).standard_normal(n)
    lam = 0.1
    s = diag_system(g, b, lam, (2, 3, 4))
    exact = g * b / (g * g + lam * lam)
    # three distinct singular values: the Krylov space holds x* after 3 steps
    assert rel(run(s, 3)["x"], exact) < 1e-13
    # Jacobi scaling makes (Abar D)^T (Abar D) = I: exact after 1 step
    d = oracle.Operator.from_system(s).jacobi()
    assert rel(run(s, 1, d=d)["x"], exact) < 1e-14


def test_single_column_closed_form():
    g = np.array([0.5, -1.0, 2.0, 3.0, 0.25, -0.75, 1.5])
    b = np.array([1.0, 2.0, -1.0, 0.5, 4.0, -2.0, 0.0])
    s = synth.RandomSystem(m=7, n=1, nx=1, ny=1, nz=1, row_ptr=np.arange(8, dtype=np.int64),
                           col=np.zeros(7, dtype=np.int32), val=g, dt=b, damp=0.3, smooth=0.5)
    assert abs(run(s, 1)["x"][0] - g @ b / (g @ g + 0.09)) < 1e-15


def test_scipy_lsmr_explicit_and_damped(small_geo):
    s = small_geo
    A = sp.csr_matrix(dense_abar(s))
    b = bbar(s)
    G = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.m, s.n))
    from _helpers import laplacian
    Aw = sp.vstack([G, s.smooth * laplacian(s.nx, s.ny, s.nz)]).tocsr()
    bw = np.r_[s.dt, np.zeros(s.n)]
    for k in (1, 2, 4, 8):
        ours = run(s, k)["x"]
        ref = spla.lsmr(A, b, atol=0, btol=0, conlim=0, maxiter=k)[0]
        # two valid summation orders: agreement degrades with k as
        # orthogonality is lost (as for LSQR)
        assert rel(ours, ref) < (1e-12 if k <= 4 else 1e-10), k
        # SciPy's own damping on [G; w L] spans the same Krylov spaces
        refd = spla.lsmr(Aw, bw, damp=s.damp, atol=0, btol=0, conlim=0, maxiter=k)[0]
        assert rel(ours, refd) < 1e-10, k


def test_lsmr_invariants(small_geo, tiny):
    for s in (small_geo, tiny):
        A, b = dense_abar(s), bbar(s)
        K = 25
        out = run(s, K)
        hist = out["hist"]
        rn, arn = [], []
        for k in range(1, K + 1):
            x = run(s, k)["x"]
            r = b - A @ x
            rn.append(np.linalg.norm(r))
            arn.append(np.linalg.norm(A.T @ r))
            # the recurrences' estimates are the explicit norms
            assert abs(hist[k, 0] - rn[-1]) <= 1e-8 * rn[0], k
            assert abs(hist[k, 1] - arn[-1]) <= 1e-8 * arn[0] + 1e-12 * hist[0, 1], k
        # LSMR: both |r_k| and |A^T r_k| are monotone
        assert np.all(np.diff(rn) <= 1e-12 * rn[0])
        assert np.all(np.diff(arn) <= 1e-12 * arn[0])
        assert np.allclose(hist[1:, 2], hist[1:, 1] / hist[0, 1], rtol=1e-15)


def test_same_solution_as_lsqr(cfg0_system):
    s = cfg0_system
    a = run(s, 20000, tol=1e-12)
    b = oracle.lsqr(s, 20000, tol=1e-12)
    assert a["istop"] == 1 and b["istop"] == 1
    assert rel(a["x"], b["x"]) < 1e-8
    # LSMR's |A^T r| is monotone while LSQR's is not; LSMR needs no more
    # iterations than LSQR to the same normal-equation tolerance (here, up to 10 %)
    assert a["iters"] <= 1.1 * b["iters"]


def test_breakdowns_and_zero_rhs(tiny):
    s = tiny
    r = lsmr(oracle.Operator.from_system(s), np.zeros(s.m), 10)
    assert r["istop"] == 0 and np.all(r["x"] == 0)
    # n = 1: the bidiagonalisation ends after one step
    g = np.array([1.0, 2.0, 2.0])
    s1 = synth.RandomSystem(m=3, n=1, nx=1, ny=1, nz=1, row_ptr=np.arange(4, dtype=np.int64),
                            col=np.zeros(3, dtype=np.int32), val=g, dt=np.array([1.0, 0.0, 1.0]),
                            damp=0.0, smooth=0.0)
    # (alpha_2 = 0 in exact arithmetic, a rounding-level value in practice)
    assert abs(run(s1, 1)["x"][0] - 3.0 / 9.0) < 1e-15
    r5 = run(s1, 5)
    assert r5["istop"] in (2, 3) and abs(r5["x"][0] - 3.0 / 9.0) < 1e-12
