"""Pins of the warm-start oracle (oracle/warm.py) against what mathematics
fixes (no GPU): the Krylov characterisation of LSQR started from x0 (dense
brute force), the dense least-squares solution reached from any x0 (with and
without column scaling), the cold start as the special case x0 = 0 (against
the independent C LSQR oracle), an exact start that needs no step, the
closed form of a diagonal system, and the LSMR form's correction problem
against SciPy's LSMR.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import warm as W
from test_oracle_pins import bbar, dense_abar, diag_system, rel


@pytest.fixture(scope="module")
def tiny():
    return synth.random_system(60, 2, 2, 5, row_len=(1, 8), seed=11, damp=0.1, smooth=0.5)


@pytest.fixture(scope="module")
def small_geo():
    return synth.make_system(synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4,
                                                region=0.5))


def test_warm_iterates_minimise_over_shifted_krylov_space(small_geo):
    # x_k = x0 + argmin over K_k(A^T A, A^T r0) of |r0 - A y| (orthonormal basis
    # by Gram-Schmidt twice, dense least squares)
    s = small_geo
    A, b = dense_abar(s), bbar(s)
    x0 = np.random.default_rng(3).standard_normal(s.n)
    r0 = b - A @ x0
    M, g = A.T @ A, A.T @ r0
    op = oracle.Operator.from_system(s)
    V = np.zeros((s.n, 0))
    vec = g.copy()
    for k in range(1, 8):
        for _ in range(2):
            vec = vec - V @ (V.T @ vec)
        V = np.hstack([V, (vec / np.linalg.norm(vec))[:, None]])
        c = np.linalg.lstsq(A @ V, r0, rcond=None)[0]
        xk = x0 + V @ c
        assert rel(W.warm(op, s.dt, x0, k)["x"], xk) < (1e-11 if k <= 5 else 1e-9), k
        vec = M @ V[:, -1]


@pytest.mark.parametrize("scaled", [False, True])
def test_warm_converges_to_dense_least_squares(tiny, small_geo, scaled):
    for s in (tiny, small_geo):
        A, b = dense_abar(s), bbar(s)
        xs = np.linalg.lstsq(A, b, rcond=None)[0]
        d = oracle.Operator.from_system(s).jacobi() if scaled else None
        op = oracle.Operator.from_system(s, d=d)
        x0 = 10.0 * np.random.default_rng(7).standard_normal(s.n)
        r = W.warm(op, s.dt, x0, 20000, tol=1e-13)
        assert r["istop"] == 1 and r["eta"] <= 1e-13
        assert rel(r["x"], xs) < 1e-9
        # the explicit eta is the one of the original problem
        eta = np.linalg.norm(A.T @ (b - A @ r["x"])) / np.linalg.norm(A.T @ b)
        assert abs(eta - r["eta"]) <= 1e-3 * r["eta"] + 1e-16


def test_cold_start_is_the_special_case(small_geo):
    # x0 = 0: the same iterates as the independent C LSQR oracle (two valid
    # summation orders: agreement degrades with k as orthogonality is lost)
    op = oracle.Operator.from_system(small_geo)
    for k in (1, 2, 5, 9):
        assert rel(W.warm(op, small_geo.dt, np.zeros(small_geo.n), k)["x"],
                   op.lsqr(small_geo.dt, k)["x"]) < (1e-12 if k <= 5 else 1e-8), k


def test_exact_start_needs_no_step(tiny):
    A, b = dense_abar(tiny), bbar(tiny)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    op = oracle.Operator.from_system(tiny)
    r = W.warm(op, tiny.dt, xs, 50, tol=1e-10)
    assert r["iters"] <= 1 and r["eta"] <= 1e-10 and rel(r["x"], xs) < 1e-12


def test_diagonal_closed_form_from_any_start():
    # three distinct singular values: the shifted Krylov space holds the
    # solution after 3 steps, whatever x0
    n = 24
    g = np.array([1.0, 2.0, 3.0] * 8)
    dt = np.random.default_rng(5).standard_normal(n)
    s = diag_system(g, dt, 0.1, (2, 3, 4))
    exact = g * dt / (g * g + 0.01)
    op = oracle.Operator.from_system(s)
    x0 = np.random.default_rng(6).standard_normal(n)
    assert rel(W.warm(op, dt, x0, 3)["x"], exact) < 1e-13


def test_lsmr_form_against_scipy(small_geo):
    s = small_geo
    A, b = dense_abar(s), bbar(s)
    x0 = np.random.default_rng(9).standard_normal(s.n)
    op = oracle.Operator.from_system(s)
    for k in (1, 3, 6):
        ours = W.warm(op, s.dt, x0, k, method="lsmr")["x"]
        ref = x0 + spla.lsmr(A, b - A @ x0, atol=0, btol=0, conlim=0, maxiter=k)[0]
        assert rel(ours, ref) < 1e-11, k
