"""Pins of the FP64 CPU oracle against what mathematics fixes (no GPU).

Every check here is independent of the oracle's own code: dense library
least squares, Kronecker-sum Laplacians, closed forms, Krylov brute force, an
independent CGLS, SciPy's damped LSQR and the invariants of Paige & Saunders'
method (monotone residual norm, the one property the paper credits LSQR with).
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth


# ----------------------------------------------------------------- helpers --
def path_laplacian(k):
    """Graph Laplacian of a path with k nodes (degree on the diagonal)."""
    L = np.zeros((k, k))
    for i in range(k - 1):
        L[i, i] += 1; L[i + 1, i + 1] += 1
        L[i, i + 1] -= 1; L[i + 1, i] -= 1
    return L


def kron_laplacian(nx, ny, nz):
    """-(graph Laplacian of the nx x ny x nz grid graph) as a Kronecker sum in
    the unknown order (iy, ix, iz), depth fastest."""
    Iy, Ix, Iz = np.eye(ny), np.eye(nx), np.eye(nz)
    G = (np.kron(np.kron(path_laplacian(ny), Ix), Iz) + np.kron(np.kron(Iy, path_laplacian(nx)), Iz)
         + np.kron(np.kron(Iy, Ix), path_laplacian(nz)))
    return -G


def dense_abar(s, damp=None, smooth=None):
    damp = s.damp if damp is None else damp
    smooth = s.smooth if smooth is None else smooth
    G = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.m, s.n)).toarray()
    return np.vstack([G, smooth * kron_laplacian(s.nx, s.ny, s.nz), damp * np.eye(s.n)])


def bbar(s, dt=None):
    return np.r_[s.dt if dt is None else dt, np.zeros(2 * s.n)]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def tiny():
    return synth.random_system(60, 2, 2, 5, row_len=(1, 8), seed=11, damp=0.1, smooth=0.5)


@pytest.fixture(scope="module")
def small_geo():
    return synth.make_system(synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4,
                                                region=0.5))


# --------------------------------------------------------------- operator ---
@pytest.mark.parametrize("grid", [(3, 4, 5), (1, 1, 6), (2, 1, 1), (4, 3, 1)])
def test_laplacian_is_kronecker_sum(grid):
    nx, ny, nz = grid
    n = nx * ny * nz
    L = np.stack([oracle.laplacian_apply(nx, ny, nz, e) for e in np.eye(n)], axis=1)
    assert np.array_equal(L, kron_laplacian(nx, ny, nz))
    assert np.all(L @ np.ones(n) == 0)
    assert np.array_equal(L, L.T)


@pytest.mark.parametrize("scaled", [False, True])
def test_operator_matches_dense_blocks(tiny, scaled):
    s = tiny
    d = np.random.default_rng(2).uniform(0.5, 2.0, s.n) if scaled else None
    op = oracle.Operator.from_system(s, d=d)
    A = np.stack([op.apply(e) for e in np.eye(s.n)], axis=1)
    ref = dense_abar(s) * (1.0 if d is None else d[None, :])
    assert np.allclose(A, ref, rtol=1e-15, atol=1e-15)
    At = np.stack([op.apply_t(e) for e in np.eye(op.mbar)], axis=1)
    assert np.allclose(At, ref.T, rtol=1e-15, atol=1e-15)


def test_jacobi_is_inverse_column_norm(tiny):
    op = oracle.Operator.from_system(tiny)
    d = op.jacobi()
    assert np.allclose(d, 1.0 / np.linalg.norm(dense_abar(tiny), axis=0), rtol=1e-14)


# ------------------------------------------------------------ closed forms --
def test_converged_matches_dense_least_squares(tiny, small_geo):
    for s in (tiny, small_geo):
        A, b = dense_abar(s), bbar(s)
        x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
        Lc = np.linalg.cholesky(A.T @ A)
        x_ne = np.linalg.solve(Lc.T, np.linalg.solve(Lc, A.T @ b))
        kappa = np.linalg.cond(A)
        r = oracle.lsqr(s, 2000, tol=1e-15)
        assert r["istop"] in (1, 2, 3)
        assert rel(r["x"], x_ls) < 50 * kappa * 1e-16
        assert rel(r["x"], x_ne) < 50 * kappa ** 2 * 1e-16


def diag_system(g, dt, damp, grid):
    n = len(g)
    return synth.RandomSystem(m=n, n=n, nx=grid[0], ny=grid[1], nz=grid[2],
                              row_ptr=np.arange(n + 1, dtype=np.int64),
                              col=np.arange(n, dtype=np.int32), val=np.asarray(g, float),
                              dt=np.asarray(dt, float), damp=damp, smooth=0.0)


def test_diagonal_closed_form():
    n = 24
    g = np.array([1.0, 2.0, 3.0] * 8)
    b = np.random.default_rng(5).standard_normal(n)
    lam = 0.1
    s = diag_system(g, b, lam, (2, 3, 4))
    exact = g * b / (g * g + lam * lam)
    # three distinct singular values -> exact after 3 steps
    r = oracle.lsqr(s, 3)
    assert rel(r["x"], exact) < 1e-14
    # Jacobi scaling makes (Abar D)^T (Abar D) = I -> exact after 1 step
    op = oracle.Operator.from_system(s)
    opd = oracle.Operator.from_system(s, d=op.jacobi())
    r1 = opd.lsqr(b, 1)
    assert rel(r1["x"], exact) < 1e-14


def test_single_column_closed_form():
    g = np.array([0.5, -1.0, 2.0, 3.0, 0.25, -0.75, 1.5])
    b = np.array([1.0, 2.0, -1.0, 0.5, 4.0, -2.0, 0.0])
    s = synth.RandomSystem(m=7, n=1, nx=1, ny=1, nz=1, row_ptr=np.arange(8, dtype=np.int64),
                           col=np.zeros(7, dtype=np.int32), val=g, dt=b, damp=0.3, smooth=0.5)
    r = oracle.lsqr(s, 1)
    assert abs(r["x"][0] - g @ b / (g @ g + 0.09)) < 1e-15


def test_rational_worked_example():
    # G = [[1,0],[0,2],[1,1]] on a 1x1x2 grid, w = 1/2, lambda = 1/10, dt = (1,2,3):
    # x* solves (G^T G + w^2 L^T L + lambda^2 I) x = G^T dt exactly in rationals
    F = Fraction
    G = [[F(1), F(0)], [F(0), F(2)], [F(1), F(1)]]
    L = [[F(-1), F(1)], [F(1), F(-1)]]
    w, lam, dt = F(1, 2), F(1, 10), [F(1), F(2), F(3)]
    N = [[sum(G[k][i] * G[k][j] for k in range(3)) + w * w * sum(L[k][i] * L[k][j] for k in range(2))
          + (lam * lam if i == j else 0) for j in range(2)] for i in range(2)]
    rhs = [sum(G[k][i] * dt[k] for k in range(3)) for i in range(2)]
    det = N[0][0] * N[1][1] - N[0][1] * N[1][0]
    xs = [(N[1][1] * rhs[0] - N[0][1] * rhs[1]) / det, (N[0][0] * rhs[1] - N[1][0] * rhs[0]) / det]
    s = synth.RandomSystem(m=3, n=2, nx=1, ny=1, nz=2, row_ptr=np.array([0, 1, 2, 4], np.int64),
                           col=np.array([0, 1, 0, 1], np.int32), val=np.array([1., 2., 1., 1.]),
                           dt=np.array([1., 2., 3.]), damp=0.1, smooth=0.5)
    r = oracle.lsqr(s, 2)            # n = 2 -> exact after 2 steps
    assert np.allclose(r["x"], [float(v) for v in xs], rtol=1e-14, atol=0)


def test_first_iterate_is_steepest_descent_step(small_geo):
    # x_1 = (|g|^2 / |Abar g|^2) g with g = Abar^T bbar
    A, b = dense_abar(small_geo), bbar(small_geo)
    g = A.T @ b
    x1 = (g @ g) / np.sum((A @ g) ** 2) * g
    assert rel(oracle.lsqr(small_geo, 1)["x"], x1) < 1e-14


def test_krylov_bruteforce(small_geo):
    A, b = dense_abar(small_geo), bbar(small_geo)
    M = A.T @ A
    V = np.zeros((small_geo.n, 0))
    vec = A.T @ b
    for k in range(1, 9):
        for _ in range(2):                         # Gram-Schmidt twice
            vec = vec - V @ (V.T @ vec)
        V = np.hstack([V, (vec / np.linalg.norm(vec))[:, None]])
        y = np.linalg.lstsq(A @ V, b, rcond=None)[0]
        xk = V @ y
        # rounding in both constructions grows with k as orthogonality is lost
        assert rel(oracle.lsqr(small_geo, k)["x"], xk) < (1e-12 if k <= 6 else 1e-10), k
        vec = M @ V[:, -1]


def cgls(A, b, k):
    """CG on the normal equations A^T A x = A^T b (Hestenes-Stiefel form)."""
    x = np.zeros(A.shape[1])
    r = b.copy()
    s = A.T @ r
    p = s.copy()
    gam = s @ s
    out = []
    for _ in range(k):
        q = A @ p
        a = gam / (q @ q)
        x = x + a * p
        r = r - a * q
        s = A.T @ r
        g2 = s @ s
        p = s + (g2 / gam) * p
        gam = g2
        out.append(x.copy())
    return out


def test_cgls_equivalence(tiny, small_geo):
    # the two recurrences round differently, and the gap grows once
    # orthogonality is lost: compare while it is below 1e-10
    for s, kmax in ((tiny, 20), (small_geo, 8)):
        A, b = dense_abar(s), bbar(s)
        xs = cgls(A, b, kmax)
        for k in range(1, kmax + 1):
            assert rel(oracle.lsqr(s, k)["x"], xs[k - 1]) < 1e-10, k


def test_scipy_damped_lsqr_and_implicit_mode(cfg0_system):
    s = cfg0_system
    G = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.m, s.n))
    Ls = sp.csr_matrix(kron_laplacian(s.nx, s.ny, s.nz)) if s.n <= 2304 else None
    A = sp.vstack([G, s.smooth * Ls]).tocsr()
    b = np.r_[s.dt, np.zeros(s.n)]
    op = oracle.Operator.from_system(s)
    for K in (1, 3, 6, 8):
        xs = spla.lsqr(A, b, damp=s.damp, atol=0, btol=0, conlim=0, iter_lim=K)[0]
        xe = op.lsqr(s.dt, K)["x"]
        xi = op.lsqr_implicit(s.dt, K)
        assert rel(xe, xs) < 1e-12, K
        assert rel(xi, xs) < 1e-12, K


# -------------------------------------------------------------- invariants --
def test_lsqr_invariants(cfg0_system):
    s = cfg0_system
    op = oracle.Operator.from_system(s)
    A = None
    K = 100
    r = op.lsqr(s.dt, K, ncap=11)
    h = r["hist"]
    # the residual norm estimate never increases (the paper's LSQR property)
    assert np.all(np.diff(h[:, 0]) <= 1e-14 * h[0, 0])
    b = bbar(s)
    xn_prev = 0.0
    for k in range(1, 31):
        xk = op.lsqr(s.dt, k)["x"]
        res = np.linalg.norm(b - op.apply(xk))
        assert abs(res - h[k, 0]) <= 1e-10 * h[0, 0] + (1e-6 * h[k, 0] if k > 10 else 0), k
        xn = np.linalg.norm(xk)
        assert xn >= xn_prev * (1 - 1e-12)      # |x_k| is non-decreasing
        xn_prev = xn
        if k <= 8:
            # Abar^T rbar_k = +- psi_k v_{k+1}, so |Abar^T rbar_k| = psi_k
            atr = np.linalg.norm(op.apply_t(b - op.apply(xk)))
            assert abs(atr - h[k, 1]) <= 1e-9 * h[0, 1], k
    # early Lanczos vectors are orthonormal
    U, V = r["U"][:7], r["V"][:7]
    assert np.abs(U @ U.T - np.eye(7)).max() < 1e-12
    assert np.abs(V @ V.T - np.eye(7)).max() < 1e-12
    # the normal-equation residual goes to zero
    assert oracle.lsqr(s, 3000, tol=1e-10)["istop"] == 1


def test_column_scaling_keeps_the_solution(small_geo):
    s = small_geo
    op = oracle.Operator.from_system(s)
    x0 = op.lsqr(s.dt, 5000, tol=1e-14)["x"]
    for d in (op.jacobi(), np.random.default_rng(9).uniform(0.2, 5.0, s.n)):
        x1 = oracle.Operator.from_system(s, d=d).lsqr(s.dt, 5000, tol=1e-14)["x"]
        assert rel(x1, x0) < 1e-10


def test_breakdowns():
    s = synth.random_system(20, 2, 2, 2, seed=3)
    r = oracle.lsqr(s, 10, dt=np.zeros(s.m))
    assert r["istop"] == 0 and np.all(r["x"] == 0)
    # Abar^T bbar = 0: both data rows hit the single column with opposite data
    z = synth.RandomSystem(m=2, n=1, nx=1, ny=1, nz=1, row_ptr=np.array([0, 1, 2], np.int64),
                           col=np.zeros(2, np.int32), val=np.array([1.0, 1.0]),
                           dt=np.array([1.0, -1.0]), damp=0.1, smooth=0.5)
    r = oracle.lsqr(z, 10)
    assert r["istop"] == 0 and np.all(r["x"] == 0)


def test_thread_count_does_not_change_results(cfg0_system):
    a = oracle.lsqr(cfg0_system, 50, nthreads=1)
    b = oracle.lsqr(cfg0_system, 50, nthreads=4)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["hist"], b["hist"])


def test_summation_order_sensitivity(cfg0_system):
    """The oracle's own sensitivity to rounding order: early iterates agree to
    rounding level, fixed-count iterates later diverge by far more than 1e-10
    (loss of orthogonality amplifies last-bit differences), and converged
    solutions agree again."""
    s = cfg0_system
    for K, bound in ((2, 1e-14), (5, 1e-13), (8, 1e-11)):
        a, b = oracle.lsqr(s, K), oracle.lsqr(s, K, compensated=True)
        assert rel(a["x"], b["x"]) < bound, K
    a, b = oracle.lsqr(s, 100), oracle.lsqr(s, 100, compensated=True)
    assert rel(a["x"], b["x"]) > 1e-8
    assert abs(a["hist"][-1, 0] - b["hist"][-1, 0]) < 1e-3 * b["hist"][-1, 0]
    a = oracle.lsqr(s, 20000, tol=1e-13)
    b = oracle.lsqr(s, 20000, tol=1e-13, compensated=True)
    assert a["istop"] == 1 and b["istop"] == 1
    assert rel(a["x"], b["x"]) < 1e-10
