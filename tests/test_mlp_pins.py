"""Pins of the learned-preconditioner reference (no GPU): gradients against
central finite differences, features against independent constructions, the
Adam step against its closed form at t = 1, and the start-as-Jacobi init."""
import numpy as np
import pytest

import synth
from oracle import mlp
from _helpers import laplacian, sparse_abar


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(3)
    theta = theta + 0.05 * rng.standard_normal(theta.size)     # away from the init point
    x = rng.standard_normal((37, mlp.NF))
    t = rng.standard_normal(37) * 0.3
    L, g = mlp.grad(theta, x, t)
    assert abs(L - mlp.loss(theta, x, t)) < 1e-15
    idx = np.r_[rng.choice(mlp.NPARAMS, 300, replace=False), mlp.NPARAMS - 1]
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp.loss(theta + e, x, t) - mlp.loss(theta - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, i


def test_init_starts_at_jacobi():
    theta = mlp.init_params(0)
    x = np.random.default_rng(1).standard_normal((1000, mlp.NF))
    s = mlp.multiplier(theta, x)
    assert np.all(np.abs(s - 1.0) < 0.25) and abs(np.median(s) - 1.0) < 0.05


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # at t = 1 the bias-corrected moments are g and g^2: a step of lr * g / (|g| + eps)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_features_against_independent_constructions():
    s = synth.make_system(synth.small_config(nx=6, ny=5, nz=4, n_stations=10, n_periods=4,
                                             region=0.5))
    f = mlp.column_features(s.row_ptr, s.col, s.val, s.nx, s.ny, s.nz, s.damp, s.smooth)
    A = sparse_abar(s)
    assert np.allclose(f[:, 0], np.log10(np.sqrt((A.multiply(A)).sum(axis=0).A1)), rtol=1e-13)
    G = s.scipy()
    hits = np.diff(G.tocsc().indptr)
    assert np.allclose(f[:, 1], np.log1p(hits), rtol=1e-15)
    assert np.allclose(f[:, 2], (np.arange(s.n) % s.nz) / (s.nz - 1))
    # neighbours: off-diagonal entries of the Laplacian are the grid graph's edges
    Ld = laplacian(s.nx, s.ny, s.nz).toarray()
    adj = (Ld > 0).astype(float)
    nb = adj @ hits / adj.sum(axis=1)
    assert np.allclose(f[:, 5], np.log1p(nb), rtol=1e-13)
    # depth centroids of rows and their |g|-weighted statistics per column
    Gd = np.abs(G.toarray())
    iz = np.arange(s.n) % s.nz
    cen = np.where(Gd.sum(1) > 0, (Gd * iz).sum(1) / np.maximum(Gd.sum(1), 1e-300), 0) / (s.nz - 1)
    for j in range(0, s.n, 7):
        w = Gd[:, j]
        if w.sum() == 0:
            assert f[j, 3] == 0 and f[j, 4] == 0
            continue
        mu = (w * cen).sum() / w.sum()
        sd = np.sqrt(max((w * (cen - mu) ** 2).sum() / w.sum(), 0))
        assert abs(f[j, 3] - mu) < 1e-12 and abs(f[j, 4] - sd) < 1e-7
