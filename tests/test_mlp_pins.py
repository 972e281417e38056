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


# Independent values: Phi(1) and Phi(2), the standard normal distribution function,
# from printed tables of the normal distribution, and ln 2.
PHI_1 = 0.8413447460685429
PHI_2 = 0.9772498680518208
LN2 = 0.6931471805599453


def test_gelu_and_softplus_at_known_points():
    # GELU(x) = x Phi(x): Phi(0) = 1/2, Phi(1) from the table, Phi(-1) = 1 - Phi(1)
    g = mlp.gelu(np.array([0.0, 1.0, -1.0, 2.0]))
    assert g[0] == 0.0
    assert abs(g[1] - PHI_1) < 1e-15
    assert abs(g[2] + (1.0 - PHI_1)) < 1e-15
    assert abs(g[3] - 2.0 * PHI_2) < 1e-15
    # far tails: GELU(x) -> x for x >> 0 and -> 0 for x << 0
    assert abs(mlp.gelu(np.array([12.0]))[0] - 12.0) < 1e-15
    assert abs(mlp.gelu(np.array([-12.0]))[0]) < 1e-30
    # softplus(0) = ln 2; softplus(z) - softplus(-z) = z; tails e^-|z|
    assert abs(mlp.softplus(np.array([0.0]))[0] - LN2) < 1e-16
    z = np.array([-7.5, -0.3, 0.0, 0.9, 31.0])
    assert np.allclose(mlp.softplus(z) - mlp.softplus(-z), z, rtol=0, atol=2e-15)
    assert abs(mlp.softplus(np.array([-40.0]))[0] - np.exp(-40.0)) < 1e-30
    # softplus(log(e - 1)) = 1: the output bias that starts the net at Jacobi
    assert abs(mlp.softplus(np.array([mlp.SOFTPLUS_INV_1]))[0] - 1.0) < 1e-15
    # sigmoid is softplus' slope: 1/2 at 0, and symmetric
    assert mlp.sigmoid(np.array([0.0]))[0] == 0.5
    assert np.allclose(mlp.sigmoid(z) + mlp.sigmoid(-z), 1.0, atol=1e-15)


def _two_unit_net():
    """A net whose only non-zero weights form two units per hidden layer, with
    values chosen so every activation is a multiple of Phi(1) or 0."""
    p = {name: np.zeros(shp) for name, shp in mlp.SIZES}
    p["W1"][0, 0] = 2.0               # a1_0 = 2 * 0.25 + 0.5 = 1       -> h1_0 = Phi(1)
    p["b1"][0] = 0.5
    p["W1"][1, 3] = -1.0              # a1_1 = -x3 = -1                  -> h1_1 = -(1 - Phi(1))
    p["W2"][0, 0] = 1.0 / PHI_1       # a2_0 = 1                          -> h2_0 = Phi(1)
    p["W2"][5, 0] = 1.0 / PHI_1       # a2_5 = 1 - 2 = -1                 -> h2_5 = -(1 - Phi(1))
    p["W2"][5, 1] = 2.0 / (1.0 - PHI_1)
    p["W3"][0] = 1.0                  # z = Phi(1) - (1 - Phi(1)) + b3
    p["W3"][5] = 1.0
    p["b3"][0] = 1.0 - 2.0 * PHI_1    # -> z = 0, multiplier ln 2
    return mlp.pack(p)


def test_forward_of_a_hand_evaluated_network():
    theta = _two_unit_net()
    x = np.zeros((2, mlp.NF))
    x[:, 0] = 0.25
    x[:, 3] = 1.0
    x[1, 2] = 123.0                   # an input no unit reads
    z, (xx, a1, h1, a2, h2) = mlp.forward(theta, x)
    assert np.allclose(a1[:, :2], [[1.0, -1.0]] * 2, atol=1e-15)
    assert np.allclose(h1[:, :2], [[PHI_1, -(1.0 - PHI_1)]] * 2, atol=1e-15)
    assert np.all(h1[:, 2:] == 0.0)
    assert np.allclose(a2[:, [0, 5]], [[1.0, -1.0]] * 2, atol=1e-14)
    assert np.allclose(h2[:, [0, 5]], [[PHI_1, -(1.0 - PHI_1)]] * 2, atol=1e-14)
    assert np.allclose(z, 0.0, atol=1e-14)
    assert np.allclose(mlp.multiplier(theta, x), LN2, atol=1e-14)
    # the loss against the exact target log(ln 2) is zero, against 0 it is log(ln 2)^2
    assert mlp.loss(theta, x, np.full(2, np.log(LN2))) < 1e-28
    assert abs(mlp.loss(theta, x, np.zeros(2)) - np.log(LN2) ** 2) < 1e-14


def _bf16_bits(x):
    """Nearest BF16 value of a double, ties to even, by integer arithmetic on
    the FP32 bits (independent of oracle/quant.py); x must be an FP32 value
    away from overflow."""
    import struct
    u = struct.unpack("<I", struct.pack("<f", x))[0]
    assert struct.unpack("<f", struct.pack("<I", u))[0] == x
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return struct.unpack("<f", struct.pack("<I", u))[0]


def test_bf16_inference_hand_evaluated():
    """One live path through the network (every other weight zero): a chain
    of three roundings worked through by hand with math.erf and an
    independent BF16 rounding of FP32 values."""
    import math
    p = {k: np.zeros_like(v) for k, v in mlp.unpack(mlp.init_params(0)).items()}
    p["W1"][0, 0] = 1.5                     # BF16 values: exact
    p["b1"][0] = -0.25
    p["W2"][0, 0] = 0.75
    p["b2"][0] = 0.125
    p["W3"][0] = 2.0
    p["b3"][0] = -0.5
    theta = mlp.pack(p)
    xin = 0.3                              # rounds to a BF16 value first

    def g(v):
        return 0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0)))

    def r(v):                             # via FP32 (no double rounding here:
        return _bf16_bits(float(np.float32(v)))   # the inputs are far from ties)

    x = r(xin)
    h1 = r(g(1.5 * x - 0.25))
    h2_0 = r(g(0.75 * h1 + 0.125))
    h2_rest = r(g(0.0))                    # zero
    z = 2.0 * h2_0 - 0.5 + 0.0 * h2_rest
    expect = max(z, 0.0) + math.log1p(math.exp(-abs(z)))
    xhat = np.zeros((1, mlp.NF))
    xhat[0, 0] = xin
    got = mlp.multiplier_bf16(theta, xhat)[0]
    assert abs(got - expect) <= 1e-15 * expect
    # and the rounding matters: the unrounded network differs
    assert abs(mlp.multiplier(theta, xhat)[0] - expect) > 1e-5 * expect
