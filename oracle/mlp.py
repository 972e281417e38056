"""ORACLE — test infrastructure only.  FP64 NumPy reference of the learned
column-scaling preconditioner: the per-column features, the MLP
6 -> 64 -> 64 -> 1 (GELU, softplus output), its loss, gradients and the Adam
step.  Written from the definitions; gradients are pinned by central finite
differences in the tests.

Column features of Abar = [G; w L; lambda I] on an (nx, ny, nz) grid:

  f1  log10 |column j of Abar|  (data, smoothing and damping entries)
  f2  log(1 + number of data rows hitting column j)  (ray coverage)
  f3  iz / (nz - 1)  (depth index)
  f4  |g|-weighted mean, over the rows hitting j, of the row's depth centroid
      c_i = sum_j |g_ij| iz(j) / sum_j |g_ij| / (nz - 1)  ("period mix": the
      depth a traveltime row senses grows with its period)
  f5  |g|-weighted standard deviation of the same centroids
  f6  log(1 + mean coverage of the in-grid 7-point neighbours of j)

Parameters are one flat vector: W1 [64, 6], b1 [64], W2 [64, 64], b2 [64],
W3 [64], b3 [1] (4673 values).  The output z gives the multiplier
softplus(z) on the Jacobi scale; the loss is the mean squared error between
log softplus(z) and the target log multiplier.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

H = 64
NF = 6
SIZES = [("W1", (H, NF)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)
SOFTPLUS_INV_1 = math.log(math.e - 1.0)      # softplus(z) = 1 at z = log(e - 1)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init_params(seed=0):
    """He-normal weights, zero hidden biases, small output weights and the
    output bias at softplus^-1(1), so the untrained net starts at Jacobi."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((H, NF)) * math.sqrt(2.0 / NF), "b1": np.zeros(H),
         "W2": rng.standard_normal((H, H)) * math.sqrt(2.0 / H), "b2": np.zeros(H),
         "W3": rng.standard_normal(H) * math.sqrt(2.0 / H) * 0.1, "b3": np.array([SOFTPLUS_INV_1])}
    return pack(p)


# ----------------------------------------------------------------- features --
def column_features(row_ptr, col, val, nx, ny, nz, damp, smooth):
    """[n, 6] features of every column (FP64)."""
    n = nx * ny * nz
    m = len(row_ptr) - 1
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    a = np.abs(val)
    iz_of_col = np.arange(n) % nz
    zden = max(nz - 1, 1)
    # row depth centroids
    wsum = np.bincount(rows, weights=a, minlength=m)
    wz = np.bincount(rows, weights=a * iz_of_col[col], minlength=m)
    cen = np.where(wsum > 0, wz / np.where(wsum > 0, wsum, 1.0), 0.0) / zden
    # column sums over the rows that hit them
    g2 = np.bincount(col, weights=val * val, minlength=n)
    hits = np.bincount(col, minlength=n).astype(np.float64)
    ca = np.bincount(col, weights=a, minlength=n)
    c1 = np.bincount(col, weights=a * cen[rows], minlength=n)
    c2 = np.bincount(col, weights=a * cen[rows] ** 2, minlength=n)
    # grid neighbours
    j = np.arange(n)
    iz, ixy = j % nz, j // nz
    ix, iy = ixy % nx, ixy // nx
    deg = ((ix > 0).astype(int) + (ix < nx - 1) + (iy > 0) + (iy < ny - 1) + (iz > 0) + (iz < nz - 1))
    nb = np.zeros(n)
    for cond, off in ((ix > 0, -nz), (ix < nx - 1, nz), (iy > 0, -nx * nz), (iy < ny - 1, nx * nz),
                      (iz > 0, -1), (iz < nz - 1, 1)):
        nb[cond] += hits[j[cond] + off]
    colnorm2 = g2 + smooth * smooth * (deg * deg + deg) + damp * damp
    f = np.empty((n, NF))
    f[:, 0] = 0.5 * np.log10(colnorm2)
    f[:, 1] = np.log1p(hits)
    f[:, 2] = iz / zden
    mean = np.where(ca > 0, c1 / np.where(ca > 0, ca, 1.0), 0.0)
    var = np.where(ca > 0, c2 / np.where(ca > 0, ca, 1.0) - mean * mean, 0.0)
    f[:, 3] = mean
    f[:, 4] = np.sqrt(np.maximum(var, 0.0))
    f[:, 5] = np.log1p(np.where(deg > 0, nb / np.maximum(deg, 1), 0.0))
    return f


# ---------------------------------------------------------------------- MLP --
def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(theta, xhat):
    """z [B] and the cached activations for a batch of standardised features."""
    p = unpack(theta)
    a1 = xhat @ p["W1"].T + p["b1"]
    h1 = gelu(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(a2)
    z = h2 @ p["W3"] + p["b3"][0]
    return z, (xhat, a1, h1, a2, h2)


def loss(theta, xhat, target):
    z, _ = forward(theta, xhat)
    return float(np.mean((np.log(softplus(z)) - target) ** 2))


def grad(theta, xhat, target):
    """(loss, gradient) of the mean squared log-multiplier error."""
    p = unpack(theta)
    z, (x, a1, h1, a2, h2) = forward(theta, xhat)
    B = len(z)
    sp = softplus(z)
    r = np.log(sp) - target
    dz = 2.0 * r / B * sigmoid(z) / sp
    g = {"W3": h2.T @ dz, "b3": np.array([dz.sum()])}
    d2 = dz[:, None] * p["W3"][None, :] * gelu_grad(a2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * gelu_grad(a1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return float(np.mean(r * r)), pack(g)


def adam_step(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def multiplier(theta, xhat):
    """softplus(z): the learned multiplier of the Jacobi scale."""
    z, _ = forward(theta, xhat)
    return softplus(z)


def multiplier_bf16(theta, xhat):
    """softplus(z) of the reduced-precision inference: the parameters, the
    standardised inputs and both layers' activations rounded to the nearest
    BF16 value (ties to even), every product and sum exact up to FP64
    rounding (the device accumulates in FP32)."""
    from .quant import round_to_format

    def b(a):
        return round_to_format(np.asarray(a, dtype=np.float64), "bf16")

    p = {k: b(v) for k, v in unpack(theta).items()}
    x = b(xhat)
    h1 = b(gelu(x @ p["W1"].T + p["b1"]))
    h2 = b(gelu(h1 @ p["W2"].T + p["b2"]))
    z = h2 @ p["W3"] + p["b3"][0]
    return softplus(z)
