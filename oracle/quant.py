"""ORACLE — test infrastructure only.  Reference quantiser of the BF16/FP16
storage forms, written from the definitions (NumPy, FP64).

Row i of G is stored as a power-of-two scale sigma_i times 16-bit codes:

* sigma_i = 2^ceil(log2 max_j |g_ij|) for BF16, so every |g_ij / sigma_i| <= 1;
  for FP16 sigma_i is that power times 2^-14, so the largest entry sits near
  2^14 and small entries stay out of the FP16 subnormal range; rows without a
  nonzero entry get sigma_i = 1;
* q_ij = the value of the target format nearest to g_ij / sigma_i, ties to the
  even significand, rounded once from the FP64 value.

The nearest value is found by scaling by the quantum of the value's binade
(2^(floor(log2|x|) - (p - 1)), not below the subnormal quantum) and rounding
to an integer with numpy.rint (round half to even); p = 8 significand bits for
BF16 and 11 for FP16.
"""
from __future__ import annotations

import numpy as np

FORMATS = {"bf16": (8, -126), "fp16": (11, -14)}    # significand bits, min normal exponent


def row_scales(row_ptr, val, fmt):
    """sigma_i as float32 powers of two."""
    m = len(row_ptr) - 1
    mx = np.zeros(m)
    nz = np.diff(row_ptr) > 0
    mx[nz] = np.maximum.reduceat(np.abs(val), row_ptr[:-1][nz])
    f, e = np.frexp(mx)                       # mx = f 2^e, f in [0.5, 1)
    E = np.where(f == 0.5, e - 1, e)          # ceil(log2 mx)
    if fmt == "fp16":
        E = E - 14
    s = np.ldexp(1.0, E)
    s[mx == 0] = 1.0
    return s.astype(np.float32)


def round_to_format(x, fmt):
    """Values of x rounded to the nearest value of fmt (ties to even), FP64."""
    p, emin = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    f, e = np.frexp(np.where(x == 0, 1.0, x))
    lead = e - 1                               # floor(log2 |x|)
    qexp = np.maximum(lead - (p - 1), emin - (p - 1))
    quantum = np.ldexp(1.0, qexp)
    r = np.rint(x / quantum) * quantum
    return np.where(x == 0, x, r)


def codes(values, fmt):
    """16-bit encodings of values that are exactly representable in fmt."""
    v = np.asarray(values, dtype=np.float64)
    if fmt == "bf16":
        f32 = v.astype(np.float32)
        assert np.array_equal(f32.astype(np.float64), v), "not representable"
        return (f32.view(np.uint32) >> 16).astype(np.uint16)
    h = v.astype(np.float16)
    assert np.array_equal(h.astype(np.float64), v), "not representable"
    return h.view(np.uint16)


def decode(codes_, fmt):
    c = np.asarray(codes_, dtype=np.uint16)
    if fmt == "bf16":
        return (c.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return c.view(np.float16).astype(np.float64)


def quantise_csr(row_ptr, val, fmt):
    """(sigma [m] float32, codes [nnz] uint16) of a CSR's values."""
    sig = row_scales(row_ptr, val, fmt)
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    q = round_to_format(val / sig[rows].astype(np.float64), fmt)
    return sig, codes(q, fmt)
