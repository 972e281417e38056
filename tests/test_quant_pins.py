"""Pins of the oracle quantiser (no GPU): library conversions that round once
from the same value, the half-unit error bound, ties to even, and the
refinement fixed point that motivates the corrected right-hand side."""
import numpy as np
import pytest

import synth
from oracle import quant

torch = pytest.importorskip("torch")


def test_bf16_matches_library_rounding_of_float32_values():
    # for inputs that are exactly float32, rounding once from FP64 is the same as
    # torch's float32 -> bfloat16 round-to-nearest-even
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = quant.codes(quant.round_to_format(x.astype(np.float64), "bf16"), "bf16")
    assert np.array_equal(got, ref)


def test_fp16_matches_numpy_rounding_of_float64():
    rng = np.random.default_rng(1)
    # normal and subnormal FP16 range, below the largest finite value
    x = rng.uniform(-1, 1, 200000) * 2.0 ** rng.uniform(-26, 15.9, 200000)
    ref = x.astype(np.float16).view(np.uint16)
    got = quant.codes(quant.round_to_format(x, "fp16"), "fp16")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("fmt,p", [("bf16", 8), ("fp16", 11)])
def test_ties_go_to_even(fmt, p):
    # 1 + (k + 1/2) ulp lies exactly halfway between two neighbours
    ulp = 2.0 ** -(p - 1)
    k = np.arange(0, 20)
    x = 1.0 + (k + 0.5) * ulp
    r = quant.round_to_format(x, fmt)
    lo, hi = 1.0 + k * ulp, 1.0 + (k + 1) * ulp
    even = np.where(k % 2 == 0, lo, hi)
    assert np.array_equal(r, even)
    # and just above / below the tie
    assert np.array_equal(quant.round_to_format(x + 2.0 ** -40, fmt), hi)
    assert np.array_equal(quant.round_to_format(x - 2.0 ** -40, fmt), lo)


@pytest.mark.parametrize("fmt,bound", [("bf16", 2.0 ** -9), ("fp16", 2.0 ** -12)])
def test_quantised_rows_error_bound(cfg0_system, fmt, bound):
    s = cfg0_system
    sig, q = quant.quantise_csr(s.row_ptr, s.val, fmt)
    rows = np.repeat(np.arange(s.m), np.diff(s.row_ptr))
    deq = quant.decode(q, fmt) * sig[rows]
    # P_i = 2^ceil(log2 max_j |g_ij|): half a unit of the top binade
    P = sig.astype(np.float64) * (2.0 ** 14 if fmt == "fp16" else 1.0)
    assert np.all(np.abs(deq - s.val) <= bound * P[rows] * (1 + 1e-12))
    assert np.all(np.abs(quant.decode(q, fmt)) <= (2.0 ** 14 if fmt == "fp16" else 1.0))
    # sigma is an exact power of two
    f, _ = np.frexp(sig.astype(np.float64))
    assert np.all(f == 0.5)


def _dense(s):
    import scipy.sparse as sp
    from _helpers import sparse_abar
    return sparse_abar(s).toarray()


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_refinement_fixed_points(fmt):
    """With exact inner solves on the quantised operator, refinement on the
    plain residual converges to a point with Ahat^T (bbar - Abar x) = 0, away
    from x* when the data are noisy; the corrected right-hand side
    [r_G; r_L; r_D + (g - ghat)/lambda] converges to x*, and so does the one
    the library uses, [0; 0; (Abar^T r)/lambda] (the same Ahat^T f, with
    the residual itself taken out), sweep by sweep to the same iterates."""
    s = synth.make_system(synth.small_config(nx=6, ny=6, nz=5, n_stations=14, n_periods=5,
                                             region=0.6))
    A = _dense(s)
    sig, q = quant.quantise_csr(s.row_ptr, s.val, fmt)
    rows = np.repeat(np.arange(s.m), np.diff(s.row_ptr))
    Gh = np.zeros((s.m, s.n))
    Gh[rows, s.col] = quant.decode(q, fmt) * sig[rows]
    Ah = A.copy()
    Ah[:s.m] = Gh
    b = np.r_[s.dt, np.zeros(2 * s.n)]
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    solve_h = np.linalg.pinv(Ah)
    x_naive = np.zeros(s.n)
    x_corr = np.zeros(s.n)
    x_norm = np.zeros(s.n)
    for sweep in range(12):
        r = b - A @ x_naive
        x_naive = x_naive + solve_h @ r
        r = b - A @ x_corr
        g, gh = A[:s.m].T @ r[:s.m], Gh.T @ r[:s.m]
        f = r.copy()
        f[s.m + s.n:] += (g - gh) / s.damp
        x_corr = x_corr + solve_h @ f
        r = b - A @ x_norm
        fn = np.zeros_like(r)
        fn[s.m + s.n:] = (A.T @ r) / s.damp
        assert np.allclose(Ah.T @ fn, A.T @ r, rtol=1e-12, atol=1e-14 * np.abs(A.T @ r).max())
        x_norm = x_norm + solve_h @ fn
        if sweep < 3:      # the same correction, up to rounding
            assert np.linalg.norm(x_norm - x_corr) <= 1e-9 * np.linalg.norm(x_corr)
    err_naive = np.linalg.norm(x_naive - xs) / np.linalg.norm(xs)
    err_corr = np.linalg.norm(x_corr - xs) / np.linalg.norm(xs)
    err_norm = np.linalg.norm(x_norm - xs) / np.linalg.norm(xs)
    assert err_corr < 1e-12
    assert err_norm < 1e-12
    assert err_naive > 1e-6
