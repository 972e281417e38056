"""GPU checks of the reduced-precision forms.

* The BF16/FP16 codes and row scales equal the oracle quantiser's bitwise, in
  both the row-major and the transposed copy.
* BF16/FP16 with FP64 refinement reach the FP64 solution x* (the oracle run to
  eta <= 1e-12) within 1e-5 relative.
* FP32 LSQR: error against the oracle reported, with bounds from FP32 rounding.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from oracle import quant

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def from_sys(s, **k):
    from paper_2604_11920_amd import Solver
    return Solver.from_system(s, **k)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_system(synth.config0())


@pytest.fixture(scope="module")
def xstar(cfg0):
    op = oracle.Operator.from_system(cfg0)
    r = oracle.Operator.from_system(cfg0, d=op.jacobi(), compensated=True).lsqr(cfg0.dt, 40000,
                                                                                 tol=1e-12)
    assert r["istop"] == 1
    return r["x"]


def ragged():
    s = synth.random_system(700, 6, 5, 4, row_len=(0, 60), seed=21)
    s.val = s.val * np.exp(np.random.default_rng(2).uniform(-20, 20, s.nnz))
    return s


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("which", ["cfg0", "ragged"])
def test_quantised_codes_bitwise(cfg0, fmt, which):
    s = cfg0 if which == "cfg0" else ragged()
    sig_ref, q_ref = quant.quantise_csr(s.row_ptr, s.val, fmt)
    with from_sys(s, precision=fmt) as sol:
        sig, qr, qc = sol.quantised()
    assert np.array_equal(sig, sig_ref)
    assert np.array_equal(qr, q_ref)
    # the transposed copy holds the same codes in column order
    order = sp.csr_matrix((np.arange(s.nnz, dtype=np.float64) + 1, s.col, s.row_ptr),
                          shape=(s.m, s.n)).tocsc()
    order.sort_indices()
    assert np.array_equal(qc, q_ref[order.data.astype(np.int64) - 1])


@pytest.mark.parametrize("fmt,precond,col_format", [
    ("bf16", "none", "auto"), ("bf16", "jacobi", "auto"), ("fp16", "none", "csc"),
    ("fp16", "jacobi", "auto"), ("bf16", "jacobi", "runs"), ("fp16", "jacobi", "runs"),
    ("bf16", "jacobi", "pairs"), ("fp16", "none", "pairs")])
def test_refinement_reaches_fp64_solution(cfg0, xstar, fmt, precond, col_format):
    # Without column scaling the error at a given eta is ~100x larger on this
    # system (|x - x*| is bounded by cond(Abar^T Abar) eta, ~3e5 unscaled), and
    # the refinement's FP32 floor (a few 1e-9) leaves little room to tighten
    # eta; the unscaled forms instead take tighter inner solves, whose sweeps
    # overshoot the tolerance.  The Jacobi-scaled forms use the default.
    tol = 1e-7
    inner = 0.0 if precond == "jacobi" else 1e-3
    with from_sys(cfg0, precision=fmt, precond=precond, refine_sweeps=10, refine_inner_tol=inner,
                  col_format=col_format) as sol:
        dm, hist, info = sol.solve(cfg0.dt, 3000, tol=tol)
    err = rel(dm, xstar)
    print(f"[{fmt}/{precond}/{col_format}] sweeps={info['sweeps']} inner iters={info['iters']} "
          f"eta={info['eta']:.2e} err_vs_x*={err:.2e}")
    # each sweep gains at least ~30x (the quantisation error and the inner
    # tolerance bound it), so the tolerance takes a handful of sweeps
    assert info["istop"] == 1 and info["eta"] <= tol and info["sweeps"] <= 8
    assert err <= 1e-5


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_refinement_floor_is_flagged(cfg0, xstar, fmt):
    # a tolerance at the FP64 rounding level: the sweeps stop contracting,
    # the inner solves switch to FP32 values, and the solve either reaches it
    # or ends with the stall flag, at the FP64 solution
    with from_sys(cfg0, precision=fmt, precond="jacobi", refine_sweeps=10) as sol:
        dm, hist, info = sol.solve(cfg0.dt, 3000, tol=1e-13)
    err = rel(dm, xstar)
    print(f"[{fmt}] floor: istop={info['istop']} sweeps={info['sweeps']} eta={info['eta']:.2e} "
          f"err={err:.2e}")
    assert info["istop"] in (1, 4) and err <= 1e-5


def test_mixed_form_rejections(cfg0):
    from paper_2604_11920_amd import LsqrError
    with pytest.raises(LsqrError):
        from_sys(cfg0, precision="bf16", damp=0.0)
    with from_sys(cfg0, precision="bf16") as sol:
        with pytest.raises(LsqrError):
            sol.solve(cfg0.dt, 100, tol=0.0)


@pytest.mark.parametrize("row_format,col_format", [("csr", "csc"), ("csr", "runs"),
                                                    ("groups", "pairs")])
def test_fp32_iterates(cfg0, row_format, col_format):
    ref = oracle.lsqr(cfg0, 5)
    with from_sys(cfg0, precision="fp32", row_format=row_format, col_format=col_format) as sol:
        dm, hist, info = sol.solve(cfg0.dt, 5)
    err = rel(dm, ref["x"])
    print(f"[fp32/{row_format}/{col_format}] K=5 rel err {err:.2e}")
    assert info["iters"] == 5 and err <= 1e-4
    assert np.allclose(hist[:, 0], ref["hist"][:, 0], rtol=1e-5)


def test_fp32_converged(cfg0, xstar):
    # at a given eta the distance to x* is set by the conditioning; compare FP32
    # with FP64 stopped at the same tolerance
    with from_sys(cfg0, precision="fp32", precond="jacobi") as sol:
        dm, hist, info = sol.solve(cfg0.dt, 5000, tol=1e-5)
    with from_sys(cfg0, precond="jacobi") as sol:
        dm64, _, info64 = sol.solve(cfg0.dt, 5000, tol=1e-5)
    err, err64 = rel(dm, xstar), rel(dm64, xstar)
    print(f"[fp32] tol 1e-5: iters={info['iters']} err_vs_x*={err:.2e} (fp64: {info64['iters']} "
          f"iters, {err64:.2e})")
    assert info["istop"] == 1 and err <= 3 * err64 + 1e-4


@pytest.mark.parametrize("row_format", ["csr", "groups"])
def test_fp64_row_formats_agree(cfg0, row_format):
    ref = oracle.lsqr(cfg0, 6)
    with from_sys(cfg0, row_format=row_format) as sol:
        dm, hist, info = sol.solve(cfg0.dt, 6)
    assert rel(dm, ref["x"]) <= 1e-10


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_stall_switches_inner_solves_to_fp32(cfg0, xstar, fmt):
    """A sweep that does not bring eta below refine_stall_ratio times the
    previous one counts as a stall: the first moves the remaining inner
    solves to FP32 values (info.inner_fp32), the second ends the solve
    (istop 4).  Forced from the host with a ratio no sweep can meet: sweep 0
    runs on the quantised values, sweep 1 on the FP32 values, and that sweep
    must carry the refinement on (eta and the error fall by the inner
    solve's gain)."""
    kw = dict(precision=fmt, precond="jacobi", refine_sweeps=10)
    with from_sys(cfg0, refine_sweeps=1, **{k: v for k, v in kw.items() if k != "refine_sweeps"}) as sol:
        dm1, _, i1 = sol.solve(cfg0.dt, 3000, tol=1e-14)
    assert i1["istop"] == 2 and i1["sweeps"] == 1 and i1["inner_fp32"] == 0
    with from_sys(cfg0, refine_stall_ratio=1e-300, **kw) as sol:
        dm2, _, i2 = sol.solve(cfg0.dt, 3000, tol=1e-14)
        # the context keeps its FP32 kernels: a second solve gives the same bits
        dm3, _, i3 = sol.solve(cfg0.dt, 3000, tol=1e-14)
    e1, e2 = rel(dm1, xstar), rel(dm2, xstar)
    print(f"[{fmt}] stall switch: sweep-0 eta {i1['eta']:.2e} err {e1:.2e}; after the FP32 sweep "
          f"eta {i2['eta']:.2e} err {e2:.2e} (istop {i2['istop']}, sweeps {i2['sweeps']})")
    assert i2["istop"] == 4 and i2["sweeps"] == 2 and i2["inner_fp32"] == 1
    assert i2["eta"] < 0.1 * i1["eta"] and e2 < 0.1 * e1
    assert i2["eta_final_fp64"] == i2["eta"]
    assert i3 == i2 and np.array_equal(dm3, dm2)


def test_plain_forms_never_switch(cfg0):
    with from_sys(cfg0, precision="fp32", precond="jacobi") as sol:
        _, _, info = sol.solve(cfg0.dt, 500, tol=1e-6)
    assert info["inner_fp32"] == 0



@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_ill_conditioned_refinement_switches_to_fp32(fmt):
    """Config 0 with damping 1e-3 and smoothing weight 0.01: the quantised
    operator is too far from the FP64 one for the sweeps to keep halving eta,
    so the stall guard moves the inner solves to FP32 values, and the
    refinement then reaches eta <= 1e-10 and the oracle's x* (stored by
    tests/golden/make_illcond_golden.py) within 1e-5."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "cfg0_illcond.npz"))
    c = synth.config0()
    c.damp, c.smooth = float(g["damp"]), float(g["smooth"])
    s = synth.make_system(c)
    assert synth.fingerprint(s) == str(g["fingerprint"]), "the generator changed"
    with from_sys(s, precision=fmt, precond="jacobi", refine_sweeps=12) as sol:
        dm, _, info = sol.solve(s.dt, 20000, tol=1e-10)
    err = rel(dm, g["xstar"])
    print(f"[{fmt}] ill-conditioned: istop={info['istop']} sweeps={info['sweeps']} "
          f"iters={info['iters']} eta_fp64={info['eta_final_fp64']:.2e} err={err:.2e}")
    assert info["inner_fp32"] == 1
    assert info["istop"] == 1 and info["eta_final_fp64"] <= 1e-10 and err <= 1e-5
