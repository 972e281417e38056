"""GPU parity of the plain FP64 path against the FP64 CPU oracle.

Parity bars (the oracle's own summation-order sensitivity, measured in
test_oracle_pins.py, decides what a fixed iteration count can promise):
  * iterates x_k for k <= 8 and converged solutions (eta <= 1e-13): <= 1e-10
    relative, the bound the plain form must meet;
  * fixed counts past the loss of orthogonality (K = 100): the residual-norm
    history within 1e-3 relative and the GPU/oracle gap a small fraction of
    the distance to the solution, as for two valid orders of summation;
  * integer-valued operators: bitwise.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from _helpers import eta_explicit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def Solver(*a, **k):
    from paper_2604_11920_amd import Solver as S
    return S(*a, **k)


def from_sys(s, **k):
    from paper_2604_11920_amd import Solver as S
    return S.from_system(s, **k)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def ragged_system(seed=0, integer=False):
    """Rows of 0..700 entries (empty rows, rows longer than the unrolled
    lane span) and columns that no row touches; several workgroups' worth."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = 7, 5, 6
    n = nx * ny * nz
    m = 900
    lens = rng.integers(0, 40, size=m)
    lens[rng.choice(m, 30, replace=False)] = rng.integers(200, 700, size=30)
    lens[:5] = 0
    avail = np.arange(n - 17)          # the last 17 columns stay empty
    row_ptr = np.zeros(m + 1, np.int64)
    row_ptr[1:] = np.cumsum(np.minimum(lens, len(avail)))
    col = np.concatenate([np.sort(rng.choice(avail, size=row_ptr[i + 1] - row_ptr[i],
                                             replace=False)) for i in range(m)]).astype(np.int32)
    if integer:
        val = rng.integers(-8, 9, size=len(col)).astype(np.float64)
        dt = rng.integers(-8, 9, size=m).astype(np.float64)
    else:
        val = rng.standard_normal(len(col))
        dt = rng.standard_normal(m)
    return synth.RandomSystem(m=m, n=n, nx=nx, ny=ny, nz=nz, row_ptr=row_ptr, col=col, val=val,
                              dt=dt, damp=0.25 if integer else 0.1, smooth=0.5)


# stored formats (forward rows, transposed columns) exercised by the solves
FORMATS = {"auto": ("auto", "auto"), "csc": ("csr", "csc"), "runs": ("csr", "runs"),
           "groups": ("groups", "auto"), "pairs": ("csr", "pairs")}


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_system(synth.config0())


@pytest.fixture(scope="module")
def cfg0_xstar(cfg0):
    return oracle.lsqr(cfg0, 40000, tol=1e-13)["x"]


# ------------------------------------------------------------ operator ------
@pytest.mark.parametrize("which", ["ragged", "cfg0"])
def test_transpose_matches_library_csc(which, cfg0):
    s = ragged_system(1) if which == "ragged" else cfg0
    with from_sys(s) as sol:
        cp, ri, cv = sol.transpose()
    ref = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.m, s.n)).tocsc()
    ref.sort_indices()
    assert np.array_equal(cp, ref.indptr) and np.array_equal(ri, ref.indices)
    assert np.array_equal(cv, ref.data)


@pytest.mark.parametrize("lanes,row_format,col_format",
                         [(0, "auto", "auto"), (4, "csr", "csc"), (16, "csr", "csc"),
                          (64, "csr", "csc"), (0, "csr", "runs"), (0, "groups", "auto"),
                          (0, "groups", "pairs"), (8, "csr", "pairs")])
def test_operator_integer_bitwise(lanes, row_format, col_format):
    s = ragged_system(2, integer=True)
    op = oracle.Operator.from_system(s)
    rng = np.random.default_rng(3)
    x = rng.integers(-8, 9, size=s.n).astype(np.float64)
    ybar = rng.integers(-8, 9, size=op.mbar).astype(np.float64)
    with from_sys(s, lanes_per_row=lanes, lanes_per_col=lanes, row_format=row_format,
                  col_format=col_format) as sol:
        yg = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        xg = sol.apply_t(torch.from_numpy(ybar).cuda()).cpu().numpy()
    assert np.array_equal(yg, op.apply(x))
    assert np.array_equal(xg, op.apply_t(ybar))


@pytest.mark.parametrize("row_format,col_format", [("csr", "csc"), ("csr", "runs"),
                                                    ("groups", "runs"), ("csr", "pairs")])
def test_operator_integer_bitwise_tomography_pattern(cfg0, row_format, col_format):
    # the tomography sparsity (runs of depth columns, merged across nodes) with
    # integer values: every sum is exact, so both row formats match bitwise
    s = synth.RandomSystem(m=cfg0.m, n=cfg0.n, nx=cfg0.nx, ny=cfg0.ny, nz=cfg0.nz,
                           row_ptr=cfg0.row_ptr, col=cfg0.col, val=np.rint(cfg0.val * 4),
                           dt=np.rint(cfg0.dt), damp=0.25, smooth=0.5)
    op = oracle.Operator.from_system(s)
    rng = np.random.default_rng(5)
    x = rng.integers(-8, 9, size=s.n).astype(np.float64)
    ybar = rng.integers(-8, 9, size=op.mbar).astype(np.float64)
    with from_sys(s, row_format=row_format, col_format=col_format) as sol:
        yg = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        xg = sol.apply_t(torch.from_numpy(ybar).cuda()).cpu().numpy()
    assert np.array_equal(yg, op.apply(x))
    assert np.array_equal(xg, op.apply_t(ybar))


def test_set_scale_in_place(cfg0):
    from paper_2604_11920_amd import LsqrError
    s = cfg0
    d = 2.0 ** np.random.default_rng(12).integers(-3, 4, s.n)
    op = oracle.Operator.from_system(s, d=d)
    x = np.random.default_rng(13).integers(-8, 9, size=s.n).astype(np.float64)
    with from_sys(s, precond="jacobi") as sol:
        sol.solve(s.dt, 4)                  # graphs captured with the Jacobi scale
        sol.set_scale(d)
        assert np.array_equal(sol.scale(), d)
        dm, _, _ = sol.solve(s.dt, 5)
        bad = d.copy()
        bad[3] = 0.0
        with pytest.raises(LsqrError):
            sol.set_scale(bad)
        assert np.array_equal(sol.scale(), d)
    ref = op.lsqr(s.dt, 5)
    assert rel(dm, ref["x"]) <= 1e-10


def test_jacobi_scale_within_rounding(cfg0):
    s = cfg0
    d = oracle.Operator.from_system(s).jacobi()
    with from_sys(s, precond="jacobi") as sol:
        dg = sol.scale()
    # sums of L_j positive squares in two orders: relative gap <= (L_j + 4) eps
    lcol = np.bincount(s.col, minlength=s.n)
    assert np.all(np.abs(dg - d) <= (lcol + 4) * 2.0 ** -52 * d)


@pytest.mark.parametrize("precond", ["none", "user"])
def test_operator_random_within_rounding(cfg0, precond):
    s = cfg0
    # a power-of-two column scale is applied exactly on both sides
    d = 2.0 ** np.random.default_rng(8).integers(-3, 4, s.n) if precond == "user" else None
    op = oracle.Operator.from_system(s, d=d)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(s.n)
    ybar = rng.standard_normal(op.mbar)
    with from_sys(s, precond=precond, col_scale=d) as sol:
        if d is not None:
            assert np.array_equal(sol.scale(), d)
        yg = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        xg = sol.apply_t(torch.from_numpy(ybar).cuda()).cpu().numpy()
    # two valid summation orders of an L-term sum differ by at most
    # 2 L eps sum|terms|; the 7-point rows have at most 7 terms of size <= 12 max|z|
    eps = 2.0 ** -52
    dd = np.ones(s.n) if d is None else d
    z = dd * x
    absG = sp.csr_matrix((np.abs(s.val), s.col, s.row_ptr), shape=(s.m, s.n))
    lr = np.diff(s.row_ptr)
    bd = np.r_[2 * (lr + 2) * eps * (absG @ np.abs(z)),
               np.full(s.n, 2 * 9 * eps * s.smooth * 12 * np.abs(z).max()),
               np.full(s.n, eps * s.damp * np.abs(z).max())]
    assert np.all(np.abs(yg - op.apply(x)) <= bd)
    yG, yL, yD = ybar[:s.m], ybar[s.m:s.m + s.n], ybar[s.m + s.n:]
    lc = np.bincount(s.col, minlength=s.n)
    bt = 2 * (lc + 4) * eps * dd * (absG.T @ np.abs(yG) + s.smooth * 12 * np.abs(yL).max()
                                    + s.damp * np.abs(yD))
    assert np.all(np.abs(xg - op.apply_t(ybar)) <= bt)


# --------------------------------------------------------------- solves -----
@pytest.mark.parametrize("precond,fmt", [("none", "auto"), ("jacobi", "auto"), ("none", "csc"),
                                         ("jacobi", "runs"), ("jacobi", "groups"),
                                         ("jacobi", "pairs")])
def test_early_iterates_strict(cfg0, precond, fmt):
    s = cfg0
    d = oracle.Operator.from_system(s).jacobi() if precond == "jacobi" else None
    op = oracle.Operator.from_system(s, d=d)
    rf, cf = FORMATS[fmt]
    with from_sys(s, precond=precond, row_format=rf, col_format=cf) as sol:
        for K in (1, 2, 3, 5, 8):
            ref = op.lsqr(s.dt, K)
            dm, hist, info = sol.solve(s.dt, K)
            assert info["iters"] == K and info["istop"] == 2
            assert rel(dm, ref["x"]) <= 1e-10, (K, rel(dm, ref["x"]))
            assert np.allclose(hist, ref["hist"], rtol=1e-10, atol=0), K


@pytest.mark.parametrize("precond,fmt", [("none", "auto"), ("jacobi", "auto"), ("none", "csc"),
                                         ("none", "runs"), ("none", "groups"), ("none", "pairs")])
def test_converged_strict(cfg0, cfg0_xstar, precond, fmt):
    s = cfg0
    d = oracle.Operator.from_system(s).jacobi() if precond == "jacobi" else None
    ref = oracle.Operator.from_system(s, d=d).lsqr(s.dt, 40000, tol=1e-13)
    rf, cf = FORMATS[fmt]
    with from_sys(s, precond=precond, row_format=rf, col_format=cf) as sol:
        dm, hist, info = sol.solve(s.dt, 40000, tol=1e-13)
    assert info["istop"] == 1 and ref["istop"] == 1
    assert info["eta"] <= 1e-13
    assert rel(dm, ref["x"]) <= 1e-10
    assert rel(dm, cfg0_xstar) <= 1e-10
    # the iteration counts of two valid summation orders differ only slightly
    assert abs(info["iters"] - ref["iters"]) <= 0.1 * ref["iters"]


def test_fixed_100_iterations(cfg0, cfg0_xstar):
    s = cfg0
    ref = oracle.lsqr(s, 100)
    with from_sys(s) as sol:
        dm, hist, info = sol.solve(s.dt, 100)
    assert info["iters"] == 100 and info["istop"] == 2
    # the oracle against itself (compensated vs plain sums) shows residual-norm
    # gaps up to 1.1e-3 relative around k = 20 on this system; allow 5x that
    assert np.all(np.abs(hist[:, 0] - ref["hist"][:, 0]) <= 5e-3 * ref["hist"][:, 0])
    assert abs(hist[-1, 0] - ref["hist"][-1, 0]) <= 1e-4 * ref["hist"][-1, 0]
    assert np.all(np.diff(hist[:, 0]) <= 1e-14 * hist[0, 0])       # monotone |r|
    gap = np.linalg.norm(dm - ref["x"])
    assert gap <= 0.1 * np.linalg.norm(ref["x"] - cfg0_xstar), gap


def test_tolerance_stop(cfg0):
    s = cfg0
    tol = 1e-6
    ref = oracle.lsqr(s, 20000, tol=tol)
    with from_sys(s, check_every=16) as sol:
        dm, hist, info = sol.solve(s.dt, 20000, tol=tol)
    assert info["istop"] == 1 and info["eta"] <= tol
    assert abs(info["iters"] - ref["iters"]) <= 0.1 * ref["iters"] + 2
    assert np.isnan(hist[info["iters"] + 1:]).all()
    # the estimate matches the explicit normal-equation residual of the returned dm
    eta, _ = eta_explicit(s, dm)
    assert eta <= 2 * tol


@pytest.mark.parametrize("fmt", ["auto", "csc", "runs", "groups", "pairs"])
def test_ragged_system_strict(fmt):
    s = ragged_system(5)
    rf, cf = FORMATS[fmt]
    for K in (1, 4, 8):
        ref = oracle.lsqr(s, K)
        with from_sys(s, row_format=rf, col_format=cf) as sol:
            dm, hist, info = sol.solve(s.dt, K)
        assert rel(dm, ref["x"]) <= 1e-10, K


@pytest.mark.parametrize("which", ["ragged", "cfg0", "no_entries"])
def test_pipelined_forward_rows(cfg0, which):
    # 64 lanes per row selects the pipelined forward product: solves use its
    # balanced row ranges, the plain products its strided rows; empty rows,
    # rows shorter than a batch and longer than several, and a system with no
    # stored entry at all
    if which == "ragged":
        s = ragged_system(7)
    elif which == "cfg0":
        s = cfg0
    else:
        s = synth.RandomSystem(m=300, n=60, nx=4, ny=3, nz=5, row_ptr=np.zeros(301, np.int64),
                               col=np.zeros(0, np.int32), val=np.zeros(0),
                               dt=np.random.default_rng(1).standard_normal(300), damp=0.1,
                               smooth=0.5)
    op = oracle.Operator.from_system(s)
    x = np.random.default_rng(5).standard_normal(s.n)
    with from_sys(s, lanes_per_row=64) as sol:
        for K in (1, 3, 8):
            ref = op.lsqr(s.dt, K)
            dm, hist, info = sol.solve(s.dt, K)
            assert info["istop"] == ref["istop"] and info["iters"] == ref["iters"]
            assert rel(dm, ref["x"]) <= 1e-10, (K, rel(dm, ref["x"]))
        y = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    yr = op.apply(x)
    assert np.abs(y - yr).max() <= 1e-12 * max(np.abs(yr).max(), 1.0)


def group_test_system(which, cfg0):
    if which == "ragged":
        return ragged_system(7)
    if which == "cfg0":
        return cfg0
    if which == "wide":       # 12,000 columns, rows of up to 1500: ~500 groups of a few rows
        return synth.random_system(3000, 40, 30, 10, row_len=(0, 1500), seed=11)
    # rays over a 30x30x8 grid: rows of one path at several periods share a group
    return synth.make_system(synth.small_config(nx=30, ny=30, nz=8, n_stations=24, n_periods=6,
                                                region=3.0))


@pytest.mark.parametrize("which", ["ragged", "cfg0", "wide", "paths"])
def test_row_groups_forward(cfg0, which):
    # row groups (each group's columns of D v staged in LDS, 16-bit slots per
    # entry; FP64 values two entries per lane and load): solves against the
    # oracle; the forward product against the oracle and the pipelined CSR rows
    s = group_test_system(which, cfg0)
    op = oracle.Operator.from_system(s)
    x = np.random.default_rng(5).standard_normal(s.n)
    with from_sys(s, row_format="groups") as sol:
        assert sol.kernel_stats()["row_format"] == 4
        for K in (1, 3, 8):
            ref = op.lsqr(s.dt, K)
            dm, hist, info = sol.solve(s.dt, K)
            assert info["istop"] == ref["istop"] and info["iters"] == ref["iters"]
            assert rel(dm, ref["x"]) <= 1e-10, (K, rel(dm, ref["x"]))
        yg = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    with from_sys(s, row_format="csr", lanes_per_row=64) as sol:
        yp = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    yr = op.apply(x)
    assert np.abs(yg - yr).max() <= 1e-12 * max(np.abs(yr).max(), 1.0)
    assert np.abs(yg - yp).max() <= 1e-12 * max(np.abs(yr).max(), 1.0)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_row_groups_reduced_precision(cfg0, precision):
    # the FP32 and quantised value types through the row groups: the same
    # iterates as the CSR rows up to the order of the partial sums of |t|^2
    # (the BF16 form refines to a tolerance: both solved to eta <= 1e-7)
    s = group_test_system("paths", cfg0)
    kw = dict(precision=precision, precond="jacobi")
    iters, tol = (6, 0.0) if precision == "fp32" else (5000, 1e-7)
    if precision == "bf16":
        kw.update(refine_sweeps=10)
    with from_sys(s, row_format="groups", **kw) as sol:
        ks = sol.kernel_stats()
        # aligned quads of FP32 values, octets of 16-bit codes
        assert ks["row_format"] == 4
        assert ks["fwd_entries_per_load"] == (4 if precision == "fp32" else 8)
        dg, _, ig = sol.solve(s.dt, iters, tol=tol)
    with from_sys(s, row_format="csr", **kw) as sol:
        dc, _, ic = sol.solve(s.dt, iters, tol=tol)
    if precision == "bf16":                  # both refinements reached the tolerance
        assert ig["istop"] == 1 and ic["istop"] == 1, (ig, ic)
    assert rel(dg, dc) <= 1e-4, rel(dg, dc)


def test_row_groups_refuse_rows_above_the_cap():
    from paper_2604_11920_amd import LsqrError
    n = 8000
    row_ptr = np.array([0, 3, 3 + 7169], np.int64)
    col = np.concatenate([[0, 5, 9], np.arange(7169)]).astype(np.int32)
    s = synth.RandomSystem(m=2, n=n, nx=40, ny=20, nz=10, row_ptr=row_ptr, col=col,
                           val=np.ones(len(col)), dt=np.ones(2), damp=0.1, smooth=0.5)
    with pytest.raises(LsqrError):
        from_sys(s, row_format="groups")
    with from_sys(s, row_format="csr") as sol:
        assert sol.kernel_stats()["row_format"] == 1


@pytest.mark.parametrize("fmt", ["auto", "csc", "runs", "groups", "pairs"])
def test_small_shapes(fmt):
    rf, cf = FORMATS[fmt]
    for grid in [(1, 1, 1), (1, 1, 3), (2, 1, 1), (3, 2, 1)]:
        s = synth.random_system(25, *grid, row_len=(0, 4), seed=sum(grid))
        ref = oracle.lsqr(s, 3)
        with from_sys(s, row_format=rf, col_format=cf) as sol:
            dm, hist, info = sol.solve(s.dt, 3)
        assert rel(dm, ref["x"]) <= 1e-10 or info["istop"] in (1, 3), grid


def test_degenerate_right_hand_sides(cfg0):
    with from_sys(cfg0) as sol:
        dm, hist, info = sol.solve(np.zeros(cfg0.m), 10)
        assert info["istop"] == 0 and np.all(dm == 0) and np.all(hist[0] == 0)
        dm, hist, info = sol.solve(cfg0.dt, 0)
        assert info["istop"] == 2 and info["iters"] == 0 and np.all(dm == 0)
        with pytest.raises(Exception):
            bad = cfg0.dt.copy()
            bad[17] = np.nan
            sol.solve(bad, 5)
    z = synth.RandomSystem(m=2, n=1, nx=1, ny=1, nz=1, row_ptr=np.array([0, 1, 2], np.int64),
                           col=np.zeros(2, np.int32), val=np.array([1.0, 1.0]),
                           dt=np.array([1.0, -1.0]), damp=0.1, smooth=0.5)
    with from_sys(z) as sol:
        dm, hist, info = sol.solve(z.dt, 10)
    assert info["istop"] == 0 and np.all(dm == 0)


def test_device_inputs_and_determinism(cfg0):
    s = cfg0
    with from_sys(s) as sol:
        dm_h, _, _ = sol.solve(s.dt, 60)
        dm_h2, _, _ = sol.solve(s.dt, 60)
    assert np.array_equal(dm_h, dm_h2)                    # run to run, bitwise
    with from_sys(s, graph=False) as sol:
        dm_e, _, _ = sol.solve(s.dt, 60)
    assert np.array_equal(dm_h, dm_e)                     # graph replay == eager
    dev = [torch.from_numpy(a).cuda() for a in (s.row_ptr, s.col, s.val)]
    with Solver(*dev, s.nx, s.ny, s.nz, s.damp, s.smooth) as sol:
        dm_d, _, _ = sol.solve(torch.from_numpy(s.dt).cuda(), 60)
    assert np.array_equal(dm_d.cpu().numpy(), dm_h)


def test_timing_counters(cfg0):
    with from_sys(cfg0, timing=True) as sol:
        dm, _, info = sol.solve(cfg0.dt, 20)
        ks = sol.kernel_stats()
    assert ks["fwd_launches"] == 20 and ks["adj_launches"] == 20
    assert ks["fwd_ms"] > 0 and ks["adj_ms"] > 0
    # at least the stored values and some index bytes; the CSC adds 4 per entry
    assert ks["fwd_bytes"] > 8 * cfg0.nnz and ks["adj_bytes"] > 8 * cfg0.nnz
    assert ks["col_format"] != 1 or ks["adj_bytes"] > 12 * cfg0.nnz
    with from_sys(cfg0) as sol:
        dm_g, _, _ = sol.solve(cfg0.dt, 20)
    assert np.array_equal(dm, dm_g)          # event timing does not change the arithmetic


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_depth_pairs_transposed(cfg0, precision):
    # the depth-pair layout of the node runs (k_adj_npair): the transposed
    # product against the oracle and the plain node runs, for every value
    # type, on systems with odd and even depth counts
    for s in (cfg0, synth.random_system(400, 5, 4, 9, row_len=(0, 60), seed=3),
              synth.random_system(300, 4, 3, 1, row_len=(0, 8), seed=5)):
        kw = dict(precision=precision, precond="jacobi")
        iters, tol = (6, 0.0) if precision != "bf16" else (5000, 1e-7)
        if precision == "bf16":
            kw.update(refine_sweeps=10)
        with from_sys(s, col_format="pairs", **kw) as sol:
            assert sol.kernel_stats()["col_format"] == 4
            dp, _, ip = sol.solve(s.dt, iters, tol=tol)
        with from_sys(s, col_format="runs", **kw) as sol:
            dr, _, ir = sol.solve(s.dt, iters, tol=tol)
        if precision == "bf16":              # both refinements reached the tolerance
            assert ip["istop"] == 1 and ir["istop"] == 1, (ip, ir)
        bar = 1e-10 if precision == "fp64" else 1e-4
        assert rel(dp, dr) <= bar, (s.nz, rel(dp, dr))
        if precision == "fp64":
            op = oracle.Operator.from_system(s)
            y = np.random.default_rng(2).standard_normal(op.mbar)
            with from_sys(s, col_format="pairs") as sol:
                xg = sol.apply_t(torch.from_numpy(y).cuda()).cpu().numpy()
            xr = op.apply_t(y)
            assert np.abs(xg - xr).max() <= 1e-12 * max(np.abs(xr).max(), 1.0)


@pytest.mark.parametrize("nz", [64, 63, 2])
def test_depth_pairs_deep_and_shallow_grids(nz):
    # the widest pair groups (32 lanes, two groups per wave), an odd depth
    # count whose last pair has one real depth, and a single pair
    s = synth.random_system(240, 2, 2, nz, row_len=(0, 3 * nz), seed=nz)
    op = oracle.Operator.from_system(s)
    y = np.random.default_rng(nz).standard_normal(op.mbar)
    with from_sys(s, col_format="pairs") as sol:
        assert sol.kernel_stats()["col_format"] == 4
        xg = sol.apply_t(torch.from_numpy(y).cuda()).cpu().numpy()
        for K in (1, 4):
            ref = op.lsqr(s.dt, K)
            dm, hist, info = sol.solve(s.dt, K)
            assert rel(dm, ref["x"]) <= 1e-10, (nz, K, rel(dm, ref["x"]))
    xr = op.apply_t(y)
    assert np.abs(xg - xr).max() <= 1e-12 * max(np.abs(xr).max(), 1.0)
    # the BF16 codes eight depths to a word (a lane owns depths 8k .. 8k+7)
    kw = dict(precision="bf16", precond="jacobi", refine_sweeps=10)
    with from_sys(s, col_format="pairs", **kw) as sol:
        dq, _, _ = sol.solve(s.dt, 5000, tol=1e-7)
    with from_sys(s, col_format="runs", **kw) as sol:
        dr, _, _ = sol.solve(s.dt, 5000, tol=1e-7)
    assert rel(dq, dr) <= 1e-4, (nz, rel(dq, dr))


@pytest.mark.parametrize("longest", [1024, 1025, 7168])
def test_row_groups_at_the_group_size_bounds(longest):
    # the group size is the longest row rounded up to 1024 columns: a row of
    # exactly 1024, one just above (group size 2048), and the largest allowed
    rng = np.random.default_rng(longest)
    n = 8000
    lens = rng.integers(0, 300, size=120)
    lens[17] = longest
    rows = [np.sort(rng.choice(n, size=L, replace=False)) for L in lens]
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    s = synth.RandomSystem(m=len(lens), n=n, nx=40, ny=20, nz=10, row_ptr=row_ptr, col=col,
                           val=rng.standard_normal(len(col)), dt=rng.standard_normal(len(lens)),
                           damp=0.1, smooth=0.5)
    op = oracle.Operator.from_system(s)
    x = rng.standard_normal(n)
    with from_sys(s, row_format="groups") as sol:
        assert sol.kernel_stats()["row_format"] == 4
        yg = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        ref = op.lsqr(s.dt, 3)
        dm, _, _ = sol.solve(s.dt, 3)
    with from_sys(s, row_format="csr", lanes_per_row=64) as sol:
        yp = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    yr = op.apply(x)
    assert np.abs(yg - yr).max() <= 1e-12 * max(np.abs(yr).max(), 1.0)
    assert np.abs(yg - yp).max() <= 1e-12 * max(np.abs(yr).max(), 1.0)
    assert rel(dm, ref["x"]) <= 1e-10


def test_row_groups_pairs_at_odd_bounds():
    # FP64 values two entries per lane: rows starting and ending at odd
    # positions, empty rows, and an odd entry count (the last pair reads the
    # padding element past the last entry)
    rng = np.random.default_rng(21)
    n = 1200
    lens = np.array([3, 0, 401, 400, 5, 1, 0, 777, 2, 2])
    assert lens.sum() % 2 == 1
    rows = [np.sort(rng.choice(n, size=L, replace=False)) for L in lens]
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    s = synth.RandomSystem(m=len(lens), n=n, nx=10, ny=12, nz=10, row_ptr=row_ptr, col=col,
                           val=rng.standard_normal(len(col)), dt=rng.standard_normal(len(lens)),
                           damp=0.1, smooth=0.5)
    op = oracle.Operator.from_system(s)
    x = rng.standard_normal(n)
    with from_sys(s, row_format="groups") as sol:
        assert sol.kernel_stats()["row_format"] == 4
        yg = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        ref = op.lsqr(s.dt, 4)
        dm, _, _ = sol.solve(s.dt, 4)
    yr = op.apply(x)
    assert np.abs(yg - yr).max() <= 1e-12 * max(np.abs(yr).max(), 1.0)
    assert rel(dm, ref["x"]) <= 1e-10
