"""GPU checks of the batched (multi right-hand side, several systems) path.

* The block products on integer data are exact in FP32 and FP64, so they
  equal the oracle's products of every column bitwise.
* Every right-hand side of a batched solve follows its own LSQR: early
  iterates match the FP64 oracle's single-RHS iterates to FP32 accuracy, and
  converged right-hand sides land within FP32 reach of the oracle's x*.
* Uneven systems, padding (nrhs not a power of two), zero right-hand sides,
  per-RHS freezing at the tolerance, determinism and the autotuner.
"""
import json

import numpy as np
import pytest

import oracle
import synth

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
def small_systems():
    """Three uneven tomography systems (different grids, stations, periods)."""
    out = []
    for i, (nx, ns, npd) in enumerate([(6, 10, 4), (8, 14, 5), (7, 18, 6)]):
        out.append(synth.make_system(synth.small_config(nx=nx, ny=nx + 1, nz=5, n_stations=ns,
                                                        n_periods=npd, region=0.7, seed=i)))
    return out


@pytest.mark.parametrize("R", [1, 8, 32])
def test_block_products_integer_bitwise(R):
    cfg0 = synth.make_system(synth.config0())
    s = synth.RandomSystem(m=cfg0.m, n=cfg0.n, nx=cfg0.nx, ny=cfg0.ny, nz=cfg0.nz,
                           row_ptr=cfg0.row_ptr, col=cfg0.col, val=np.rint(cfg0.val * 4),
                           dt=np.rint(cfg0.dt), damp=0.25, smooth=0.5)
    op = oracle.Operator.from_system(s)
    rng = np.random.default_rng(R)
    X = rng.integers(-8, 9, size=(s.n, R)).astype(np.float32)
    Y = rng.integers(-8, 9, size=(op.mbar, R)).astype(np.float32)
    with from_sys(s) as sol:
        yg = sol.apply_block(torch.from_numpy(X).cuda()).cpu().numpy()
        xg = sol.apply_t_block(torch.from_numpy(Y).cuda()).cpu().numpy()
    for r in range(R):
        assert np.array_equal(yg[:, r].astype(np.float64), op.apply(X[:, r].astype(np.float64)))
        assert np.array_equal(xg[:, r].astype(np.float64), op.apply_t(Y[:, r].astype(np.float64)))


def rhs_block(s, nrhs, seed=0):
    """Checkerboards of several sizes plus noise draws, as [m, nrhs]."""
    B = synth.checker_rhs_batch(s, n_checker=(nrhs + 1) // 2, n_boot=nrhs // 2)
    return B[:, :nrhs]


def test_batched_early_iterates_follow_oracle(small_systems):
    from paper_2604_11920_amd import solve_batched
    nrhs = 6
    sols = [from_sys(s) for s in small_systems]
    dts = [rhs_block(s, nrhs, i) for i, s in enumerate(small_systems)]
    K = 5
    dms, hists, infos = solve_batched(sols, dts, K)
    for s, dm, h, inf, dt in zip(small_systems, dms, hists, infos, dts):
        op = oracle.Operator.from_system(s)
        for r in range(nrhs):
            ref = op.lsqr(dt[:, r], K)
            assert inf[r]["iters"] == K and inf[r]["istop"] == 2
            assert rel(dm[:, r], ref["x"]) <= 1e-4, (r, rel(dm[:, r], ref["x"]))
            assert np.allclose(h[:, r, 0], ref["hist"][:, 0], rtol=1e-5)
    for sol in sols:
        sol.close()


def test_batched_converges_per_rhs(small_systems):
    from paper_2604_11920_amd import solve_batched
    nrhs = 5                      # padded to 8 internally
    tol = 1e-5
    sols = [from_sys(s, precond="jacobi", check_every=8) for s in small_systems]
    dts = [rhs_block(s, nrhs) for s in small_systems]
    dts[1][:, 2] = 0.0            # a zero right-hand side
    dms, hists, infos = solve_batched(sols, dts, 4000, tol=tol)
    for si, (s, dm, inf, dt) in enumerate(zip(small_systems, dms, infos, dts)):
        for r in range(nrhs):
            if si == 1 and r == 2:
                assert inf[r]["istop"] == 0 and np.all(dm[:, r] == 0)
                continue
            assert inf[r]["istop"] == 1 and inf[r]["eta"] <= tol, (si, r, inf[r])
            # the FP64 oracle stopped at the same tolerance, and x*
            ref = oracle.Operator.from_system(s).lsqr(dt[:, r], 20000, tol=tol)["x"]
            xs = oracle.Operator.from_system(s).lsqr(dt[:, r], 40000, tol=1e-12)["x"]
            assert rel(dm[:, r], xs) <= 3 * rel(ref, xs) + 1e-4, (si, r)
    for sol in sols:
        sol.close()


def test_batched_deterministic_and_graph_equal(small_systems):
    from paper_2604_11920_amd import solve_batched
    nrhs = 8
    dts = [rhs_block(s, nrhs) for s in small_systems]
    sols = [from_sys(s) for s in small_systems]
    a, _, _ = solve_batched(sols, dts, 40)
    b, _, _ = solve_batched(sols, dts, 40)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    for sol in sols:
        sol.close()
    sols = [from_sys(s, graph=False) for s in small_systems]
    c, _, _ = solve_batched(sols, dts, 40)
    for x, y in zip(a, c):
        assert np.array_equal(x, y)
    for sol in sols:
        sol.close()


@pytest.mark.parametrize("grid", [256, 1024])
def test_batched_32_wide_tiles_follow_oracle(small_systems, grid):
    # 32-wide tiles take the matrix-core forms: the two-phase forward product
    # (per-run partial rows, then per-row sums) and the transposed product
    # reduced over runs on the matrix cores
    from paper_2604_11920_amd import solve_batched
    nrhs = 32
    dts = [rhs_block(s, nrhs, i) for i, s in enumerate(small_systems)]
    sols = [from_sys(s) for s in small_systems]
    try:
        for sol in sols:
            sol.set_batch_config(32, grid)
        dm, _, infos = solve_batched(sols, dts, 5)
        dm2, _, _ = solve_batched(sols, dts, 5)
    finally:
        for sol in sols:
            sol.close()
    for i, s in enumerate(small_systems):
        ref = oracle.Operator.from_system(s)
        assert np.array_equal(dm[i], dm2[i])              # fixed summation orders
        for r in (0, 9, 31):
            assert rel(dm[i][:, r], ref.lsqr(dts[i][:, r], 5)["x"]) <= 1e-4, (i, r)


def test_autotune_and_cache(small_systems, tmp_path):
    from paper_2604_11920_amd import solve_batched
    s = small_systems[2]
    nrhs = 32
    cache = str(tmp_path / "sched.json")
    dt = rhs_block(s, nrhs)
    with from_sys(s) as sol:
        t = sol.autotune_batched(nrhs, probe_iters=4, cache=cache)
        assert t["rhs_tile"] in (8, 16, 32) and t["grid"] in (256, 512, 1024, 2048)
        assert not t["cached"] and t["ms_per_iter"] > 0
        t2 = sol.autotune_batched(nrhs, cache=cache)
        assert t2["cached"] and t2["rhs_tile"] == t["rhs_tile"]
        dm, _, inf = solve_batched([sol], [dt], 5)
    table = json.load(open(cache))
    assert len(table) == 1
    # the tuned schedule keeps the FP32 bar of the early-iterate test; past ~8
    # iterations FP32 iterates drift from the FP64 ones by loss of orthogonality
    ref = oracle.Operator.from_system(s)
    for r in (0, 17, 31):
        assert rel(dm[0][:, r], ref.lsqr(dt[:, r], 5)["x"]) <= 1e-4
