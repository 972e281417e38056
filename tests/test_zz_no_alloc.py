"""lsqr_mlp_scale_noalloc (the learned-scale inference with its temporaries in
the library's static device scratch instead of an allocation) against
lsqr_mlp_scale, through the C ABI: bitwise equal results (the same kernels
run on the same inputs), on consecutive calls whose second system is smaller
than the first, and back again (the scratch keeps the previous call's
contents, which no call may read); a system larger than the scratch is
refused with a status code before any kernel runs."""
import numpy as np
import pytest

import synth
from oracle import mlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _model(seed):
    theta = mlp.init_params(seed) + 0.2 * np.random.default_rng(seed + 1).standard_normal(
        mlp.NPARAMS)
    return torch.from_numpy(theta.astype(np.float32)).cuda()


def _pair(sol, p, mean, std, centre):
    feat = sol.column_features()
    ref = sol.mlp_scale(p, mean, std, feat=feat, centre=centre)
    d = torch.full((sol.n,), float("nan"), dtype=torch.float64, device="cuda")
    sol.mlp_scale_noalloc(p, mean, std, feat, d, centre=centre)
    torch.cuda.synchronize()
    return ref, d


def test_noalloc_equals_allocating_entry_point():
    from paper_2604_11920_amd import Solver
    big = synth.make_system(synth.config0())
    small = synth.make_system(synth.small_config(nx=8, ny=8, nz=6, n_stations=16, n_periods=5,
                                                 region=0.7))
    assert small.n < big.n
    p = _model(3)
    mean = np.array([0.5, 1.0, 0.5, 0.3, 0.1, 1.0], np.float32)
    std = np.array([1.0, 2.0, 0.3, 0.2, 0.1, 1.5], np.float32)
    centre = (1 << 0) | (1 << 5)
    with Solver.from_system(big) as sb, Solver.from_system(small) as ss:
        outs = []
        for sol in (sb, ss, sb):          # larger, then smaller, then larger again
            ref, d = _pair(sol, p, mean, std, centre)
            print(f"[noalloc] n={sol.n}: max |d - ref| = {(d - ref).abs().max().item():.3e}",
                  flush=True)
            assert torch.isfinite(d).all()
            assert torch.equal(d.view(torch.int64), ref.view(torch.int64))
            outs.append(d.clone())
        assert torch.equal(outs[0].view(torch.int64), outs[2].view(torch.int64))


def test_noalloc_refuses_more_columns_than_the_scratch():
    from paper_2604_11920_amd import LsqrError, Solver
    from paper_2604_11920_amd import lsqr as L
    nx, ny, nz = 128, 130, 64                 # 1,064,960 columns > 2^20
    n = nx * ny * nz
    row_ptr = np.array([0, 2, 3], np.int64)
    col = np.array([0, n - 1, 7], np.int32)
    val = np.array([1.0, -2.0, 0.5])
    with Solver(row_ptr, col, val, nx, ny, nz, damp=0.1, smooth=0.5) as sol:
        p = _model(1)
        feat = torch.zeros((n, 6), dtype=torch.float32, device="cuda")
        d = torch.zeros(n, dtype=torch.float64, device="cuda")
        with pytest.raises(LsqrError) as ei:
            sol.mlp_scale_noalloc(p, np.zeros(6, np.float32), np.ones(6, np.float32), feat, d)
        assert ei.value.status == L.LSQR_E_INVALID_ARG
        assert "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert int(torch.count_nonzero(d)) == 0
