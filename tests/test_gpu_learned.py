"""GPU checks of the learned column scale.

* Features (FP64 sums, stored FP32) match the oracle's features.
* The training gradient (FP32) matches the oracle's FP64 gradient to 1e-4
  relative; a few Adam steps on the GPU follow the oracle's Adam.
* BF16 inference matches the FP64 reference multiplier to ~1e-2 relative, and
  any learned scale leaves the solution unchanged (learned vs Jacobi at the
  tolerance: <= 1e-5, the judge), with the Jacobi fallback for bad scales.
* If a trained model is present, it does not need more iterations than Jacobi
  on held-out systems on average (the gain test).
"""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2604_11920_amd", "colscale_mlp.npz")


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


def test_features_match_oracle(cfg0):
    s = cfg0
    ref = mlp.column_features(s.row_ptr, s.col, s.val, s.nx, s.ny, s.nz, s.damp, s.smooth)
    with from_sys(s) as sol:
        f = sol.column_features().cpu().numpy().astype(np.float64)
    for k in range(6):
        assert np.allclose(f[:, k], ref[:, k], rtol=2e-6, atol=2e-6), k


def batch(seed, B=512):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, 6)), rng.standard_normal(B) * 0.3


def test_training_gradient_matches_oracle():
    from paper_2604_11920_amd import Trainer
    theta = mlp.init_params(5) + 0.05 * np.random.default_rng(1).standard_normal(mlp.NPARAMS)
    x, t = batch(2)
    L, g = mlp.grad(theta, x, t)
    tr = Trainer(theta.astype(np.float32), 512)
    gg, lg = tr.grad(torch.from_numpy(x.astype(np.float32)).cuda(),
                     torch.from_numpy(t.astype(np.float32)).cuda())
    gg = gg.cpu().numpy().astype(np.float64)
    tr.close()
    assert abs(lg - L) <= 1e-5 * L
    assert np.linalg.norm(gg - g) <= 1e-4 * np.linalg.norm(g)


def test_adam_steps_follow_oracle():
    from paper_2604_11920_amd import Trainer
    theta = mlp.init_params(7)
    tr = Trainer(theta.astype(np.float32), 512)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    th = theta.copy()
    for step in range(1, 6):
        x, t = batch(10 + step)
        _, g = mlp.grad(th, x, t)
        th, m, v = mlp.adam_step(th, m, v, g, step, lr=1e-3)
        tr.step(torch.from_numpy(x.astype(np.float32)).cuda(),
                torch.from_numpy(t.astype(np.float32)).cuda(), 1e-3)
    p = tr.params().astype(np.float64)
    tr.close()
    assert np.linalg.norm(p - th) <= 1e-4 * np.linalg.norm(th - theta) + 1e-6


def test_bf16_inference_matches_reference(cfg0):
    s = cfg0
    theta = mlp.init_params(3) + 0.2 * np.random.default_rng(4).standard_normal(mlp.NPARAMS)
    feat = mlp.column_features(s.row_ptr, s.col, s.val, s.nx, s.ny, s.nz, s.damp, s.smooth)
    mean, std = feat.mean(0), feat.std(0)
    std[std == 0] = 1.0
    djac = oracle.Operator.from_system(s).jacobi()
    ref = djac * mlp.multiplier(theta, (feat - mean) / std)
    with from_sys(s) as sol:
        p = torch.from_numpy(theta.astype(np.float32)).cuda()
        d = sol.mlp_scale(p, mean.astype(np.float32), std.astype(np.float32)).cpu().numpy()
    r = np.abs(d / ref - 1)
    assert np.median(r) < 1e-2 and r.max() < 6e-2


def test_bf16_inference_centred_features(cfg0):
    # flagged features are centred on the system's own means (computed by the
    # library); the reference centres the oracle's FP64 features the same way
    s = cfg0
    theta = mlp.init_params(6) + 0.2 * np.random.default_rng(9).standard_normal(mlp.NPARAMS)
    feat = mlp.column_features(s.row_ptr, s.col, s.val, s.nx, s.ny, s.nz, s.damp, s.smooth)
    centre = (1 << 0) | (1 << 1) | (1 << 5)
    mean, std = feat.mean(0) * 0.5, feat.std(0)
    std[std == 0] = 1.0
    mu = mean.copy()
    for f in range(6):
        if (centre >> f) & 1:
            mu[f] = feat[:, f].mean()
    djac = oracle.Operator.from_system(s).jacobi()
    ref = djac * mlp.multiplier(theta, (feat - mu) / std)
    with from_sys(s) as sol:
        p = torch.from_numpy(theta.astype(np.float32)).cuda()
        d = sol.mlp_scale(p, mean.astype(np.float32), std.astype(np.float32),
                          centre=centre).cpu().numpy()
    r = np.abs(d / ref - 1)
    assert np.median(r) < 1e-2 and r.max() < 6e-2


def test_any_positive_scale_keeps_the_solution_and_bad_scales_fall_back(cfg0):
    s = cfg0
    theta = mlp.init_params(3) + 0.2 * np.random.default_rng(4).standard_normal(mlp.NPARAMS)
    from paper_2604_11920_amd import learned
    model = learned.ColumnScaleModel(params=theta.astype(np.float32),
                                     mean=np.zeros(6, np.float32), std=np.ones(6, np.float32),
                                     meta={})
    tol = 1e-10
    with from_sys(s, precond="jacobi") as sol:
        dj, _, ij = sol.solve(s.dt, 20000, tol=tol)
    dl, il = learned.solve_learned(s, model, tol, k_jacobi=ij["iters"])
    assert il["istop"] == 1 and rel(dl, dj) <= 1e-5          # the judge
    bad = np.ones(s.n)
    bad[5] = -1.0
    with from_sys(s, precond="user", col_scale=bad) as sol:
        db, _, ib = sol.solve(s.dt, 20000, tol=tol)
    assert ib["fallback_used"] == 1 and rel(db, dj) <= 1e-8


@pytest.mark.skipif(not os.path.exists(MODEL), reason="no trained model in the tree")
def test_trained_model_gain_on_heldout():
    from paper_2604_11920_amd import learned
    model = learned.ColumnScaleModel.load(MODEL)
    tol = 1e-6
    ratios = []
    for cfg in synth.learned_family(1001, 6):
        s = synth.make_system(cfg)
        kj, _ = learned.iterations_to_tol(s, None, tol, 20000)
        dl, il = learned.solve_learned(s, model, tol, k_jacobi=kj)
        with from_sys(s, precond="jacobi") as sol:
            dj, _, _ = sol.solve(s.dt, 20000, tol=tol)
        assert il["istop"] == 1
        assert rel(dl, dj) <= 1e-3           # both stopped at eta <= 1e-6
        ratios.append(il["iters_total"] / kj)
        print(f"[learned] {cfg.name}: jacobi {kj} learned {il['iters']}")
    assert np.mean(ratios) <= 1.0
