"""Host-side logic of the learned column scale (no GPU): per-system centring
of the size-dependent features, the target families, the model file."""
import numpy as np

from paper_2604_11920_amd import learned


def test_centred_flagged_columns_only():
    f = np.random.default_rng(0).standard_normal((50, 6)) + 3.0
    c = learned.centred(f, learned.CENTRE)
    for k in range(6):
        if (learned.CENTRE >> k) & 1:
            assert abs(c[:, k].mean()) < 1e-12
            assert np.allclose(c[:, k] - c[:, k].mean(), f[:, k] - f[:, k].mean())
        else:
            assert np.array_equal(c[:, k], f[:, k])


def test_family_log_multiplier_depth_and_linear():
    nz = 4
    f = np.random.default_rng(1).standard_normal((3 * nz, 6))
    theta = np.array([0.5, -0.25, 0.0, 1.0, 0.3, -0.2])          # nz + 2 parameters
    l = learned.family_log_multiplier(f, theta, nz)
    iz = np.arange(3 * nz) % nz
    ref = theta[iz] + 0.3 * (f[:, 1] - f[:, 1].mean()) - 0.2 * (f[:, 5] - f[:, 5].mean())
    assert np.allclose(l, ref, rtol=0, atol=1e-15)
    th4 = np.array([0.1, 0.2, 0.3, 0.4])
    l4 = learned.family_log_multiplier(f, th4, nz)
    ref4 = 0.1 + 0.2 * f[:, 2] + 0.3 * (f[:, 1] - f[:, 1].mean()) + 0.4 * (f[:, 5] - f[:, 5].mean())
    assert np.allclose(l4, ref4, rtol=0, atol=1e-15)


def test_model_roundtrip(tmp_path):
    m = learned.ColumnScaleModel(params=learned.initial_params(3), mean=np.arange(6, dtype=np.float32),
                                 std=np.ones(6, np.float32), meta={"centre": learned.CENTRE, "x": 1})
    p = str(tmp_path / "m.npz")
    m.save(p)
    r = learned.ColumnScaleModel.load(p)
    assert np.array_equal(r.params, m.params) and r.centre == learned.CENTRE and r.meta["x"] == 1
    assert len(r.params) == learned.NPARAMS


def test_initial_model_is_jacobi():
    # the untrained net outputs softplus(z) ~ 1 for any input: W3 is small and
    # b3 = softplus^-1(1)
    p = learned.initial_params(0).astype(np.float64)
    assert abs(np.log1p(np.exp(p[-1])) - 1.0) < 1e-6
