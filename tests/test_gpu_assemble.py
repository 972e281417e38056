"""GPU checks of the device-side assembly of G from the rays: bitwise equal
to the generator's CSR (structure and FP64 values) on several geometries,
including dropped paths, and a context created from the device arrays
solving exactly as one created from the host arrays."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.mark.parametrize("cfg", [
    synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4, region=0.5),
    synth.small_config(nx=7, ny=6, nz=5, n_stations=12, n_periods=6, region=0.8,
                       min_wavelengths=1.0),
    synth.config0()])
def test_assembly_bitwise_equals_generator(cfg):
    from paper_2604_11920_amd import assemble_rays
    s = synth.make_system(cfg)
    rp, col, val = assemble_rays(s.rays)
    assert np.array_equal(rp.cpu().numpy(), s.row_ptr)
    assert np.array_equal(col.cpu().numpy(), s.col)
    assert np.array_equal(val.cpu().numpy().view(np.uint64), s.val.view(np.uint64))


def test_context_from_device_assembly_solves_identically():
    from paper_2604_11920_amd import Solver, assemble_rays
    s = synth.make_system(synth.config0())
    rp, col, val = assemble_rays(s.rays)
    with Solver(rp, col, val, s.nx, s.ny, s.nz, damp=s.damp, smooth=s.smooth,
                precond="jacobi") as a, Solver.from_system(s, precond="jacobi") as b:
        xa, ha, ia = a.solve(s.dt, 50)
        xb, hb, ib = b.solve(s.dt, 50)
    assert np.array_equal(xa, xb) and np.array_equal(ha, hb)


def test_no_rows():
    from paper_2604_11920_amd import assemble_rays, rays_size
    s = synth.make_system(synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4,
                                             region=0.5))
    r = dict(s.rays)
    r["keep"] = np.zeros_like(np.asarray(r["keep"]))
    assert rays_size(r) == (0, 0)
    rp, col, val = assemble_rays(r)
    assert rp.cpu().numpy().tolist() == [0] and col.numel() == 0 and val.numel() == 0
