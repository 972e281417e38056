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


@pytest.mark.parametrize("cfg", [
    synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4, region=0.5),
    synth.small_config(nx=12, ny=11, nz=7, n_stations=24, n_periods=6, region=1.1, seed=5),
    synth.small_config(nx=9, ny=9, nz=5, n_stations=30, n_periods=4, region=0.8, bent=False,
                       seed=3),
    synth.config0()])
def test_polyline_split_and_assembly_bitwise(cfg):
    """The bilinear split of the ray polylines on the device (node lists and
    lengths) and G assembled from it: bitwise equal to the generator's."""
    from paper_2604_11920_amd import assemble_polylines, split_polylines
    s = synth.make_system(cfg)
    node_ptr, node_k, node_len = split_polylines(s.rays["polyline"])
    print(f"[split] {cfg.name}: {len(node_ptr) - 1} paths, {int(node_ptr[-1])} nodes", flush=True)
    assert np.array_equal(node_ptr, s.rays["node_ptr"])
    assert np.array_equal(node_k.cpu().numpy(), s.rays["node_k"])
    assert np.array_equal(node_len.cpu().numpy().view(np.uint64),
                          np.asarray(s.rays["node_len"]).view(np.uint64))
    rp, col, val = assemble_polylines(s.rays)
    assert np.array_equal(rp.cpu().numpy(), s.row_ptr)
    assert np.array_equal(col.cpu().numpy(), s.col)
    assert np.array_equal(val.cpu().numpy().view(np.uint64), s.val.view(np.uint64))


def test_polyline_refusals():
    from paper_2604_11920_amd import LsqrError, split_polylines
    s = synth.make_system(synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4,
                                             region=0.5))
    pl = dict(s.rays["polyline"])
    bad = dict(pl, px=np.array(pl["px"], copy=True))
    bad["px"][3] = np.nan
    with pytest.raises(LsqrError):
        split_polylines(bad)
    long_piece = dict(pl, px=np.array(pl["px"], copy=True))
    long_piece["px"][1] = long_piece["px"][0] + 1.5 * pl["h"]     # spans a whole cell
    with pytest.raises(LsqrError):
        split_polylines(long_piece)
    with pytest.raises(LsqrError):
        split_polylines(dict(pl, h=0.0))
    # no paths: an empty split
    empty = dict(pl, pt_ptr=np.zeros(1, np.int64), px=np.zeros(0), py=np.zeros(0),
                 plen=np.zeros(0))
    node_ptr, node_k, node_len = split_polylines(empty)
    assert node_ptr.tolist() == [0] and node_k.numel() == 0
