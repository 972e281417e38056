"""Host side of the device-side assembly of G from the rays (no GPU): the
row and entry counts of lsqr_rays_size equal the generator's for several
geometries (including paths dropped by the wavelength rule), and malformed
rays are refused."""
import numpy as np
import pytest

import synth


def lib_or_skip():
    try:
        from paper_2604_11920_amd import rays_size  # noqa: F401
        from paper_2604_11920_amd import load
        load()
    except (ImportError, OSError) as e:
        pytest.skip(f"library not built: {e}")


@pytest.mark.parametrize("cfg", [
    synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4, region=0.5),
    synth.small_config(nx=7, ny=6, nz=5, n_stations=12, n_periods=6, region=0.8,
                       min_wavelengths=1.0),
    synth.config0()])
def test_sizes_match_generator(cfg):
    lib_or_skip()
    from paper_2604_11920_amd import rays_size
    s = synth.make_system(cfg)
    assert rays_size(s.rays) == (s.m, s.nnz)


def test_malformed_rays_refused():
    lib_or_skip()
    from paper_2604_11920_amd import LsqrError, rays_size
    s = synth.make_system(synth.small_config(nx=5, ny=4, nz=4, n_stations=8, n_periods=4,
                                             region=0.5))
    bad = []
    r = dict(s.rays); r["j0"] = np.asarray(r["j0"]) + s.nz; bad.append(r)
    r = dict(s.rays); r["w_ptr"] = np.asarray(r["w_ptr"]).copy(); r["w_ptr"][-1] += 1; bad.append(r)
    r = dict(s.rays); r["node_ptr"] = np.asarray(r["node_ptr"]).copy(); r["node_ptr"][1] = -1
    bad.append(r)
    r = dict(s.rays); r["node_len"] = np.asarray(r["node_len"]).copy(); r["node_len"][0] = np.nan
    bad.append(r)
    r = dict(s.rays); r["cvel"] = np.zeros_like(np.asarray(r["cvel"])); bad.append(r)
    r = dict(s.rays); r["node_k"] = np.asarray(r["node_k"]).copy(); r["node_k"][0] = -3
    bad.append(r)
    for r in bad:
        with pytest.raises(LsqrError):
            rays_size(r)
