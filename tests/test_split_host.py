"""The bilinear split of the ray polylines that the device assembly runs
(paper_2604_11920_amd/csrc/split_path.h), compiled for the host with g++
(-ffp-contract=off) and run on the generator's polylines: node lists and
node lengths bitwise equal to the generator's own split (synth.bilinear_split,
NumPy), for straight and bent rays on several grids, including the paths
along grid lines and through cell corners that the crossing logic and the
corner clipping have to get right."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "split_check.cpp")
INC = os.path.join(ROOT, "paper_2604_11920_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("split") / "split_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-I", INC, SRC, "-o", exe],
                   check=True)
    return exe


def run_split(exe, tmp, pl):
    fin, fout = str(tmp / "in.bin"), str(tmp / "out.bin")
    pt = np.asarray(pl["pt_ptr"], np.int64)
    with open(fin, "wb") as f:
        np.array([len(pt) - 1, len(pl["px"]), pl["nx"], pl["ny"]], np.int64).tofile(f)
        np.array([pl["h"], pl["km_per_deg"]], np.float64).tofile(f)
        pt.tofile(f)
        for k in ("px", "py", "plen"):
            np.asarray(pl[k], np.float64).tofile(f)
    subprocess.run([exe, fin, fout], check=True)
    buf = open(fout, "rb").read()
    np_ = len(pt) - 1
    node_ptr = np.frombuffer(buf, np.int64, np_ + 1, 0)
    tot = int(np.frombuffer(buf, np.int64, 1, 8 * (np_ + 1))[0])
    off = 8 * (np_ + 2)
    node_k = np.frombuffer(buf, np.int32, tot, off)
    node_len = np.frombuffer(buf, np.float64, tot, off + 4 * tot)
    return node_ptr, node_k, node_len


def check(exe, tmp, pl):
    node_ptr, node_k, node_len, _ = synth.bilinear_split(pl["pt_ptr"], pl["px"], pl["py"], pl["h"],
                                                          pl["nx"], pl["ny"])
    a, b, c = run_split(exe, tmp, pl)
    assert np.array_equal(a, node_ptr)
    assert np.array_equal(b, node_k)
    assert np.array_equal(c.view(np.int64), np.asarray(node_len, np.float64).view(np.int64))


@pytest.mark.parametrize("cfg", [
    synth.config0(),
    synth.small_config(nx=12, ny=11, nz=7, n_stations=24, n_periods=6, region=1.1, seed=5),
    synth.small_config(nx=9, ny=9, nz=5, n_stations=30, n_periods=4, region=0.8, bent=False, seed=3),
])
def test_split_matches_generator(driver, tmp_path, cfg):
    s = synth.make_system(cfg)
    check(driver, tmp_path, s.rays["polyline"])


def test_split_grid_aligned_paths(driver, tmp_path):
    """Paths along grid lines, through node corners, diagonal, with points on
    the lines and the region edge."""
    h, nx, ny = 0.25, 6, 5
    region = h * (nx - 1)
    ends = [((0.0, 0.5), (1.25, 0.5)), ((0.25, 0.0), (0.25, 1.0)), ((0.0, 0.0), (1.0, 1.0)),
            ((1.25, 1.0), (0.0, 0.0)), ((0.3, 0.7), (0.3, 0.2)), ((0.1, 0.1), (1.2, 0.95))]
    a = np.array([e[0] for e in ends])
    b = np.array([e[1] for e in ends])
    pt_ptr, px, py = synth.polylines(a, b, h, region)
    plen = np.zeros(len(px))
    plen[:-1] = np.hypot(px[1:] - px[:-1], py[1:] - py[:-1])
    plen[pt_ptr[1:] - 1] = 0.0
    pl = dict(pt_ptr=pt_ptr, px=px, py=py, plen=plen, h=h, nx=nx, ny=ny,
              km_per_deg=synth.KM_PER_DEG)
    check(driver, tmp_path, pl)
