"""The host-side index builders (csrc/runs_host.h: node runs, their padded
layouts, row groups, the row order of the node runs) and the ray split shared
with the device assembly (csrc/split_path.h), built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer (no recovery: the first
report ends the program with a non-zero status) and run on the test systems
of their functional checks.  Each sanitized driver must exit cleanly and
write exactly what the plain build writes.  CPU only; the device code is not
built here."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
INC = os.path.join(ROOT, "paper_2604_11920_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _build(tmp, src, extra, sanitize):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp / (os.path.splitext(src)[0] + ("_san" if sanitize else "")))
    cmd = [gxx, "-std=c++17", *extra, "-I", INC, os.path.join(NATIVE, src), "-o", exe]
    cmd[1:1] = SAN if sanitize else ["-O2"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if sanitize and r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("the sanitizer runtime is not installed")
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


@pytest.fixture(scope="module")
def runs_exes(tmp_path_factory):
    tmp = tmp_path_factory.mktemp("san_runs")
    return (_build(tmp, "runs_check.cpp", ["-pthread"], False),
            _build(tmp, "runs_check.cpp", ["-pthread"], True))


@pytest.fixture(scope="module")
def split_exes(tmp_path_factory):
    tmp = tmp_path_factory.mktemp("san_split")
    return (_build(tmp, "split_check.cpp", ["-ffp-contract=off"], False),
            _build(tmp, "split_check.cpp", ["-ffp-contract=off"], True))


def _run(exe, args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]


def _runs_input(path, row_ptr, col, n, nz):
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int32)
    with open(path, "wb") as f:
        np.array([len(row_ptr) - 1, n, nz, len(col)], np.int64).tofile(f)
        row_ptr.tofile(f)
        col.tofile(f)


def _runs_cases():
    s = synth.make_system(synth.small_config(nx=8, ny=8, nz=6, n_stations=14, seed=2))
    yield "small", s.row_ptr, s.col, s.n, s.nz, 4096
    yield "small_cap64", s.row_ptr, s.col, s.n, s.nz, 64
    r = synth.random_system(300, 5, 4, 6, row_len=(0, 30), seed=4)
    yield "ragged", r.row_ptr, r.col, r.n, r.nz, 4096
    # empty rows only
    yield "empty", np.zeros(6, np.int64), np.zeros(0, np.int32), 24, 4, 4096


@pytest.mark.parametrize("case", [c[0] for c in _runs_cases()])
def test_runs_builders_clean_under_sanitizers(runs_exes, tmp_path, case):
    plain, san = runs_exes
    name, row_ptr, col, n, nz, cap = next(c for c in _runs_cases() if c[0] == case)
    fin = str(tmp_path / "in.bin")
    _runs_input(fin, row_ptr, col, n, nz)
    outs = []
    for exe in (plain, san):
        fout = str(tmp_path / (os.path.basename(exe) + ".out"))
        _run(exe, [fin, fout, str(cap)])
        outs.append(open(fout, "rb").read())
    assert outs[0] == outs[1]


def _split_input(path, pl):
    pt = np.asarray(pl["pt_ptr"], np.int64)
    with open(path, "wb") as f:
        np.array([len(pt) - 1, len(pl["px"]), pl["nx"], pl["ny"]], np.int64).tofile(f)
        np.array([pl["h"], pl["km_per_deg"]], np.float64).tofile(f)
        pt.tofile(f)
        for k in ("px", "py", "plen"):
            np.asarray(pl[k], np.float64).tofile(f)


@pytest.mark.parametrize("bent", [False, True])
def test_split_clean_under_sanitizers(split_exes, tmp_path, bent):
    plain, san = split_exes
    cfg = synth.small_config(nx=12, ny=11, nz=5, n_stations=20, n_periods=4, region=1.1,
                             bent=bent, seed=5)
    pl = synth.make_system(cfg).rays["polyline"]
    fin = str(tmp_path / "in.bin")
    _split_input(fin, pl)
    outs = []
    for exe in (plain, san):
        fout = str(tmp_path / (os.path.basename(exe) + ".out"))
        _run(exe, [fin, fout])
        outs.append(open(fout, "rb").read())
    assert outs[0] == outs[1]
