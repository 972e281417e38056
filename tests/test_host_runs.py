"""CPU checks of the host builders of the index formats (no GPU).

The forward product's row groups and the transposed product's node runs (and
their padded layouts) are built on the host from the CSR structure
(csrc/runs_host.h); the kernels index memory with them, so they are checked
here exhaustively against the CSR they describe: every stored entry covered
exactly once, node runs maximal and in ascending row order, value offsets
and quarter offsets consistent, the node order a stable sort by decreasing
run count, and the row order of the node runs (the batched forward
product's per-row sums) a permutation listing each row's runs in the order
of its stored entries.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "runs_check.cpp")
INC = os.path.join(ROOT, "paper_2604_11920_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("runs") / "runs_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", "-I", INC, SRC, "-o", exe], check=True)
    return exe


def run_builders(exe, tmp, row_ptr, col, n, nz, cap=4096):
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int32)
    m, nnz = len(row_ptr) - 1, len(col)
    fin, fout = str(tmp / "in.bin"), str(tmp / "out.bin")
    with open(fin, "wb") as f:
        np.array([m, n, nz, nnz], np.int64).tofile(f)
        row_ptr.tofile(f)
        col.tofile(f)
    subprocess.run([exe, fin, fout, str(cap)], check=True)
    buf = open(fout, "rb").read()
    pos = 0

    def take(dt, k):
        nonlocal pos
        a = np.frombuffer(buf, dtype=dt, count=k, offset=pos)
        pos += a.nbytes
        return a

    out = {}
    ok2, nr2, nn = take(np.int64, 3)
    out["nodes_ok"] = bool(ok2)
    if ok2:
        out["nrp"] = take(np.int64, nn + 1)
        out["nvq"] = take(np.int64, 4 * nn + 1)
        out["row"] = take(np.uint32, nr2)
        out["src"] = take(np.uint32, nr2)
        out["dst"] = take(np.uint32, nr2)
        out["desc"] = take(np.uint16, nr2)
        out["order"] = take(np.int32, nn)
    if ok2:
        out["rrp"] = take(np.int64, m + 1)
        out["rrid"] = take(np.uint32, nr2)
    ok5, ng5, nc5 = take(np.int64, 3)
    out["groups_ok"] = bool(ok5)
    if ok5:
        out["gp"] = take(np.int32, ng5 + 1)
        out["gcp"] = take(np.int64, ng5 + 1)
        out["gcol"] = take(np.int32, nc5)
        out["slot"] = take(np.uint16, len(col))
    for W in ((2, 4, 8) if ok2 else ()):
        ok6, tot6 = take(np.int64, 2)
        out[f"pairs_ok{W}"] = bool(ok6)
        out[f"pad_total{W}"] = int(tot6)
        out[f"dstp{W}"] = take(np.uint32, nr2)
        out[f"nvqp{W}"] = take(np.int64, 4 * nn + 1)
    assert pos == len(buf)
    return out


def check_row_groups(o, row_ptr, col, cap):
    """Groups tile the rows in order; each group's list is the sorted set of
    its rows' columns (at most cap); every entry's slot points at its column;
    a group is closed only when the next row would not fit."""
    gp, gcp, gcol, slot = (o[k] for k in ("gp", "gcp", "gcol", "slot"))
    m = len(row_ptr) - 1
    assert gp[0] == 0 and gp[-1] == m and np.all(np.diff(gp) >= 1)
    assert gcp[0] == 0 and gcp[-1] == len(gcol) and np.all(np.diff(gcp) >= 0)
    for g in range(len(gp) - 1):
        p0, p1 = row_ptr[gp[g]], row_ptr[gp[g + 1]]
        lst = gcol[gcp[g]:gcp[g + 1]]
        assert np.array_equal(lst, np.unique(col[p0:p1]))
        assert len(lst) <= cap
        sl = slot[p0:p1].astype(np.int64)
        assert np.all(sl < len(lst))
        assert np.array_equal(lst[sl], col[p0:p1])
        if g + 2 < len(gp):                        # greedy: the next row did not fit
            nxt = col[row_ptr[gp[g + 1]]:row_ptr[gp[g + 1] + 1]]
            assert len(np.union1d(lst, nxt)) > cap


def check_node_runs(o, row_ptr, col, n, nz):
    nrp, nvq, row, src, dst, desc, order = (o[k] for k in
                                            ("nrp", "nvq", "row", "src", "dst", "desc", "order"))
    nn = n // nz
    nnz = len(col)
    assert nrp[0] == 0 and np.all(np.diff(nrp) >= 0) and nrp[-1] == len(row)
    iz0 = (desc >> 8).astype(np.int64)
    ln = (desc & 255).astype(np.int64)
    assert np.all(ln >= 1) and np.all(iz0 + ln <= nz)
    # values: node-major, consecutive
    assert np.array_equal(dst.astype(np.int64), np.concatenate([[0], np.cumsum(ln)[:-1]]))
    covered = np.zeros(nnz, np.int64)
    for k in range(nn):
        r0, r1 = nrp[k], nrp[k + 1]
        key_prev = None
        for r in range(r0, r1):
            i, s, a, L = int(row[r]), int(src[r]), int(iz0[r]), int(ln[r])
            assert row_ptr[i] <= s and s + L <= row_ptr[i + 1]
            assert np.array_equal(col[s:s + L], k * nz + a + np.arange(L))
            # maximal within the node: the entries before/after are not adjacent
            if s > row_ptr[i] and a > 0:
                assert col[s - 1] != k * nz + a - 1
            if s + L < row_ptr[i + 1] and a + L < nz:
                assert col[s + L] != k * nz + a + L
            covered[s:s + L] += 1
            key = (i, a)
            if key_prev is not None:
                assert key > key_prev
            key_prev = key
        c = r1 - r0
        end = dst[r1 - 1] + ln[r1 - 1] if c else (nvq[4 * k] if k else 0)
        for w in range(4):
            q = r0 + c * w // 4
            assert nvq[4 * k + w] == (dst[q] if q < r1 else end)
    assert nvq[4 * nn] == nnz
    assert np.all(covered == 1)
    counts = np.diff(nrp)
    assert np.array_equal(order, np.argsort(-counts, kind="stable"))


def test_small_config(driver, tmp_path):
    s = synth.make_system(synth.small_config(nx=8, ny=8, nz=6, n_stations=14, seed=2))
    o = run_builders(driver, tmp_path, s.row_ptr, s.col, s.n, s.nz)
    assert o["nodes_ok"]
    check_node_runs(o, s.row_ptr, s.col, s.n, s.nz)


def test_full_depth_rows_cross_node_boundaries(driver, tmp_path):
    # every row covers all depths of consecutive lateral nodes: node runs
    # split each row at every node boundary
    nx, ny, nz = 6, 5, 4
    n = nx * ny * nz
    rng = np.random.default_rng(3)
    rows = []
    for _ in range(40):
        k0 = int(rng.integers(0, nx * ny - 3))
        k1 = k0 + int(rng.integers(1, 4))
        rows.append(np.arange(k0 * nz, k1 * nz))
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])])
    col = np.concatenate(rows)
    o = run_builders(driver, tmp_path, rp, col, n, nz)
    check_node_runs(o, rp, col, n, nz)
    assert len(o["row"]) == sum(len(r) // nz for r in rows)


def test_random_structure_with_gaps_and_empty_rows(driver, tmp_path):
    nx, ny, nz = 7, 3, 9
    n = nx * ny * nz
    rng = np.random.default_rng(5)
    rows = []
    for i in range(300):
        if i % 17 == 0:
            rows.append(np.zeros(0, np.int64))
            continue
        keep = rng.random(n) < rng.uniform(0.02, 0.6)
        rows.append(np.nonzero(keep)[0])
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])])
    col = np.concatenate(rows)
    o = run_builders(driver, tmp_path, rp, col, n, nz)
    check_node_runs(o, rp, col, n, nz)


def test_node_runs_refused_for_deep_grids(driver, tmp_path):
    n, nz = 130, 65
    rp = np.array([0, 3])
    col = np.array([0, 1, 70])
    o = run_builders(driver, tmp_path, rp, col, n, nz)
    assert not o["nodes_ok"]


def test_config0(driver, tmp_path):
    s = synth.make_system(synth.config0())
    o = run_builders(driver, tmp_path, s.row_ptr, s.col, s.n, s.nz)
    # node runs: vectorised subset of the checks (the system is ~1M entries)
    nrp, row, src, desc, dst = o["nrp"], o["row"], o["src"], o["desc"], o["dst"]
    ln = (desc & 255).astype(np.int64)
    iz0 = (desc >> 8).astype(np.int64)
    node = np.repeat(np.arange(len(nrp) - 1), np.diff(nrp))
    assert ln.sum() == s.nnz
    starts = src.astype(np.int64)
    assert np.array_equal(s.col[starts], node * s.nz + iz0)
    last = starts + ln - 1
    assert np.array_equal(s.col[last], node * s.nz + iz0 + ln - 1)
    assert np.all(s.row_ptr[row] <= starts) and np.all(last < s.row_ptr[row.astype(np.int64) + 1])
    cov = np.zeros(s.nnz + 1, np.int64)
    np.add.at(cov, starts, 1)
    np.add.at(cov, last + 1, -1)
    assert np.all(np.cumsum(cov)[:-1] == 1)
    assert np.array_equal(dst.astype(np.int64), np.concatenate([[0], np.cumsum(ln)[:-1]]))


def check_row_order(o, row_ptr, col, nz):
    """rrid lists every node run once; row i's runs are those with row i, and
    their stored entries, taken in the listed order, are row i's entries in
    CSR order (so per-run partial sums are added in entry order)."""
    rrp, rrid, row, src, desc = o["rrp"], o["rrid"], o["row"], o["src"], o["desc"]
    m = len(row_ptr) - 1
    assert rrp[0] == 0 and rrp[-1] == len(row) and np.all(np.diff(rrp) >= 0)
    assert np.array_equal(np.sort(rrid), np.arange(len(row)))
    for i in range(m):
        ids = rrid[rrp[i]:rrp[i + 1]].astype(np.int64)
        assert np.all(row[ids] == i)
        ent = np.concatenate([src[r] + np.arange(desc[r] & 255) for r in ids]) if len(ids) else \
            np.zeros(0, np.int64)
        assert np.array_equal(ent, np.arange(row_ptr[i], row_ptr[i + 1]))


def test_row_order_of_runs(driver, tmp_path):
    for s in (synth.make_system(synth.small_config(nx=6, ny=5, nz=4, n_stations=10, seed=2)),
              synth.random_system(300, 5, 4, 6, row_len=(0, 40), seed=9)):
        o = run_builders(driver, tmp_path, s.row_ptr, s.col, s.n, s.nz)
        assert o["nodes_ok"]
        check_row_order(o, s.row_ptr, s.col, s.nz)


def test_row_groups(driver, tmp_path):
    s = synth.make_system(synth.small_config(nx=8, ny=8, nz=6, n_stations=14, seed=2))
    longest = int(np.diff(s.row_ptr).max())
    for cap in (4096, 3 * longest, longest):
        o = run_builders(driver, tmp_path, s.row_ptr, s.col, s.n, s.nz, cap=cap)
        assert o["groups_ok"]
        check_row_groups(o, s.row_ptr, s.col, cap)
    assert len(o["gp"]) > 10
    assert not run_builders(driver, tmp_path, s.row_ptr, s.col, s.n, s.nz, cap=longest - 1)["groups_ok"]
    # random structure with gaps and empty rows (an empty row joins any group)
    nx, ny, nz = 7, 3, 9
    n = nx * ny * nz
    rng = np.random.default_rng(5)
    rows = [np.zeros(0, np.int64) if i % 17 == 0 else np.nonzero(rng.random(n) < rng.uniform(0.02, 0.6))[0]
            for i in range(300)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])])
    col = np.concatenate(rows)
    for cap in (n, 150):
        o = run_builders(driver, tmp_path, rp, col, n, nz, cap=cap)
        assert o["groups_ok"]
        check_row_groups(o, rp, col, cap)


def test_row_groups_refused_for_a_row_above_the_cap(driver, tmp_path):
    rp = np.array([0, 3, 8])
    col = np.array([0, 1, 2, 0, 1, 2, 3, 4])
    assert run_builders(driver, tmp_path, rp, col, 10, 1, cap=5)["groups_ok"]
    o = run_builders(driver, tmp_path, rp, col, 10, 1, cap=4)
    assert not o["groups_ok"]


def check_pair_layout(o, nz, W=2):
    """Depth-pair (W = 2), four-depth (W = 4) and eight-depth (W = 8)
    layouts: every run's depth
    iz sits at an index congruent to iz mod W (depths Wk .. Wk+W-1 share an
    aligned word), runs do not overlap, the padding is below W values on each
    side, and the quarter offsets are the padded starts of the quarters'
    first runs."""
    nrp, desc = o["nrp"], o["desc"]
    dstp, nvqp, total = o[f"dstp{W}"].astype(np.int64), o[f"nvqp{W}"], o[f"pad_total{W}"]
    iz0 = (desc >> 8).astype(np.int64)
    ln = (desc & 255).astype(np.int64)
    start = dstp - (iz0 % W)                    # padded start of each run
    plen = -(-(ln + iz0 % W) // W) * W
    assert np.all(start % W == 0) and np.all((dstp - iz0) % W == 0)
    assert np.array_equal(start[1:], start[:-1] + plen[:-1]) and start[0] == 0
    assert total == start[-1] + plen[-1]
    assert total - ln.sum() <= 2 * (W - 1) * len(ln)
    nn = len(nrp) - 1
    for k in range(nn):
        r0, r1 = nrp[k], nrp[k + 1]
        c = r1 - r0
        end = start[r1 - 1] + plen[r1 - 1] if c else None
        for w in range(4):
            q = r0 + c * w // 4
            exp = start[q] if q < r1 else (end if c else None)
            if exp is not None:
                assert nvqp[4 * k + w] == exp
    assert nvqp[4 * nn] == total


def test_pair_layout(driver, tmp_path):
    for s in (synth.make_system(synth.small_config(nx=8, ny=8, nz=6, n_stations=14, seed=2)),
              synth.random_system(300, 5, 4, 9, row_len=(0, 40), seed=9),
              synth.random_system(200, 3, 3, 1, row_len=(0, 6), seed=4)):
        o = run_builders(driver, tmp_path, s.row_ptr, s.col, s.n, s.nz)
        assert o["nodes_ok"] and o["pairs_ok2"] and o["pairs_ok4"] and o["pairs_ok8"]
        check_node_runs(o, s.row_ptr, s.col, s.n, s.nz)     # nz = 6, 9 and 1
        for W in (2, 4, 8):
            check_pair_layout(o, s.nz, W)
