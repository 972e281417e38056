"""Seeded synthetic surface-wave tomography systems G . dm ~ dt.

This module only generates inputs: station layouts, ray paths, the sensitivity
matrix G in CSR form, checkerboard models and noisy traveltime residuals.  It
holds none of the least-squares method's arithmetic (no Laplacian, no damping,
no LSQR) and is shared by the tests, the benchmark and the oracle's checks.

What it mimics from the paper:

* eq. (1): a row per (path, period); the traveltime residual is a sum over the
  lateral grid nodes k of bilinear interpolation coefficients v_ik times the
  slowness perturbation, with delta S = -delta C / C**2; written here in relative
  velocity perturbation units m = delta Vs / Vs so that G . 1 = -t_ref;
* eqs. (2)/(5): each lateral node contributes a run of consecutive depth
  columns (here a normalised Gaussian depth kernel instead of dispersion
  derivatives, which need a forward-modelling code);
* eq. (7): unknowns are ordered depth fastest, column = (iy*nx + ix)*nz + iz.

The bilinear split along a ray is exact: every polyline piece is cut at grid
lines and the four bilinear corner weights (quadratic along a straight piece)
are integrated with Simpson's rule.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

KM_PER_DEG = 111.195
_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_assemble.so")


# ----------------------------------------------------------------------------
# native row assembler (plain C, built with gcc)
# ----------------------------------------------------------------------------
def build_native(force: bool = True) -> str:
    """Compile synth/_assemble.c into synth/_assemble.so with gcc."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "_assemble.c")
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build_native(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        lib.synth_count.restype = ctypes.c_int64
        lib.synth_count.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, P]
        lib.synth_fill.restype = None
        lib.synth_fill.argtypes = [ctypes.c_int64, ctypes.c_int32] + [P] * 15
        lib.synth_count_rows.restype = ctypes.c_int64
        lib.synth_count_rows.argtypes = [ctypes.c_int64, ctypes.c_int32] + [P] * 6
        lib.synth_fill_rows.restype = None
        lib.synth_fill_rows.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32] + [P] * 15
        _lib_handle = lib
    return _lib_handle


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


# ----------------------------------------------------------------------------
# configuration
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Config:
    name: str
    region_deg: float            # square region side, degrees
    nx: int                      # lateral nodes in x (= y)
    ny: int
    z_nodes: tuple               # depth node positions, km
    n_stations: int
    periods: tuple               # periods, s
    min_wavelengths: float | None = None   # keep path if L >= min * lambda_T
    max_wavelengths: float | None = None   # keep path if L <= max * lambda_T
    bent: bool = False
    seed: int = 0
    damp: float = 0.1
    smooth: float = 0.5
    noise_frac: float = 0.005    # noise std as a fraction of t_ref
    checker_cells: int = 4       # checkerboard block size (cells)
    checker_amp: float = 0.05
    # closer to the paper's G: a ray of its own for every (pair, period) (the
    # paper traces each period's ray on that period's phase-velocity map) and
    # a depth kernel of its own for every lateral node (eq. (5): the depth
    # sensitivity follows the local model; here the kernel centre is scaled by
    # 1 + depth_factor_amp * a smooth lateral pattern)
    per_period_rays: bool = False
    depth_factor_amp: float = 0.0

    @property
    def nz(self) -> int:
        return len(self.z_nodes)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def h(self) -> float:
        return self.region_deg / (self.nx - 1)


def config0(seed: int = 0) -> Config:
    """Small plain-FP64 case: 16x16x9 grid, 40 stations, 780 pairs x 10 periods,
    straight rays, no wavelength filter."""
    return Config(name="cfg0", region_deg=1.5, nx=16, ny=16,
                  z_nodes=tuple(np.arange(9) * 5.0), n_stations=40,
                  periods=tuple(np.linspace(2.0, 20.0, 10)), seed=seed)


def config1(seed: int = 0, variant: str = "ge2", n_stations: int = 229,
            n_periods: int = 20) -> Config:
    """Paper-shaped case: 80x80x20 grid, 229 stations (the paper's array size),
    all pairs x 20 periods 1-40 s, bent rays, paths of >= 2 wavelengths
    (variant "2to8" also drops paths longer than 8 wavelengths)."""
    return Config(name=f"cfg1_{variant}_s{n_stations}_p{n_periods}", region_deg=10.0,
                  nx=80, ny=80, z_nodes=tuple(np.linspace(0.0, 80.0, 20)),
                  n_stations=n_stations, periods=tuple(np.linspace(1.0, 40.0, n_periods)),
                  min_wavelengths=2.0, max_wavelengths=8.0 if variant == "2to8" else None,
                  bent=True, seed=seed)


def config1_paperlike(seed: int = 0) -> Config:
    """Config 1's geometry and sizes with a bent ray of its own for every
    (pair, period) and node-dependent depth kernels (centre scaled by 0.8 ..
    1.2 over the lateral grid): no two periods of a pair share their lateral
    nodes, and no two nodes share their depth weights."""
    c = config1(seed=seed)
    c.per_period_rays = True
    c.depth_factor_amp = 0.2
    c.name = f"cfg1_paperlike_seed{seed}"
    return c


def depth_factor(nx, ny, amp):
    """Smooth lateral pattern in [1 - amp, 1 + amp], node order k = iy*nx + ix."""
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    f = np.sin(2.0 * np.pi * 1.5 * ix / max(nx - 1, 1)) * np.cos(2.0 * np.pi * 1.2 * iy / max(ny - 1, 1))
    return (1.0 + amp * f).reshape(-1)


def config3_systems() -> list[Config]:
    """Four uneven systems of the batched case: (stations, periods) =
    (60,10), (120,14), (180,17), (229,20), seeds 0..3."""
    out = []
    for s, (ns, npd) in enumerate([(60, 10), (120, 14), (180, 17), (229, 20)]):
        out.append(config1(seed=s, n_stations=ns, n_periods=npd))
    return out


def config0_variant(seed: int, n_stations: int, damp: float) -> Config:
    """Config-0 geometry (16x16x9 grid, 1.5 degree region, 10 periods 2-20 s,
    straight rays) with another station draw, station count and damping: the
    family the learned column scale is trained and evaluated on."""
    c = config0(seed)
    c.n_stations = int(n_stations)
    c.damp = float(damp)
    c.name = f"cfg0_s{n_stations}_d{damp:.3f}_seed{seed}"
    return c


def learned_family(first_seed: int, count: int, stations=(20, 60), damp=(0.05, 0.5)):
    """`count` config-0-variant systems with station counts uniform in
    `stations` and damping log-uniform in `damp`, seeds first_seed, ..."""
    rng = np.random.default_rng(first_seed * 7919 + count)
    out = []
    for i in range(count):
        ns = int(rng.integers(stations[0], stations[1] + 1))
        dp = float(np.exp(rng.uniform(np.log(damp[0]), np.log(damp[1]))))
        out.append(config0_variant(first_seed + i, ns, dp))
    return out


def learned_family_wide(first_seed: int, count: int, stations=(30, 80), periods=(6, 12),
                        damp=(0.05, 0.5)):
    """`count` systems of the config-1 geometry (80x80x20 grid, 10 degree
    region, bent rays, >= 2 wavelengths) with few stations and periods, so the
    learned scale also sees the large grid; seeds first_seed, ..."""
    rng = np.random.default_rng(first_seed * 104729 + count)
    out = []
    for i in range(count):
        ns = int(rng.integers(stations[0], stations[1] + 1))
        npd = int(rng.integers(periods[0], periods[1] + 1))
        dp = float(np.exp(rng.uniform(np.log(damp[0]), np.log(damp[1]))))
        c = config1(seed=first_seed + i, n_stations=ns, n_periods=npd)
        c.damp = dp
        c.name = f"cfg1_s{ns}_p{npd}_d{dp:.3f}_seed{first_seed + i}"
        out.append(c)
    return out


def learned_family_large(first_seed: int, count: int, stations=(100, 200), periods=(14, 20),
                         damp=(0.05, 0.2)):
    """`count` config-1-geometry systems near the benchmark's size (100-200
    stations, 14-20 periods), for the learned scale's targets."""
    return learned_family_wide(first_seed, count, stations=stations, periods=periods, damp=damp)


def c17_family(shape: str, first_seed: int, count: int) -> list[Config]:
    """The learned scale's training and held-out systems: for every seed,
    stations uniform in {30, ..., 229} and damping log-uniform in [0.05, 0.5]
    (drawn from a generator of their own, so a system depends on its seed
    only); shape "cfg0" keeps config 0's geometry (16x16x9 grid, 10 periods
    2-20 s, straight rays), "cfg1" config 1's (80x80x20 grid, 20 periods 1-40 s,
    bent rays, paths >= 2 wavelengths)."""
    if shape not in ("cfg0", "cfg1"):
        raise ValueError(shape)
    out = []
    for seed in range(first_seed, first_seed + count):
        rng = np.random.default_rng(10_000 + seed)
        ns = int(rng.integers(30, 230))
        dp = float(np.exp(rng.uniform(np.log(0.05), np.log(0.5))))
        c = config0(seed) if shape == "cfg0" else config1(seed=seed, n_stations=ns)
        c.n_stations = ns
        c.damp = dp
        c.name = f"c17{shape}_s{ns}_d{dp:.3f}_seed{seed}"
        out.append(c)
    return out


def load_config_file(path: str) -> dict:
    """A workload description (configs/config{0..4}.json) with its systems
    as Config objects: "systems" lists them, and "families" entries
    ({"family": "c17", "shape", "first_seed", "count"}) expand to the
    c17_family systems they name."""
    import json
    with open(path) as f:
        d = json.load(f)
    fields = {f.name for f in dataclasses.fields(Config)}

    def cfg(x):
        x = {k: v for k, v in x.items() if k in fields}
        x["z_nodes"] = tuple(float(z) for z in x["z_nodes"])
        x["periods"] = tuple(float(p) for p in x["periods"])
        return Config(**x)

    d["systems"] = [cfg(x) for x in d.get("systems", [])]
    for key, fams in d.get("families", {}).items():
        out = []
        for fam in fams:
            if fam.get("family") != "c17":
                raise ValueError(f"unknown family {fam.get('family')!r}")
            out += c17_family(fam["shape"], int(fam["first_seed"]), int(fam["count"]))
        d["families"][key] = out
    return d


def small_config(nx=8, ny=8, nz=6, n_stations=12, n_periods=5, region=0.7, bent=True,
                 seed=0, damp=0.1, smooth=0.5, min_wavelengths=None) -> Config:
    """A reduced geometry with the same structure, for fast tests."""
    return Config(name=f"small_{nx}x{ny}x{nz}_s{n_stations}", region_deg=region, nx=nx, ny=ny,
                  z_nodes=tuple(np.linspace(0.0, 5.0 * (nz - 1), nz)), n_stations=n_stations,
                  periods=tuple(np.linspace(2.0, 2.0 * (n_periods + 0.0), n_periods)),
                  min_wavelengths=min_wavelengths, bent=bent, seed=seed, damp=damp, smooth=smooth)


def phase_velocity(T):
    """Reference phase velocity c(T) = 2.8 + 0.03 T km/s."""
    return 2.8 + 0.03 * np.asarray(T, dtype=np.float64)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def depth_kernel(z_nodes, T, factor=1.0):
    """Normalised Gaussian depth weights for period T: centre T km (times
    `factor`), width 0.3 * centre, nodes below 1e-3 of the peak dropped.
    Returns (j0, w)."""
    z = np.asarray(z_nodes, dtype=np.float64)
    zc = float(T) * 1.0 * float(factor)
    sig = 0.3 * zc
    g = np.exp(-((z - zc) ** 2) / (2.0 * sig * sig))
    keep = np.nonzero(g >= 1e-3)[0]
    j0, j1 = int(keep[0]), int(keep[-1]) + 1
    assert np.all(g[j0:j1] >= 1e-3), "depth support must be contiguous"
    w = g[j0:j1] / np.sum(g[j0:j1])
    return j0, w


def polylines(sta_a, sta_b, h, region, bend_amp=None):
    """Ray polylines between station pairs, pieces no longer than h/4 (degrees).

    Returns (pt_ptr, px, py): pair p owns points pt_ptr[p]..pt_ptr[p+1]-1."""
    d = sta_b - sta_a
    D = np.hypot(d[:, 0], d[:, 1])
    npc = np.maximum(1, np.ceil(D * 1.05 / (h / 4.0)).astype(np.int64))
    pt_ptr = np.zeros(len(D) + 1, dtype=np.int64)
    pt_ptr[1:] = np.cumsum(npc + 1)
    pair_of_pt = np.repeat(np.arange(len(D)), npc + 1)
    local = np.arange(pt_ptr[-1]) - pt_ptr[pair_of_pt]
    s = local / npc[pair_of_pt]
    px = sta_a[pair_of_pt, 0] + s * d[pair_of_pt, 0]
    py = sta_a[pair_of_pt, 1] + s * d[pair_of_pt, 1]
    if bend_amp is not None:
        nrm = np.stack([-d[:, 1], d[:, 0]], axis=1) / np.maximum(D, 1e-300)[:, None]
        off = bend_amp[pair_of_pt] * np.sin(np.pi * s)
        px = px + off * nrm[pair_of_pt, 0]
        py = py + off * nrm[pair_of_pt, 1]
    px = np.clip(px, 0.0, region)
    py = np.clip(py, 0.0, region)
    return pt_ptr, px, py


def bilinear_split(pt_ptr, px, py, h, nx, ny):
    """Exact per-node path integrals of the bilinear hat functions.

    Returns (node_ptr, node_k, node_len_km, path_len_km): pair p touches lateral
    nodes node_k[node_ptr[p]:node_ptr[p+1]] (ascending, k = iy*nx + ix) with
    lengths node_len_km (km); path_len_km[p] is the polyline length."""
    npairs = len(pt_ptr) - 1
    last = np.zeros(len(px), dtype=bool)
    last[pt_ptr[1:] - 1] = True
    first_idx = np.nonzero(~last)[0]                       # piece = (i, i+1)
    pair_of_piece = np.searchsorted(pt_ptr, first_idx, side="right") - 1
    x0, y0 = px[first_idx], py[first_idx]
    x1, y1 = px[first_idx + 1], py[first_idx + 1]
    dx, dy = x1 - x0, y1 - y0
    plen = np.hypot(dx, dy)
    assert plen.size == 0 or plen.max() <= h / 4.0 * (1 + 1e-9), "pieces must be <= h/4"

    def crossing(a0, a1, da):
        i0, i1 = np.floor(a0 / h), np.floor(a1 / h)
        t = np.full(a0.shape, np.nan)
        msk = i0 != i1
        xc = np.maximum(i0[msk], i1[msk]) * h
        t[msk] = (xc - a0[msk]) / da[msk]
        return t

    tx = crossing(x0, x1, dx)
    ty = crossing(y0, y1, dy)
    t1 = np.fmin(tx, ty)
    t2 = np.fmax(tx, ty)
    t1 = np.where(np.isnan(t1), 1.0, t1)
    t2 = np.where(np.isnan(t2), 1.0, t2)
    ta = np.stack([np.zeros_like(t1), t1, t2], axis=1)        # [P, 3]
    tb = np.stack([t1, t2, np.ones_like(t1)], axis=1)
    ta, tb = ta.ravel(), tb.ravel()
    rep = np.repeat(np.arange(len(x0)), 3)
    seg = (tb - ta) * plen[rep] * KM_PER_DEG                  # sub-piece length, km
    ok = seg > 0.0
    ta, tb, rep, seg = ta[ok], tb[ok], rep[ok], seg[ok]
    X0, Y0, DX, DY = x0[rep], y0[rep], dx[rep], dy[rep]
    ax, ay = X0 + ta * DX, Y0 + ta * DY
    bx, by = X0 + tb * DX, Y0 + tb * DY
    mx, my = 0.5 * (ax + bx), 0.5 * (ay + by)
    ci = np.clip(np.floor(mx / h).astype(np.int64), 0, nx - 2)
    cj = np.clip(np.floor(my / h).astype(np.int64), 0, ny - 2)

    def corner_w(xx, yy):
        fx = xx / h - ci
        fy = yy / h - cj
        return ((1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy)

    wa, wm, wb = corner_w(ax, ay), corner_w(mx, my), corner_w(bx, by)
    contrib = np.stack([seg / 6.0 * (wa[c] + 4.0 * wm[c] + wb[c]) for c in range(4)], axis=1)
    nodes = np.stack([cj * nx + ci, cj * nx + ci + 1, (cj + 1) * nx + ci, (cj + 1) * nx + ci + 1],
                     axis=1)
    pp = pair_of_piece[rep]
    key = (pp[:, None] * (nx * ny) + nodes).ravel()
    val = contrib.ravel()
    order = np.argsort(key, kind="stable")
    key, val = key[order], val[order]
    starts = np.nonzero(np.r_[True, key[1:] != key[:-1]])[0]
    ukey = key[starts]
    ulen = np.add.reduceat(val, starts)
    keep = ulen > 0.0
    ukey, ulen = ukey[keep], ulen[keep]
    upair = ukey // (nx * ny)
    node_k = (ukey % (nx * ny)).astype(np.int32)
    node_ptr = np.zeros(npairs + 1, dtype=np.int64)
    np.add.at(node_ptr, upair + 1, 1)
    node_ptr = np.cumsum(node_ptr)
    path_len = np.zeros(npairs)
    np.add.at(path_len, pair_of_piece, plen * KM_PER_DEG)
    return node_ptr, node_k, ulen, path_len


# ----------------------------------------------------------------------------
# models
# ----------------------------------------------------------------------------
def checkerboard(nx, ny, nz, cells=4, amp=0.05, phase=1.0, depth_cells=None):
    """amp * phase * (-1)^(ix//cells + iy//cells + iz//depth_cells) in column
    order (iy*nx + ix)*nz + iz."""
    dc = cells if depth_cells is None else depth_cells
    iy, ix, iz = np.meshgrid(np.arange(ny), np.arange(nx), np.arange(nz), indexing="ij")
    sgn = 1.0 - 2.0 * ((ix // cells + iy // cells + iz // dc) % 2)
    return (amp * phase * sgn).reshape(-1).astype(np.float64)


# ----------------------------------------------------------------------------
# system
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class System:
    cfg: Config
    m: int
    n: int
    nx: int
    ny: int
    nz: int
    row_ptr: np.ndarray      # int64 [m+1]
    col: np.ndarray          # int32 [nnz]
    val: np.ndarray          # float64 [nnz]
    dt: np.ndarray           # float64 [m]
    m_true: np.ndarray       # float64 [n]
    t_ref: np.ndarray        # float64 [m]
    gm_true: np.ndarray      # float64 [m]  G . m_true (no noise)
    row_pair: np.ndarray     # int32 [m]
    row_period: np.ndarray   # int32 [m]
    periods: np.ndarray      # float64 [nper]
    path_len: np.ndarray     # float64 [npairs] km
    damp: float
    smooth: float
    # the rays G was built from (node_ptr, node_k, node_len, cvel, j0, nj,
    # w_ptr, w, keep [npairs * nper], nz): input of the device-side assembly
    rays: dict = dataclasses.field(default=None, repr=False)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.m, self.n))

    def matvec(self, x):
        """G . x via scipy (input generation helper)."""
        return self.scipy() @ np.asarray(x, dtype=np.float64)


def fingerprint(s) -> str:
    """SHA-256 of a generated system's sizes, row pointer, right-hand side and
    a stride of its column indices and values: identifies the system that
    stored reference results were computed for."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.array([s.m, s.n, s.nnz], dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(s.row_ptr).tobytes())
    h.update(np.ascontiguousarray(s.dt).tobytes())
    h.update(np.ascontiguousarray(s.col[::997]).tobytes())
    h.update(np.ascontiguousarray(s.val[::997]).tobytes())
    return h.hexdigest()


def _make_paperlike(cfg: Config, threads: int | None = None) -> System:
    """make_system for per-period rays and node-dependent depth kernels (see
    Config).  Draw order: stations, then per period the bends of all pairs,
    then the noise."""
    rng = np.random.default_rng(cfg.seed)
    R = cfg.region_deg
    sta = rng.uniform(0.0, R, size=(cfg.n_stations, 2))
    ia, ib = np.triu_indices(cfg.n_stations, k=1)
    a, b = sta[ia], sta[ib]
    npairs = len(ia)
    periods = np.asarray(cfg.periods, dtype=np.float64)
    nper = len(periods)
    cvel = phase_velocity(periods)
    lam = cvel * periods
    Dst = np.hypot(*(b - a).T)
    cnt = np.zeros((npairs, nper), dtype=np.int64)
    per_t = []
    path_len = np.zeros((npairs, nper))
    for t in range(nper):
        bend = rng.uniform(-0.05, 0.05, size=npairs) * Dst if cfg.bent else None
        pt_ptr, px, py = polylines(a, b, cfg.h, R, bend)
        node_ptr, node_k, node_len, plen = bilinear_split(pt_ptr, px, py, cfg.h, cfg.nx, cfg.ny)
        cnt[:, t] = np.diff(node_ptr)
        path_len[:, t] = plen
        per_t.append((node_ptr, node_k, node_len))
    path_ptr = np.zeros(npairs * nper + 1, dtype=np.int64)
    path_ptr[1:] = np.cumsum(cnt.reshape(-1))
    node_k = np.empty(path_ptr[-1], dtype=np.int32)
    node_len = np.empty(path_ptr[-1], dtype=np.float64)
    for t, (nptr, nk, nl) in enumerate(per_t):
        dst0 = path_ptr[np.arange(npairs) * nper + t]          # start of (p, t)
        rep = np.repeat(dst0 - nptr[:-1], np.diff(nptr))
        pos = np.arange(len(nk)) + rep
        node_k[pos] = nk
        node_len[pos] = nl
    keep = np.ones((npairs, nper), dtype=bool)
    if cfg.min_wavelengths is not None:
        keep &= path_len >= cfg.min_wavelengths * lam[None, :]
    if cfg.max_wavelengths is not None:
        keep &= path_len <= cfg.max_wavelengths * lam[None, :]
    keep &= cnt > 0
    # depth kernels per (lateral node, period)
    nn = cfg.nx * cfg.ny
    fac = depth_factor(cfg.nx, cfg.ny, cfg.depth_factor_amp)
    dj0 = np.zeros(nn * nper, dtype=np.int32)
    dnj = np.zeros(nn * nper, dtype=np.int32)
    wl = []
    for k in range(nn):
        for t, T in enumerate(periods):
            j, w = depth_kernel(cfg.z_nodes, T, fac[k])
            dj0[k * nper + t], dnj[k * nper + t] = j, len(w)
            wl.append(w)
    dw_ptr = np.zeros(nn * nper + 1, dtype=np.int64)
    dw_ptr[1:] = np.cumsum(dnj)
    dw = np.concatenate(wl)
    lib = _lib()
    keep_u8 = np.ascontiguousarray(keep.astype(np.uint8))
    m = lib.synth_count_rows(npairs, nper, _ptr(keep_u8), _ptr(path_ptr), _ptr(node_k),
                             _ptr(dnj), None, None, None)
    row_ptr = np.empty(m + 1, dtype=np.int64)
    row_pair = np.empty(m, dtype=np.int32)
    row_period = np.empty(m, dtype=np.int32)
    lib.synth_count_rows(npairs, nper, _ptr(keep_u8), _ptr(path_ptr), _ptr(node_k), _ptr(dnj),
                         _ptr(row_ptr), _ptr(row_pair), _ptr(row_period))
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    gm = np.empty(m, dtype=np.float64)
    m_true = checkerboard(cfg.nx, cfg.ny, cfg.nz, cfg.checker_cells, cfg.checker_amp)
    lib.synth_fill_rows(m, cfg.nz, nper, _ptr(row_ptr), _ptr(row_pair), _ptr(row_period),
                        _ptr(path_ptr), _ptr(node_k), _ptr(node_len), _ptr(cvel), _ptr(dj0),
                        _ptr(dnj), _ptr(dw_ptr), _ptr(dw), _ptr(m_true), _ptr(col), _ptr(val),
                        _ptr(gm))
    t_ref = path_len[row_pair, row_period] / cvel[row_period]
    noise = rng.standard_normal(m) * (cfg.noise_frac * t_ref)
    return System(cfg=cfg, m=int(m), n=cfg.n, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, row_ptr=row_ptr,
                  col=col, val=val, dt=gm + noise, m_true=m_true, t_ref=t_ref, gm_true=gm,
                  row_pair=row_pair, row_period=row_period, periods=periods,
                  path_len=path_len.mean(axis=1), damp=cfg.damp, smooth=cfg.smooth, rays=None)


def make_system(cfg: Config, threads: int | None = None) -> System:
    if cfg.per_period_rays or cfg.depth_factor_amp:
        return _make_paperlike(cfg, threads)
    rng = np.random.default_rng(cfg.seed)
    R = cfg.region_deg
    sta = rng.uniform(0.0, R, size=(cfg.n_stations, 2))
    ia, ib = np.triu_indices(cfg.n_stations, k=1)
    a, b = sta[ia], sta[ib]
    bend = None
    if cfg.bent:
        Dst = np.hypot(*(b - a).T)
        bend = rng.uniform(-0.05, 0.05, size=len(ia)) * Dst
    pt_ptr, px, py = polylines(a, b, cfg.h, R, bend)
    node_ptr, node_k, node_len, path_len = bilinear_split(pt_ptr, px, py, cfg.h, cfg.nx, cfg.ny)
    npairs = len(ia)
    # the polylines as a ray tracer would hand them over: points and the
    # length of every piece (point i to i + 1; unused at a path's last point)
    plen = np.zeros(len(px))
    plen[:-1] = np.hypot(px[1:] - px[:-1], py[1:] - py[:-1])
    plen[pt_ptr[1:] - 1] = 0.0
    periods = np.asarray(cfg.periods, dtype=np.float64)
    cvel = phase_velocity(periods)
    lam = cvel * periods
    keep = np.ones((npairs, len(periods)), dtype=bool)
    if cfg.min_wavelengths is not None:
        keep &= path_len[:, None] >= cfg.min_wavelengths * lam[None, :]
    if cfg.max_wavelengths is not None:
        keep &= path_len[:, None] <= cfg.max_wavelengths * lam[None, :]
    keep &= (node_ptr[1:] > node_ptr[:-1])[:, None]
    j0 = np.zeros(len(periods), dtype=np.int32)
    nj = np.zeros(len(periods), dtype=np.int32)
    wl = []
    for t, T in enumerate(periods):
        j, w = depth_kernel(cfg.z_nodes, T)
        j0[t], nj[t] = j, len(w)
        wl.append(w)
    w_ptr = np.zeros(len(periods) + 1, dtype=np.int64)
    w_ptr[1:] = np.cumsum(nj)
    wflat = np.concatenate(wl)

    lib = _lib()
    keep_u8 = np.ascontiguousarray(keep.astype(np.uint8))
    m = lib.synth_count(npairs, len(periods), _ptr(keep_u8), _ptr(node_ptr), _ptr(nj),
                        None, None, None)
    row_ptr = np.empty(m + 1, dtype=np.int64)
    row_pair = np.empty(m, dtype=np.int32)
    row_period = np.empty(m, dtype=np.int32)
    lib.synth_count(npairs, len(periods), _ptr(keep_u8), _ptr(node_ptr), _ptr(nj),
                    _ptr(row_ptr), _ptr(row_pair), _ptr(row_period))
    nnz = int(row_ptr[-1])
    assert nnz < 2**62
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    gm = np.empty(m, dtype=np.float64)
    m_true = checkerboard(cfg.nx, cfg.ny, cfg.nz, cfg.checker_cells, cfg.checker_amp)
    node_k = np.ascontiguousarray(node_k, dtype=np.int32)
    node_len = np.ascontiguousarray(node_len, dtype=np.float64)
    old = os.environ.get("OMP_NUM_THREADS")
    if threads is not None:
        os.environ["OMP_NUM_THREADS"] = str(threads)
    lib.synth_fill(m, cfg.nz, _ptr(row_ptr), _ptr(row_pair), _ptr(row_period), _ptr(node_ptr),
                   _ptr(node_k), _ptr(node_len), _ptr(cvel), _ptr(j0), _ptr(nj), _ptr(w_ptr),
                   _ptr(wflat), _ptr(m_true), _ptr(col), _ptr(val), _ptr(gm))
    if threads is not None:
        if old is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = old
    t_ref = path_len[row_pair] / cvel[row_period]
    noise = rng.standard_normal(m) * (cfg.noise_frac * t_ref)
    dt = gm + noise
    return System(cfg=cfg, m=int(m), n=cfg.n, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, row_ptr=row_ptr,
                  col=col, val=val, dt=dt, m_true=m_true, t_ref=t_ref, gm_true=gm,
                  row_pair=row_pair, row_period=row_period, periods=periods, path_len=path_len,
                  damp=cfg.damp, smooth=cfg.smooth,
                  rays=dict(node_ptr=node_ptr, node_k=node_k, node_len=node_len, cvel=cvel,
                            j0=j0, nj=nj, w_ptr=w_ptr, w=wflat, keep=keep_u8.reshape(-1),
                            nz=cfg.nz,
                            polyline=dict(pt_ptr=pt_ptr, px=px, py=py, plen=plen, h=cfg.h,
                                          nx=cfg.nx, ny=cfg.ny, km_per_deg=KM_PER_DEG)))


# ----------------------------------------------------------------------------
# right-hand-side batches (resolution tests and bootstrap noise draws)
# ----------------------------------------------------------------------------
def checker_rhs_batch(sys: System, n_checker: int = 16, n_boot: int = 16) -> np.ndarray:
    """[m, n_checker + n_boot] right-hand sides, column r:

    * r < n_checker: checkerboard with block size 2 + floor(6 r / 15) cells,
      +-5 %, sign phase negated for odd r, plus 0.5 % noise drawn with seed 200 + r;
    * otherwise: G . m_true plus a fresh 0.5 % noise draw with seed 100 + (r - n_checker).
    """
    G = sys.scipy()
    out = np.empty((sys.m, n_checker + n_boot), dtype=np.float64)
    for r in range(n_checker):
        cells = 2 + (6 * r) // 15
        mr = checkerboard(sys.nx, sys.ny, sys.nz, cells, 0.05, -1.0 if r % 2 else 1.0)
        noise = np.random.default_rng(200 + r).standard_normal(sys.m)
        out[:, r] = G @ mr + noise * (sys.cfg.noise_frac * sys.t_ref)
    for r in range(n_boot):
        noise = np.random.default_rng(100 + r).standard_normal(sys.m)
        out[:, n_checker + r] = sys.gm_true + noise * (sys.cfg.noise_frac * sys.t_ref)
    return out


# ----------------------------------------------------------------------------
# generic random sparse systems on a grid (for kernel and edge-case tests)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class RandomSystem:
    m: int
    n: int
    nx: int
    ny: int
    nz: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    dt: np.ndarray
    damp: float
    smooth: float

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self):
        A = np.zeros((self.m, self.n))
        for i in range(self.m):
            s, e = self.row_ptr[i], self.row_ptr[i + 1]
            A[i, self.col[s:e]] = self.val[s:e]
        return A


def random_system(m, nx, ny, nz, row_len=(0, 12), seed=0, integer=False, damp=0.1,
                  smooth=0.5, max_abs=8) -> RandomSystem:
    """Random CSR with sorted unique columns per row.  integer=True draws values
    and dt from the integers in [-max_abs, max_abs] (exact in FP32 and FP64)."""
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    lens = rng.integers(row_len[0], min(row_len[1], n) + 1, size=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(lens)
    col = np.empty(row_ptr[-1], dtype=np.int32)
    for i in range(m):
        col[row_ptr[i]:row_ptr[i + 1]] = np.sort(rng.choice(n, size=lens[i], replace=False))
    if integer:
        val = rng.integers(-max_abs, max_abs + 1, size=row_ptr[-1]).astype(np.float64)
        dt = rng.integers(-max_abs, max_abs + 1, size=m).astype(np.float64)
    else:
        val = rng.standard_normal(row_ptr[-1])
        dt = rng.standard_normal(m)
    return RandomSystem(m=m, n=n, nx=nx, ny=ny, nz=nz, row_ptr=row_ptr, col=col, val=val, dt=dt,
                        damp=damp, smooth=smooth)
