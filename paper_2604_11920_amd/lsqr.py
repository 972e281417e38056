"""Thin ctypes binding of the C ABI in include/lsqr_mi355x.h.

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch supplies device memory (its caching allocator is handed to the
library as the allocation callback) and the stream (torch's current stream).
There is no CPU fallback: if the compiled library is missing this module
raises on import of the library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblsqr_mi355x.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "lsqr_mi355x.h")

LSQR_OK, LSQR_E_INVALID_ARG, LSQR_E_BAD_CSR, LSQR_E_NONFINITE = 0, -1, -2, -3
LSQR_E_DEVICE, LSQR_E_OOM, LSQR_E_UNSUPPORTED = -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}
PRECOND = {"none": 0, "jacobi": 1, "user": 2}
FLAG_TIMING, FLAG_NO_GRAPH = 1, 2

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class LsqrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class CSR(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("mem", ctypes.c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("precond", ctypes.c_int),
                ("col_scale", ctypes.c_void_p), ("refine_sweeps", ctypes.c_int),
                ("check_every", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("alloc", _ALLOC_FN), ("dealloc", _FREE_FN), ("alloc_user", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("lanes_per_row", ctypes.c_int),
                ("lanes_per_col", ctypes.c_int), ("row_format", ctypes.c_int),
                ("col_format", ctypes.c_int), ("refine_inner_tol", ctypes.c_double),
                ("method", ctypes.c_int), ("fallback_iters", ctypes.c_int),
                ("refine_stall_ratio", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("istop", ctypes.c_int), ("iters", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("fallback_used", ctypes.c_int), ("eta", ctypes.c_double),
                ("phibar", ctypes.c_double), ("eta_final_fp64", ctypes.c_double),
                ("inner_fp32", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchCfg(ctypes.Structure):
    _fields_ = [("rhs_tile", ctypes.c_int), ("grid", ctypes.c_int), ("ms_per_iter", ctypes.c_double)]


class KStats(ctypes.Structure):
    _fields_ = [("fwd_ms", ctypes.c_double), ("adj_ms", ctypes.c_double),
                ("fwd_launches", ctypes.c_int), ("adj_launches", ctypes.c_int),
                ("fwd_bytes", ctypes.c_double), ("adj_bytes", ctypes.c_double),
                ("row_format", ctypes.c_int), ("col_format", ctypes.c_int),
                ("fwd_entries_per_load", ctypes.c_int), ("adj_depths_per_word", ctypes.c_int),
                ("groups", ctypes.c_int64), ("staged_cols", ctypes.c_int64),
                ("padded_values", ctypes.c_int64)]


class Rays(ctypes.Structure):
    _fields_ = [("npairs", ctypes.c_int64), ("nper", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("node_ptr", ctypes.c_void_p), ("node_k", ctypes.c_void_p),
                ("node_len", ctypes.c_void_p), ("cvel", ctypes.c_void_p),
                ("j0", ctypes.c_void_p), ("nj", ctypes.c_void_p), ("w_ptr", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("keep", ctypes.c_void_p), ("node_mem", ctypes.c_int)]


class Polylines(ctypes.Structure):
    _fields_ = [("npaths", ctypes.c_int64), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("h", ctypes.c_double), ("km_per_deg", ctypes.c_double),
                ("pt_ptr", ctypes.c_void_p), ("px", ctypes.c_void_p), ("py", ctypes.c_void_p),
                ("plen", ctypes.c_void_p)]


_lib = None


def load():
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2604_11920_amd.build.build()")
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "lsqr_create": (I, [ctypes.POINTER(CSR), D, D, ctypes.POINTER(Opts), ctypes.POINTER(P)]),
        "lsqr_solve": (I, [P, P, I, I, D, P, P, ctypes.POINTER(Info)]),
        "lsqr_solve_x0": (I, [P, P, P, I, I, D, P, P, ctypes.POINTER(Info)]),
        "lsqr_apply": (I, [P, P, P]),
        "lsqr_apply_t": (I, [P, P, P]),
        "lsqr_apply_stored": (I, [P, P, P]),
        "lsqr_apply_t_stored": (I, [P, P, P, P]),
        "lsqr_get_scale": (I, [P, P]),
        "lsqr_set_scale": (I, [P, P]),
        "lsqr_get_transpose": (I, [P, P, P, P]),
        "lsqr_kernel_stats": (I, [P, ctypes.POINTER(KStats)]),
        "lsqr_get_quantised": (I, [P, P, P, P]),
        "lsqr_solve_batched": (I, [ctypes.POINTER(P), I, I, ctypes.POINTER(P), I, I, D,
                                   ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(Info)]),
        "lsqr_solve_batched_refined": (I, [ctypes.POINTER(P), I, I, ctypes.POINTER(P), I, I, D, D, I,
                                           ctypes.POINTER(P), ctypes.POINTER(Info)]),
        "lsqr_apply_block": (I, [P, I, P, P]),
        "lsqr_apply_t_block": (I, [P, I, P, P]),
        "lsqr_set_batch_config": (I, [P, ctypes.POINTER(BatchCfg)]),
        "lsqr_autotune_batched": (I, [P, I, I, ctypes.POINTER(BatchCfg)]),
        "lsqr_column_features": (I, [P, P]),
        "lsqr_mlp_scale": (I, [P, P, P, P, ctypes.c_uint, P, P]),
        "lsqr_mlp_scale_noalloc": (I, [P, P, P, P, ctypes.c_uint, P, P]),
        "lsqr_trainer_create": (I, [I, P, P, _ALLOC_FN, _FREE_FN, P, ctypes.POINTER(P)]),
        "lsqr_trainer_grad": (I, [P, I, P, P, P, ctypes.POINTER(D)]),
        "lsqr_trainer_step": (I, [P, I, P, P, ctypes.c_float, ctypes.POINTER(D)]),
        "lsqr_trainer_params": (I, [P, P, P]),
        "lsqr_trainer_destroy": (None, [P]),
        "lsqr_rays_size": (I, [ctypes.POINTER(Rays), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_int64)]),
        "lsqr_assemble_rays": (I, [ctypes.POINTER(Rays), P, _ALLOC_FN, _FREE_FN, P, P, P, P]),
        "lsqr_split_polylines": (I, [ctypes.POINTER(Polylines), P, _ALLOC_FN, _FREE_FN, P, P, P,
                                     P]),
        "lsqr_destroy": (None, [P]),
        "lsqr_status_string": (ctypes.c_char_p, [I]),
        "lsqr_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_functions():
    """Names of the functions declared in include/lsqr_mi355x.h."""
    import re
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lsqr_[a-z_]+)\s*\(", txt)))


def torch_allocator(device, stream):
    """(alloc, dealloc) ctypes callbacks drawing device memory from PyTorch's
    caching allocator on `stream`; keep both referenced while in use."""
    import torch
    blocks = {}

    def _alloc(nbytes, user):
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except Exception:
            return None
        blocks[p] = nbytes
        return p

    def _free(p, nbytes, user):
        if p in blocks:
            del blocks[p]
            torch.cuda.caching_allocator_delete(p)

    return _ALLOC_FN(_alloc), _FREE_FN(_free)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())      # torch tensor


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class Solver:
    """One regularised LSQR system on the GPU (wraps an lsqr_ctx).

    row_format: "auto" | "csr" | "groups" (forward product);
    col_format: "auto" | "csc" | "runs" | "pairs" (transposed product).  The formats are those of opts.row_format / opts.col_format in
    include/lsqr_mi355x.h; "auto" picks row groups and depth pairs where the
    matrix fits them."""

    def __init__(self, row_ptr, col, val, nx, ny, nz, damp, smooth, precision="fp64",
                 precond="none", col_scale=None, stream=None, timing=False, graph=True,
                 lanes_per_row=0, lanes_per_col=0, check_every=0, refine_sweeps=5,
                 row_format="auto", col_format="auto", refine_inner_tol=0.0,
                 method="lsqr", torch_alloc=True, fallback_iters=0, refine_stall_ratio=0.0):
        import torch
        lib = load()
        self._torch = torch
        self._keep = []
        dev = all(_is_torch(a) for a in (row_ptr, col, val))
        if not dev:
            row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            val = np.ascontiguousarray(val, dtype=np.float64)
        self._keep += [row_ptr, col, val]
        m = len(row_ptr) - 1
        self.m, self.n = int(m), int(nx) * int(ny) * int(nz)
        self.nnz = int(row_ptr[-1]) if not dev else int(row_ptr[-1].item())
        csr = CSR(self.m, self.n, self.nnz, int(nx), int(ny), int(nz), _ptr(row_ptr), _ptr(col),
                  _ptr(val), MEM_DEVICE if dev else MEM_HOST)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._device = torch.cuda.current_device()
        opts = Opts()
        opts.precision = PRECISION[precision]
        opts.precond = PRECOND[precond]
        if col_scale is not None:
            cs = np.ascontiguousarray(col_scale, dtype=np.float64)
            self._keep.append(cs)
            opts.col_scale = cs.ctypes.data
        opts.refine_sweeps = int(refine_sweeps)
        opts.refine_inner_tol = float(refine_inner_tol)
        opts.method = {"lsqr": 0, "lsmr": 1}[method]
        opts.fallback_iters = int(fallback_iters)
        opts.refine_stall_ratio = float(refine_stall_ratio)
        opts.check_every = int(check_every)
        opts.stream = stream.cuda_stream
        opts.flags = (FLAG_TIMING if timing else 0) | (0 if graph else FLAG_NO_GRAPH)
        opts.lanes_per_row = int(lanes_per_row)
        opts.lanes_per_col = int(lanes_per_col)
        opts.row_format = {"auto": 0, "csr": 1, "groups": 4}[row_format]
        opts.col_format = {"auto": 0, "csc": 1, "runs": 2, "pairs": 4}[col_format]
        self.precision = precision
        if torch_alloc:
            self._alloc_cb, self._free_cb = torch_allocator(self._device, stream)
            opts.alloc, opts.dealloc = self._alloc_cb, self._free_cb
        ctx = ctypes.c_void_p()
        rc = lib.lsqr_create(ctypes.byref(csr), float(damp), float(smooth), ctypes.byref(opts),
                             ctypes.byref(ctx))
        if rc != LSQR_OK:
            raise LsqrError(rc, lib.lsqr_last_error(None).decode())
        self._ctx = ctx
        self._lib = lib

    @classmethod
    def from_system(cls, s, **kw):
        kw.setdefault("damp", s.damp)
        kw.setdefault("smooth", s.smooth)
        return cls(s.row_ptr, s.col, s.val, s.nx, s.ny, s.nz, **kw)

    def _check(self, rc):
        if rc != LSQR_OK:
            raise LsqrError(rc, self._lib.lsqr_last_error(self._ctx).decode())

    def solve(self, dt, iters, tol=0.0, dm=None, history=True, x0=None):
        """Run the solver.  dt: numpy (host) or torch CUDA float64 tensor
        (device); x0: optional initial solution of the same kind (warm start,
        lsqr_solve_x0).  Returns (dm, hist [iters+1, 3] or None, info dict)."""
        torch = self._torch
        if _is_torch(dt):
            assert dt.is_cuda and dt.dtype == torch.float64 and dt.is_contiguous()
            mem = MEM_DEVICE
            if dm is None:
                dm = torch.empty(self.n, dtype=torch.float64, device=dt.device)
            if x0 is not None:
                assert _is_torch(x0) and x0.is_cuda and x0.dtype == torch.float64
                x0 = x0.contiguous()
        else:
            dt = np.ascontiguousarray(dt, dtype=np.float64)
            mem = MEM_HOST
            if dm is None:
                dm = np.empty(self.n)
            if x0 is not None:
                x0 = np.ascontiguousarray(x0, dtype=np.float64)
        hist = np.empty((iters + 1, 3)) if history else None
        info = Info()
        if x0 is None:
            self._check(self._lib.lsqr_solve(self._ctx, _ptr(dt), mem, int(iters), float(tol),
                                             _ptr(dm), _ptr(hist), ctypes.byref(info)))
        else:
            assert x0.shape == (self.n,)
            self._check(self._lib.lsqr_solve_x0(self._ctx, _ptr(dt), _ptr(x0), mem, int(iters),
                                                float(tol), _ptr(dm), _ptr(hist),
                                                ctypes.byref(info)))
        return dm, hist, info.as_dict()

    def apply(self, x, y=None):
        """y = Abar D x (device tensors, float64)."""
        if y is None:
            y = self._torch.empty(self.m + 2 * self.n, dtype=self._torch.float64, device=x.device)
        self._check(self._lib.lsqr_apply(self._ctx, _ptr(x), _ptr(y)))
        return y

    def apply_t(self, y, x=None):
        """x = D Abar^T y (device tensors, float64)."""
        if x is None:
            x = self._torch.empty(self.n, dtype=self._torch.float64, device=y.device)
        self._check(self._lib.lsqr_apply_t(self._ctx, _ptr(y), _ptr(x)))
        return x

    def apply_stored(self, z, y=None):
        """y = [Ghat z; w L z; lambda z] with the solver's stored values (no
        column scale); device tensors of the solver's vector type."""
        dt = self._torch.float64 if self.precision == "fp64" else self._torch.float32
        if y is None:
            y = self._torch.empty(self.m + 2 * self.n, dtype=dt, device=z.device)
        self._check(self._lib.lsqr_apply_stored(self._ctx, _ptr(z), _ptr(y)))
        return y

    def apply_t_stored(self, y, tg=None, q=None):
        """q = Ghat^T (tg or y_G) + w L y_L + lambda y_D with the solver's
        stored values (no column scale); for the 16-bit forms tg = sigma * y_G."""
        dt = self._torch.float64 if self.precision == "fp64" else self._torch.float32
        if q is None:
            q = self._torch.empty(self.n, dtype=dt, device=y.device)
        self._check(self._lib.lsqr_apply_t_stored(self._ctx, _ptr(y), _ptr(tg), _ptr(q)))
        return q

    def set_scale(self, d):
        """Replace the column scaling D (host array [n], finite, > 0)."""
        d = np.ascontiguousarray(d, dtype=np.float64)
        assert d.shape == (self.n,)
        self._check(self._lib.lsqr_set_scale(self._ctx, d.ctypes.data))

    def scale(self):
        d = np.empty(self.n)
        self._check(self._lib.lsqr_get_scale(self._ctx, _ptr(d)))
        return d

    def transpose(self):
        cp = np.empty(self.n + 1, dtype=np.int64)
        ri = np.empty(self.nnz, dtype=np.int32)
        cv = np.empty(self.nnz, dtype=np.float64)
        self._check(self._lib.lsqr_get_transpose(self._ctx, _ptr(cp), _ptr(ri), _ptr(cv)))
        return cp, ri, cv

    def quantised(self):
        """(row scales [m] float32, codes in CSR order, codes in CSC order), uint16."""
        sc = np.empty(self.m, dtype=np.float32)
        qr = np.empty(self.nnz, dtype=np.uint16)
        qc = np.empty(self.nnz, dtype=np.uint16)
        self._check(self._lib.lsqr_get_quantised(self._ctx, _ptr(sc), _ptr(qr), _ptr(qc)))
        return sc, qr, qc

    def apply_block(self, x, y=None):
        """Y = Abar D X for a row-major [n][R] float32 device block (R a power of 2 <= 32)."""
        R = x.shape[1]
        if y is None:
            y = self._torch.empty((self.m + 2 * self.n, R), dtype=self._torch.float32,
                                  device=x.device)
        self._check(self._lib.lsqr_apply_block(self._ctx, R, _ptr(x), _ptr(y)))
        return y

    def apply_t_block(self, y, x=None):
        """X = D Abar^T Y for a row-major [m+2n][R] float32 device block."""
        R = y.shape[1]
        if x is None:
            x = self._torch.empty((self.n, R), dtype=self._torch.float32, device=y.device)
        self._check(self._lib.lsqr_apply_t_block(self._ctx, R, _ptr(y), _ptr(x)))
        return x

    def set_batch_config(self, rhs_tile, grid):
        cfg = BatchCfg(int(rhs_tile), int(grid), 0.0)
        self._check(self._lib.lsqr_set_batch_config(self._ctx, ctypes.byref(cfg)))

    def autotune_batched(self, nrhs, probe_iters=4, cache=None):
        """Choose the batched schedule for nrhs right-hand sides: from the JSON
        cache file `cache` when it holds this shape, else by timing every
        schedule on the device (median of 5) and storing the winner."""
        import json
        key = self.shape_key(nrhs)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            t = table[key]
            self.set_batch_config(t["rhs_tile"], t["grid"])
            return dict(t, cached=True)
        cfg = BatchCfg()
        self._check(self._lib.lsqr_autotune_batched(self._ctx, int(nrhs), int(probe_iters),
                                                    ctypes.byref(cfg)))
        t = {"rhs_tile": cfg.rhs_tile, "grid": cfg.grid, "ms_per_iter": cfg.ms_per_iter}
        if cache:
            table[key] = t
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(t, cached=False)

    def shape_key(self, nrhs):
        """Shape signature of a batched schedule: system size, padded RHS count, device."""
        R = 1
        while R < nrhs:
            R *= 2
        name = self._torch.cuda.get_device_name(self._device).replace(" ", "_")
        return f"m{self.m}_n{self.n}_nnz{self.nnz}_R{R}_{name}"

    def column_features(self):
        """[n, 6] float32 device tensor of the learned scale's column features."""
        f = self._torch.empty((self.n, 6), dtype=self._torch.float32, device="cuda")
        self._check(self._lib.lsqr_column_features(self._ctx, _ptr(f)))
        return f

    def mlp_scale(self, params, mean, std, feat=None, centre=0, d=None):
        """Learned column scale (device float64 [n]): Jacobi times softplus of the
        BF16 MLP on standardised features.  params: float32 device tensor;
        centre: bit mask of features centred on this system's own means."""
        if feat is None:
            feat = self.column_features()
        mean = np.ascontiguousarray(mean, dtype=np.float32)
        std = np.ascontiguousarray(std, dtype=np.float32)
        if d is None:
            d = self._torch.empty(self.n, dtype=self._torch.float64, device="cuda")
        self._check(self._lib.lsqr_mlp_scale(self._ctx, _ptr(params), _ptr(mean), _ptr(std),
                                             int(centre), _ptr(feat), _ptr(d)))
        return d

    def mlp_scale_noalloc(self, params, mean, std, feat, d, centre=0):
        """lsqr_mlp_scale_noalloc: as mlp_scale, into the caller's d, with the
        temporaries in the library's static device scratch (no allocation)."""
        mean = np.ascontiguousarray(mean, dtype=np.float32)
        std = np.ascontiguousarray(std, dtype=np.float32)
        self._check(self._lib.lsqr_mlp_scale_noalloc(self._ctx, _ptr(params), _ptr(mean),
                                                     _ptr(std), int(centre), _ptr(feat), _ptr(d)))
        return d

    def kernel_stats(self):
        ks = KStats()
        self._check(self._lib.lsqr_kernel_stats(self._ctx, ctypes.byref(ks)))
        return {f: getattr(ks, f) for f, _ in ks._fields_}

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lsqr_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def solve_batched(solvers, dts, iters, tol=0.0, history=True):
    """LSQR for several systems with nrhs right-hand sides each, in one batched
    call.  dts: list of [m_s, nrhs] arrays (numpy: host, torch CUDA float64:
    device), all on the same side.  Returns (dms, hists, infos): dms [n_s, nrhs],
    hists [iters+1, nrhs, 3] per system (or None), infos[s][r] dicts."""
    lib = load()
    nsys = len(solvers)
    nrhs = int(dts[0].shape[1])
    dev = _is_torch(dts[0])
    if dev:
        import torch
        dts = [d.contiguous() for d in dts]
        dms = [torch.empty((s.n, nrhs), dtype=torch.float64, device=dts[0].device) for s in solvers]
    else:
        dts = [np.ascontiguousarray(d, dtype=np.float64) for d in dts]
        dms = [np.empty((s.n, nrhs)) for s in solvers]
    for s, d in zip(solvers, dts):
        assert tuple(d.shape) == (s.m, nrhs)
    hists = [np.empty((iters + 1, nrhs, 3)) for _ in solvers] if history else None
    P = ctypes.c_void_p
    ctxs = (P * nsys)(*[s._ctx.value for s in solvers])
    dtp = (P * nsys)(*[_ptr(d).value for d in dts])
    dmp = (P * nsys)(*[_ptr(d).value for d in dms])
    hp = (P * nsys)(*[h.ctypes.data for h in hists]) if history else None
    infos = (Info * (nsys * nrhs))()
    rc = lib.lsqr_solve_batched(ctxs, nsys, nrhs, dtp, MEM_DEVICE if dev else MEM_HOST, int(iters),
                                float(tol), dmp, hp, infos)
    if rc != LSQR_OK:
        raise LsqrError(rc, lib.lsqr_last_error(solvers[0]._ctx).decode())
    out = [[infos[s * nrhs + r].as_dict() for r in range(nrhs)] for s in range(nsys)]
    return dms, hists, out


def solve_batched_refined(solvers, dts, iters, tol, inner_tol=1e-4, sweeps=8):
    """lsqr_solve_batched_refined: the batched solve with FP64 iterative
    refinement per right-hand side (tol > 0).  dts as in solve_batched.
    Returns (dms, infos)."""
    lib = load()
    nsys = len(solvers)
    nrhs = int(dts[0].shape[1])
    dev = _is_torch(dts[0])
    if dev:
        import torch
        dts = [d.contiguous() for d in dts]
        dms = [torch.empty((s.n, nrhs), dtype=torch.float64, device=dts[0].device) for s in solvers]
    else:
        dts = [np.ascontiguousarray(d, dtype=np.float64) for d in dts]
        dms = [np.empty((s.n, nrhs)) for s in solvers]
    for s, d in zip(solvers, dts):
        assert tuple(d.shape) == (s.m, nrhs)
    P = ctypes.c_void_p
    ctxs = (P * nsys)(*[s._ctx.value for s in solvers])
    dtp = (P * nsys)(*[_ptr(d).value for d in dts])
    dmp = (P * nsys)(*[_ptr(d).value for d in dms])
    infos = (Info * (nsys * nrhs))()
    rc = lib.lsqr_solve_batched_refined(ctxs, nsys, nrhs, dtp, MEM_DEVICE if dev else MEM_HOST,
                                        int(iters), float(tol), float(inner_tol), int(sweeps), dmp,
                                        infos)
    if rc != LSQR_OK:
        raise LsqrError(rc, lib.lsqr_last_error(solvers[0]._ctx).decode())
    out = [[infos[s * nrhs + r].as_dict() for r in range(nrhs)] for s in range(nsys)]
    return dms, out


class Trainer:
    """FP32 training state of the column-scale MLP on the GPU."""

    NPARAMS = 4673

    def __init__(self, params, max_batch, stream=None):
        import torch
        self._lib = load()
        self._torch = torch
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.NPARAMS
        stream = stream or torch.cuda.current_stream()
        self._alloc_cb, self._free_cb = torch_allocator(torch.cuda.current_device(), stream)
        h = ctypes.c_void_p()
        rc = self._lib.lsqr_trainer_create(int(max_batch), _ptr(p), stream.cuda_stream,
                                           self._alloc_cb, self._free_cb, None, ctypes.byref(h))
        if rc != LSQR_OK:
            raise LsqrError(rc, "trainer creation failed")
        self._h = h
        self.max_batch = int(max_batch)

    def grad(self, x, target):
        g = self._torch.empty(self.NPARAMS, dtype=self._torch.float32, device="cuda")
        loss = ctypes.c_double()
        rc = self._lib.lsqr_trainer_grad(self._h, int(x.shape[0]), _ptr(x), _ptr(target), _ptr(g),
                                         ctypes.byref(loss))
        if rc != LSQR_OK:
            raise LsqrError(rc, "trainer gradient failed")
        return g, loss.value

    def step(self, x, target, lr=1e-3, want_loss=False):
        loss = ctypes.c_double()
        rc = self._lib.lsqr_trainer_step(self._h, int(x.shape[0]), _ptr(x), _ptr(target),
                                         float(lr), ctypes.byref(loss) if want_loss else None)
        if rc != LSQR_OK:
            raise LsqrError(rc, "trainer step failed")
        return loss.value if want_loss else None

    def params(self):
        p = np.empty(self.NPARAMS, dtype=np.float32)
        rc = self._lib.lsqr_trainer_params(self._h, _ptr(p), None)
        if rc != LSQR_OK:
            raise LsqrError(rc, "trainer read-back failed")
        return p

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lsqr_trainer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _rays_struct(rays, node_k=None, node_len=None, node_ptr=None):
    """ctypes view of a ray description (dict of numpy arrays, see synth's
    System.rays); returns (struct, arrays kept alive).  node_k / node_len /
    node_ptr, when given, replace the dict's (node_k and node_len as device
    tensors)."""
    dev = node_k is not None
    keep = [np.ascontiguousarray(rays["node_ptr"] if node_ptr is None else node_ptr, dtype=np.int64),
            node_k if dev else np.ascontiguousarray(rays["node_k"], dtype=np.int32),
            node_len if dev else np.ascontiguousarray(rays["node_len"], dtype=np.float64),
            np.ascontiguousarray(rays["cvel"], dtype=np.float64),
            np.ascontiguousarray(rays["j0"], dtype=np.int32),
            np.ascontiguousarray(rays["nj"], dtype=np.int32),
            np.ascontiguousarray(rays["w_ptr"], dtype=np.int64),
            np.ascontiguousarray(rays["w"], dtype=np.float64),
            np.ascontiguousarray(rays["keep"], dtype=np.uint8).reshape(-1)]
    st = Rays(len(keep[0]) - 1, len(keep[3]), int(rays["nz"]), *[_ptr(a) for a in keep],
              MEM_DEVICE if dev else MEM_HOST)
    return st, keep


def rays_size(rays):
    """(m, nnz) of the G assembled from `rays` (host work only)."""
    lib = load()
    st, _keep = _rays_struct(rays)
    m, nnz = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.lsqr_rays_size(ctypes.byref(st), ctypes.byref(m), ctypes.byref(nnz))
    if rc != LSQR_OK:
        raise LsqrError(rc, lib.lsqr_last_error(None).decode())
    return int(m.value), int(nnz.value)


def split_polylines(poly, stream=None):
    """lsqr_split_polylines on the ray polylines `poly` (dict: pt_ptr, px, py,
    plen, h, nx, ny, km_per_deg; see synth's System.rays["polyline"]):
    (node_ptr numpy int64, node_k torch int32, node_len torch float64), the
    node arrays on the device."""
    import torch
    lib = load()
    keep = [np.ascontiguousarray(poly[k], dtype=np.int64 if k == "pt_ptr" else np.float64)
            for k in ("pt_ptr", "px", "py", "plen")]
    st = Polylines(len(keep[0]) - 1, int(poly["nx"]), int(poly["ny"]), float(poly["h"]),
                   float(poly["km_per_deg"]), *[a.ctypes.data for a in keep])
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = stream or torch.cuda.current_stream()
    alloc_cb, free_cb = torch_allocator(dev.index, stream)
    node_ptr = np.empty(len(keep[0]), dtype=np.int64)
    rc = lib.lsqr_split_polylines(ctypes.byref(st), stream.cuda_stream, alloc_cb, free_cb, None,
                                  _ptr(node_ptr), None, None)
    if rc != LSQR_OK:
        raise LsqrError(rc, lib.lsqr_last_error(None).decode())
    nn = int(node_ptr[-1])
    node_k = torch.empty(max(nn, 1), dtype=torch.int32, device=dev)[:nn]
    node_len = torch.empty(max(nn, 1), dtype=torch.float64, device=dev)[:nn]
    rc = lib.lsqr_split_polylines(ctypes.byref(st), stream.cuda_stream, alloc_cb, free_cb, None,
                                  _ptr(node_ptr), _ptr(node_k) if nn else None,
                                  _ptr(node_len) if nn else None)
    if rc != LSQR_OK:
        raise LsqrError(rc, lib.lsqr_last_error(None).decode())
    return node_ptr, node_k, node_len


def assemble_polylines(rays, stream=None):
    """G assembled on the device from the ray polylines: the bilinear split
    (split_polylines) and the row assembly (lsqr_assemble_rays with the
    node arrays left on the device).  `rays` as synth's System.rays (its
    "polyline" entry and the per-period arrays).  Returns (row_ptr, col, val)
    torch CUDA tensors."""
    node_ptr, node_k, node_len = split_polylines(rays["polyline"], stream)
    return assemble_rays(rays, stream, node_ptr=node_ptr, node_k=node_k, node_len=node_len)


def assemble_rays(rays, stream=None, node_ptr=None, node_k=None, node_len=None):
    """G assembled on the device from `rays`: (row_ptr, col, val) as torch
    CUDA tensors (int64, int32, float64), ready for Solver(..., device G).
    node_ptr / node_k / node_len (device tensors for the last two) replace
    the dict's node arrays when given."""
    import torch
    lib = load()
    st, _keep = _rays_struct(rays, node_k, node_len, node_ptr)
    m, nnz = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.lsqr_rays_size(ctypes.byref(st), ctypes.byref(m), ctypes.byref(nnz))
    if rc != LSQR_OK:
        raise LsqrError(rc, lib.lsqr_last_error(None).decode())
    m, nnz = int(m.value), int(nnz.value)
    dev = torch.device("cuda", torch.cuda.current_device())
    rp = torch.empty(m + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)[:nnz]
    val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)[:nnz]
    stream = stream or torch.cuda.current_stream()
    alloc_cb, free_cb = torch_allocator(dev.index, stream)
    rc = lib.lsqr_assemble_rays(ctypes.byref(st), stream.cuda_stream, alloc_cb, free_cb, None,
                                _ptr(rp), _ptr(col), _ptr(val))
    if rc != LSQR_OK:
        raise LsqrError(rc, lib.lsqr_last_error(None).decode())
    return rp, col, val
