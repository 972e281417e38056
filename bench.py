"""Benchmark: damped, smoothing-regularised LSQR on one MI355X.

A step is one LSQR solve of the paper-shaped synthetic system (80x80x20 grid,
229 stations, all pairs x 20 periods, paths >= 2 wavelengths, bent rays;
~0.49M rows, ~0.59B stored entries) for a fixed 300 iterations with the
system and right-hand side already resident in HBM.  value = LSQR
iterations per second.  The two sparse kernels are timed with HIP events on
the solve's stream inside the timed region; the dominant one is reported
against the HBM roofline.  The FP64 CPU oracle is timed on a bounded sample
of the same solve on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cfg1|cfg0]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LSQR iters/s + SpMV HBM GB/s; time-to-tol mixed/learned vs plain FP64"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_threads():
    """Threads for the CPU legs: the host CPUs this process may use, at most 16
    (the host-core share of one GPU on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def trimmed_mean(xs):
    """The paper's timing protocol: drop the largest and the smallest run,
    average the rest."""
    xs = sorted(xs)
    core = xs[1:-1] if len(xs) > 2 else xs
    return sum(core) / len(core)


def cpu_baseline(s, iters_sample, runs=10):
    """The FP64 oracle on the same system: `runs` timed runs of a bounded
    number of LSQR iterations on the host cores after one untimed warm-up,
    the slowest and fastest dropped (transpose set-up excluded)."""
    import oracle
    nt = host_threads()
    op = oracle.Operator.from_system(s, nthreads=nt)
    op.lsqr(s.dt, max(1, iters_sample // 4))            # warm-up (untimed)
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        r = op.lsqr(s.dt, iters_sample)
        times.append(time.perf_counter() - t0)
    t = trimmed_mean(times)
    return {"value": r["iters"] / t, "unit": "iters/s", "cores": nt, "kind": "oracle",
            "sample": f"{r['iters']} FP64 LSQR iterations (plus the start step) of the same "
                      f"system, {runs} runs after a warm-up, slowest and fastest dropped, "
                      f"{t:.2f} s per run",
            "runs_s": times, "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def scipy_lsqr_context(s, iters=3):
    """SciPy's LSQR (single-threaded sparse products) on the same regularised
    operator for a few iterations: the analogue of the paper's CPU solver
    path, for context only."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import LinearOperator, lsqr
    G = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.m, s.n), copy=False)
    Gt = G.T                                   # CSC view, no copy
    nx, ny, nz = s.nx, s.ny, s.nz

    def lap(x):
        u = x.reshape(ny, nx, nz)
        y = np.zeros_like(u)
        for ax in range(3):
            k = u.shape[ax]
            if k < 2:
                continue
            d = np.diff(u, axis=ax)
            sl_lo = [slice(None)] * 3
            sl_hi = [slice(None)] * 3
            sl_lo[ax] = slice(0, k - 1)
            sl_hi[ax] = slice(1, k)
            y[tuple(sl_lo)] += d
            y[tuple(sl_hi)] -= d
        return y.reshape(-1)

    m, n = s.m, s.n

    def mv(x):
        return np.concatenate([G @ x, s.smooth * lap(x), s.damp * x])

    def rmv(y):
        return Gt @ y[:m] + s.smooth * lap(y[m:m + n]) + s.damp * y[m + n:]

    A = LinearOperator((m + 2 * n, n), matvec=mv, rmatvec=rmv, dtype=np.float64)
    b = np.concatenate([s.dt, np.zeros(2 * n)])
    t0 = time.perf_counter()
    lsqr(A, b, damp=0.0, atol=0.0, btol=0.0, conlim=0.0, iter_lim=iters)
    t = time.perf_counter() - t0
    return {"value": iters / t, "unit": "iters/s", "iters": iters, "seconds": t,
            "threads": 1, "kind": "scipy.sparse.linalg.lsqr on the same operator (context)"}


KERNEL_SRCS = [os.path.join(ROOT, "paper_2604_11920_amd", "csrc", f)
               for f in ("lsqr_kernels.cuh", "internal.h", "kernels_f64.hip", "kernels_common.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_cfg1_fp64.txt")
CALIB_BYTES = float(1 << 30)        # the calibration kernel reads 1 GiB and writes 1 GiB


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def pmc_summary(fetch_csv, write_csv, formats=None):
    """Per-launch HBM bytes of the solver kernels from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by what the same
    counter reads for the 1 GiB elementwise calibration kernel."""
    import csv
    out = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        calib = [float(r["Counter_Value"]) for r in rows
                 if "elementwise" in r["Kernel_Name"] and "MulFunctor" in r["Kernel_Name"]]
        factor = CALIB_BYTES / 1024.0 / (sum(calib) / len(calib))
        out[counter + "_factor"] = factor
        for tag, key in (("fwd", "k_fwd"), ("adj", "k_adj")):
            v = [float(r["Counter_Value"]) for r in rows if key in r["Kernel_Name"]]
            out[f"{tag}_{counter}_bytes"] = sum(v) / len(v) * 1024.0 * factor
    for tag in ("fwd", "adj"):
        out[f"{tag}_traffic_bytes"] = out[f"{tag}_FETCH_SIZE_bytes"] + out[f"{tag}_WRITE_SIZE_bytes"]
    out["source_sha256_16"] = source_hash()
    if formats:
        out["formats"] = formats
    return out


def measured_traffic(tag, formats=None):
    """Traffic of kernel `tag` from the committed counter summary, or None when
    the kernel source changed since the counters were taken."""
    try:
        kv = dict(line.split(None, 1) for line in open(TRAFFIC_FILE).read().splitlines()
                  if line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("source_sha256_16", "").strip() != source_hash():
        return None
    if formats is not None and kv.get("formats", "").strip() != formats:
        return None
    v = kv.get(f"{tag}_traffic_bytes")
    return float(v) if v else None



def kernel_label(tag, ks):
    """Name of the kernel the solver's formats select (as lsqr_kernel_stats
    reports them)."""
    if tag == "fwd":
        rf = ks["row_format"]
        if rf == 4:
            e = ks["fwd_entries_per_load"]
            return (f"k_fwd_lcol_pair<{e}> (forward product, row groups, entries in aligned "
                    + {2: "pairs)", 4: "quads)", 8: "octets)"}[e] if e > 1 else
                    "k_fwd_lcol (forward product, row groups, columns staged in LDS)")
        return "k_fwd_pipe / k_fwd_csr (forward product, CSR rows)"
    cf = ks["col_format"]
    if cf == 4:
        w = ks["adj_depths_per_word"]
        return (f"k_adj_npair<{w}> (transposed product, node runs, "
                + {2: "depth pairs)", 4: "four-depth words)", 8: "eight-depth words)"}[w])
    return {1: "k_adj (transposed product, CSC)",
            2: "k_adj_nruns (transposed product, node runs)"}[cf]


def assembly_check(s, host_s):
    """Device-side assembly of G from the same rays: seconds (host row
    structure + device fill, median of 3) against the host generator, and a
    bitwise comparison with the generator's arrays."""
    import torch
    from paper_2604_11920_amd import assemble_rays
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rp, col, val = assemble_rays(s.rays)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if _ < 2:
            del rp, col, val
    same = (torch.equal(rp.cpu(), torch.from_numpy(s.row_ptr))
            and torch.equal(col, torch.from_numpy(s.col).cuda())
            and torch.equal(val.view(torch.int64), torch.from_numpy(s.val).cuda().view(torch.int64)))
    del rp, col, val
    torch.cuda.empty_cache()
    r = {"device_s": sorted(times)[1], "host_generator_s": host_s, "bitwise_equal": bool(same)}
    log(f"[bench] assembly on the device {r['device_s']:.3f} s (host generator {host_s:.2f} s), "
        f"bitwise equal: {same}")
    return r


def fp32_rate(s, dt, iters, fmt, gold=None, steps=3):
    """FP32 values, vectors and accumulation (FP64 scalars): iterations/s and
    kernel rates on the same system, same iteration count; with the stored
    oracle results, the error of the last iterate against the oracle's FP64
    iterate at the same count and against x*."""
    import torch
    from paper_2604_11920_amd import Solver
    with Solver.from_system(s, precision="fp32", timing=True, **fmt) as sol:
        dm = torch.empty(s.n, dtype=torch.float64, device="cuda")
        sol.solve(dt, iters, dm=dm, history=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fwd = adj = 0.0
        nf = na = 0
        for _ in range(steps):
            sol.solve(dt, iters, dm=dm, history=False)
            ks = sol.kernel_stats()
            fwd += ks["fwd_ms"]; adj += ks["adj_ms"]; nf += ks["fwd_launches"]; na += ks["adj_launches"]
        wall = time.perf_counter() - t0
    fa, aa = fwd / nf, adj / na
    r = {"iters_per_s": iters * steps / wall, "ms_per_step": wall * 1e3 / steps,
         "fwd": {"avg_us": fa * 1e3, "alg_bytes": ks["fwd_bytes"], "gbs": ks["fwd_bytes"] / fa / 1e6},
         "adj": {"avg_us": aa * 1e3, "alg_bytes": ks["adj_bytes"], "gbs": ks["adj_bytes"] / aa / 1e6}}
    if gold is not None and f"x{iters}_comp" in gold:
        x = dm.cpu().numpy()
        ref, xs = gold[f"x{iters}_comp"], gold["x_star"]
        r["err_vs_oracle_same_iters"] = float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
        r["err_vs_xstar"] = float(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    log(f"[bench] fp32: {r['iters_per_s']:.1f} it/s; fwd {r['fwd']['gbs']:.0f} GB/s, "
        f"adj {r['adj']['gbs']:.0f} GB/s")
    return r


GOLDEN = os.path.join(ROOT, "tests", "golden", "cfg1_seed0.npz")


def golden_reference(s):
    """The oracle's converged solution x* and fixed-count iterates for this
    system, when the stored reference results describe it (else None)."""
    import synth
    try:
        z = np.load(GOLDEN, allow_pickle=False)
        meta = json.loads(str(z["meta"]))
    except (OSError, KeyError, ValueError):
        return None
    if meta.get("fingerprint") != synth.fingerprint(s):
        return None
    return {k: z[k] for k in z.files if k != "meta"}


def time_to_tol(s, dt, tol, fmt, model_path=None, xstar=None):
    """Wall time to eta = |Abar^T r| / |Abar^T bbar| <= tol for each form, each
    result's eta re-checked explicitly with the FP64 operator on the GPU.  The
    system is resident (created before the clock starts); for the learned
    forms the feature + MLP inference time is reported beside the solve."""
    import torch
    from paper_2604_11920_amd import Solver
    # (precision, scaling, iteration cap, inner tolerance of the refinement)
    forms = [("fp64", "none", 20000, 0.0), ("fp64", "jacobi", 20000, 0.0),
             ("fp64", "jacobi_lsmr", 20000, 0.0),
             ("bf16", "jacobi", 4000, 0.0), ("bf16", "jacobi", 4000, 1e-3),
             ("bf16", "jacobi_lsmr", 4000, 0.0),
             ("fp16", "jacobi", 4000, 0.0)]
    model = None
    if model_path and os.path.exists(model_path):
        from paper_2604_11920_amd import learned
        model = learned.ColumnScaleModel.load(model_path)
        forms += [("fp64", "learned", 20000, 0.0), ("bf16", "learned", 4000, 0.0)]
    out = {}
    ref = None
    checker = Solver.from_system(s, **fmt)
    b = torch.zeros(s.m + 2 * s.n, dtype=torch.float64, device="cuda")
    b[:s.m] = dt
    atb = checker.apply_t(b).norm().item()
    d_learned = None
    infer_s = None
    if model is not None:
        p = torch.from_numpy(np.ascontiguousarray(model.params, dtype=np.float32)).cuda()
        checker.mlp_scale(p, model.mean, model.std, centre=model.centre)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d_learned = checker.mlp_scale(p, model.mean, model.std, centre=model.centre)
        torch.cuda.synchronize()
        infer_s = time.perf_counter() - t0
        d_learned = d_learned.cpu().numpy()
    for prec, pc, cap, itol in forms:
        if pc == "learned":
            kw = dict(precond="user", col_scale=d_learned)
        elif pc == "jacobi_lsmr":     # LSMR (its eta is in the scaled variables)
            kw = dict(precond="jacobi", method="lsmr")
        else:
            kw = dict(precond=pc)
        with Solver.from_system(s, precision=prec, refine_sweeps=8, refine_inner_tol=itol,
                                **kw, **fmt) as sol:
            dm = torch.empty(s.n, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = sol.solve(dt, cap, tol=tol, dm=dm, history=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        r = b - checker.apply(dm)
        eta = checker.apply_t(r).norm().item() / atb
        key = f"{prec}_{pc}" + (f"_inner{itol:g}" if itol else "")
        out[key] = {"seconds": wall, "iters": info["iters"], "sweeps": info["sweeps"],
                    "istop": info["istop"], "eta_fp64": eta}
        if pc == "learned":
            out[key]["inference_seconds"] = infer_s
            out[key]["fallback_used"] = info["fallback_used"]
        if prec == "fp64" and pc == "jacobi":
            ref = dm.clone()
        if ref is not None and not (prec == "fp64" and pc == "jacobi"):
            out[key]["rel_diff_vs_fp64_jacobi"] = ((dm - ref).norm() / ref.norm()).item()
        if xstar is not None:
            out[key]["err_vs_xstar"] = ((dm - xstar).norm() / xstar.norm()).item()
        out[key]["eta_final_fp64_lib"] = info["eta_final_fp64"]
        log(f"[bench] time-to-tol {key}: {wall:.2f}s, iters={info['iters']} "
            f"sweeps={info['sweeps']} istop={info['istop']} eta_fp64={eta:.2e}")
    checker.close()
    base = out["fp64_none"]["seconds"]
    for k in out:
        out[k]["speedup_vs_fp64_none"] = base / out[k]["seconds"]
    return out


def batched_measure(iters=300, steps=1, warmup=1, row_format="auto", col_format="auto",
                    refine=False):
    """The batched workload: the four uneven systems of the batched case
    (config-1 geometry, (stations, periods) = (60,10), (120,14), (180,17),
    (229,20), seeds 0..3), 32 right-hand sides each (16 checkerboards, 16
    noise draws), schedules from the autotuner, `iters` iterations per step.
    Returns the right-hand-side iteration rate, the matrix bytes per batched
    iteration (FP32 CSR + CSC values and indices) and their rate against the
    HBM peak, and per system the block products' times."""
    import torch

    import synth
    from paper_2604_11920_amd import Solver, solve_batched, solve_batched_refined
    sols, dts, nnz, rows = [], [], 0, 0
    try:
        for cfg in synth.config3_systems():
            t0 = time.perf_counter()
            s = synth.make_system(cfg)
            rhs = synth.checker_rhs_batch(s)
            sols.append(Solver.from_system(s, row_format=row_format, col_format=col_format,
                                           precond="jacobi" if refine else "none"))
            dts.append(torch.from_numpy(rhs).cuda())
            nnz += s.nnz
            rows += s.m
            log(f"[batched] {cfg.name}: m={s.m} nnz={s.nnz} ({time.perf_counter() - t0:.1f}s)")
            del s, rhs
        R = int(dts[0].shape[1])
        tuned = [sol.autotune_batched(R, probe_iters=8) for sol in sols]
        log(f"[batched] tuned {tuned}")
        for _ in range(warmup):
            solve_batched(sols, dts, iters, history=False)
        torch.cuda.synchronize()
        per = []
        for _ in range(steps):
            t0 = time.perf_counter()
            solve_batched(sols, dts, iters, history=False)
            per.append(time.perf_counter() - t0)
        wall = sum(per)
        sec_per_it = wall / (iters * steps)
        products = []
        for sol in sols:
            x = torch.randn(sol.n, R, device="cuda", dtype=torch.float32)
            yb = torch.randn(sol.m + 2 * sol.n, R, device="cuda", dtype=torch.float32)
            y = sol.apply_block(x)
            xt = sol.apply_t_block(yb)
            row = {}
            for name, f in (("fwd_ms", lambda: sol.apply_block(x, y)),
                            ("adj_ms", lambda: sol.apply_t_block(yb, xt))):
                f()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(10):
                    f()
                e1.record()
                torch.cuda.synchronize()
                row[name] = e0.elapsed_time(e1) / 10
            products.append(row)
        mat_bytes = 2 * nnz * 8.0
        out = {"value": len(sols) * R * iters * steps / wall, "unit": "rhs-iters/s",
               "systems": len(sols), "rhs_per_system": R, "iters": iters, "steps": steps,
               "ms_per_step": 1e3 * wall / steps, "batched_iters_per_s": 1.0 / sec_per_it,
               "matrix_bytes_per_batched_iter": mat_bytes,
               "matrix_gbs": mat_bytes / sec_per_it / 1e9,
               "matrix_frac_of_hbm_peak": mat_bytes / sec_per_it / 1e9 / HBM_PEAK_GBS,
               "nnz_total": nnz, "rows_total": rows, "tuned": tuned, "block_products": products}
        if refine:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos = solve_batched_refined(sols, dts, 3000, 1e-6, inner_tol=1e-4, sweeps=8)
            torch.cuda.synchronize()
            flat = [i for sys_i in infos for i in sys_i]
            out["refined_to_1e-6"] = {
                "seconds": time.perf_counter() - t0,
                "inner_iters_max": max(i["iters"] for i in flat),
                "sweeps_max": max(i["sweeps"] for i in flat),
                "istop_counts": {str(k): sum(1 for i in flat if i["istop"] == k)
                                 for k in sorted({i["istop"] for i in flat})},
                "eta_fp64_max": max(i["eta_final_fp64"] for i in flat)}
        return out
    finally:
        for sol in sols:
            sol.close()


def batched_bench(args):
    """Batched form alone (see batched_measure), with the refined solve of
    every right-hand side to eta <= 1e-6.  Prints one JSON line."""
    iters = args.iters or 300
    out = {"metric": "batched LSQR right-hand-side iterations/s"}
    out.update(batched_measure(iters, args.steps, args.warmup, args.row_format, args.col_format,
                               refine=True))
    out.update(dtype="f32 values/vectors, f64 scalars", data="synthetic")
    print(json.dumps(out), flush=True)


def copy_calibration():
    """An elementwise kernel that reads 1 GiB and writes 1 GiB, three times:
    the reference the HBM counters are scaled by."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    del a, b


def block_products_bench(args):
    """The batched solver's two block products alone, 32 right-hand sides, on
    the batched workload's largest system (config-1 geometry, 229 stations,
    20 periods, seed 3) in its tuned schedule (32-wide tiles, 2,048
    workgroups): lsqr_apply_block (the per-run partial rows on the matrix
    cores, then their sums per data row) and lsqr_apply_t_block, timed with
    HIP events on the solver's stream, mean of `--steps` x 10 calls.  The
    run's HBM counters give the bytes each kernel moves.  Prints one JSON
    line."""
    import numpy as np
    import torch

    import synth
    from paper_2604_11920_amd import Solver
    s = synth.make_system(synth.config3_systems()[-1])
    k = s.col // s.nz                         # node runs: stretches of one lateral node
    new_run = np.ones(s.nnz, dtype=bool)
    new_run[1:] = k[1:] != k[:-1]
    new_run[s.row_ptr[:-1][np.diff(s.row_ptr) > 0]] = True
    runs = int(new_run.sum())
    del k, new_run
    if args.copy_calib:
        copy_calibration()
    R = 32
    with Solver.from_system(s, precond="jacobi") as sol:
        sol.set_batch_config(32, 2048)
        g = torch.Generator(device="cuda").manual_seed(1)
        x = torch.randn((s.n, R), dtype=torch.float32, device="cuda", generator=g)
        yb = torch.randn((s.m + 2 * s.n, R), dtype=torch.float32, device="cuda", generator=g)
        y, q = torch.empty_like(yb), torch.empty_like(x)
        st = torch.cuda.current_stream()
        res = {}
        for name, f in (("fwd", lambda: sol.apply_block(x, y)), ("adj", lambda: sol.apply_t_block(yb, q))):
            for _ in range(max(args.warmup, 1)):
                f()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10 * max(args.steps, 1)
            e0.record(st)
            for _ in range(reps):
                f()
            e1.record(st)
            torch.cuda.synchronize()
            res[name] = e0.elapsed_time(e1) / reps * 1e3
    print(json.dumps({"metric": "32-wide block products: microseconds per call",
                      "m": s.m, "n": s.n, "nnz": s.nnz, "node_runs": runs, "rhs": R,
                      "fwd_us": res["fwd"], "adj_us": res["adj"],
                      "fp32_value_bytes": 4 * s.nnz,
                      "partial_row_bytes_per_pass": runs * R * 4}), flush=True)


def products_bench(args):
    """The solver's two sparse products alone for one precision on the
    paper-shaped system, in the formats the solver picks (lsqr_apply_stored /
    lsqr_apply_t_stored: the same kernels and launch configuration as inside
    its iterations), timed with HIP events on the solver's stream, mean of
    `--steps` x 20 calls.  Prints one JSON line."""
    import torch

    import synth
    from paper_2604_11920_amd import Solver
    prec = args.products
    s = synth.make_system(synth.config1())
    if args.copy_calib:
        copy_calibration()
    kw = dict(precision=prec, row_format=args.row_format, col_format=args.col_format)
    if prec in ("bf16", "fp16"):
        kw["precond"] = "jacobi"
    with Solver.from_system(s, **kw) as sol:
        vdt = torch.float64 if prec == "fp64" else torch.float32
        g = torch.Generator(device="cuda").manual_seed(1)
        z = torch.randn(s.n, dtype=vdt, device="cuda", generator=g)
        yb = torch.randn(s.m + 2 * s.n, dtype=vdt, device="cuda", generator=g)
        y, q = torch.empty_like(yb), torch.empty_like(z)
        tg = yb[:s.m].clone() if prec in ("bf16", "fp16") else None
        st = torch.cuda.current_stream()
        res = {}
        for name, f in (("fwd", lambda: sol.apply_stored(z, y)),
                        ("adj", lambda: sol.apply_t_stored(yb, tg, q))):
            for _ in range(max(args.warmup, 1)):
                f()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20 * max(args.steps, 1)
            e0.record(st)
            for _ in range(reps):
                f()
            e1.record(st)
            torch.cuda.synchronize()
            res[name] = e0.elapsed_time(e1) / reps * 1e3
        ks = sol.kernel_stats()
    out = {"metric": f"{prec} sparse products: microseconds per launch and GB/s",
           "precision": prec, "m": s.m, "n": s.n, "nnz": s.nnz,
           "fwd": {"kernel": kernel_label("fwd", ks), "avg_us": res["fwd"],
                   "alg_bytes": ks["fwd_bytes"], "gbs": ks["fwd_bytes"] / res["fwd"] / 1e3,
                   "frac_of_hbm_peak": ks["fwd_bytes"] / res["fwd"] / 1e3 / HBM_PEAK_GBS},
           "adj": {"kernel": kernel_label("adj", ks), "avg_us": res["adj"],
                   "alg_bytes": ks["adj_bytes"], "gbs": ks["adj_bytes"] / res["adj"] / 1e3,
                   "frac_of_hbm_peak": ks["adj_bytes"] / res["adj"] / 1e3 / HBM_PEAK_GBS,
                   "padded_values": ks["padded_values"]},
           "data": "synthetic"}
    print(json.dumps(out), flush=True)


def outer_bench(args):
    """Outer iterations with synthetic re-linearisation on config 1 (3 steps,
    total form, FP64 + Jacobi, eta <= 1e-6 per step): warm start from the
    current model against a cold start, and the update form of eq. (6).
    Prints one JSON line."""
    import synth
    from paper_2604_11920_amd.outer import SyntheticForward, gauss_newton
    s = synth.make_system(synth.config1())
    fwd = SyntheticForward(s, 0.0, precond="jacobi")
    g0 = fwd.g0m(s.m_true)
    fwd.beta = 0.3 / float(np.abs(g0).max())
    d_obs = fwd.travel(s.m_true)
    runs = {}
    try:
        for name, kw in (("total_warm", dict(form="total", warm=True)),
                         ("total_cold", dict(form="total", warm=False)),
                         ("update", dict(form="update"))):
            out = gauss_newton(fwd, d_obs, np.zeros(s.n), outer=3, tol=1e-6, log=log, **kw)
            runs[name] = {"iters": out["iters"], "seconds": out["seconds"],
                          "rms": out["rms"].tolist(), "eta": out["eta"]}
    finally:
        fwd.close()
    res = {"metric": "outer iterations: LSQR iterations and seconds per outer step",
           "workload": "cfg1 re-linearised: T(m) = G0 m + beta/2 (G0 m)^2, beta = 0.3 / max|G0 m_true|",
           "tol": 1e-6, "precond": "jacobi", "runs": runs, "data": "synthetic"}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cfg1", choices=["cfg1", "cfg0"])
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--cpu-runs", type=int, default=10,
                    help="timed runs of the CPU oracle sample (the paper's protocol: 10)")
    ap.add_argument("--no-scipy", action="store_true", help="skip the SciPy LSQR context timing")
    ap.add_argument("--row-format", default="auto", choices=["auto", "csr", "groups"])
    ap.add_argument("--col-format", default="auto", choices=["auto", "csc", "runs", "pairs"])
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched multi-right-hand-side measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP32 rate and the time-to-tolerance comparisons")
    ap.add_argument("--ttt-tol", type=float, default=1e-6)
    ap.add_argument("--model", default=os.path.join(ROOT, "paper_2604_11920_amd", "colscale_mlp_c17.npz"),
                    help="learned column-scale model for the learned time-to-tolerance forms "
                         "(default: the model fitted on the 200 training systems of both shapes)")
    ap.add_argument("--outer", action="store_true",
                    help="measure the outer iterations with re-linearisation instead (one JSON line)")
    ap.add_argument("--products", choices=["fp64", "fp32", "bf16", "fp16"], default=None,
                    help="time the two sparse products alone in this precision (one JSON line)")
    ap.add_argument("--block-products", action="store_true",
                    help="time the batched form's two block products alone (one JSON line)")
    ap.add_argument("--batched", action="store_true",
                    help="measure the batched multi-RHS form instead (one JSON line)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print per-launch HBM traffic from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--pmc-formats", default=None,
                    help="'row/col' formats the counter runs used (as in kernel_stats: 1 CSR/CSC, 2 runs)")
    args = ap.parse_args()
    if args.pmc_summary:
        for k, v in pmc_summary(*args.pmc_summary, formats=args.pmc_formats).items():
            print(k, v)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the solver is single-GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2604_11920_amd import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.outer:
        outer_bench(args)
        return
    if args.batched:
        batched_bench(args)
        return
    if args.products:
        products_bench(args)
        return
    if args.block_products:
        block_products_bench(args)
        return
    t0 = time.perf_counter()
    if args.config == "cfg1":
        cfg = synth.config1()
        iters = args.iters or 300
        workload = ("cfg1: 80x80x20 grid (128,000 unknowns), 229 stations, 26,106 pairs x 20 "
                    "periods 1-40 s, paths >= 2 wavelengths, bent rays, 7-point smoothing x0.5, "
                    f"damp 0.1, {iters} LSQR iterations per step")
    else:
        cfg = synth.config0()
        iters = args.iters or 100
        workload = ("cfg0: 16x16x9 grid (2,304 unknowns), 40 stations, 780 pairs x 10 periods, "
                    f"straight rays, smoothing x0.5, damp 0.1, {iters} LSQR iterations per step")
    s = synth.make_system(cfg)
    gen_s = time.perf_counter() - t0
    log(f"[bench] generated {args.config}: m={s.m} n={s.n} nnz={s.nnz} in {gen_s:.1f}s")
    t0 = time.perf_counter()
    fmt = dict(row_format=args.row_format, col_format=args.col_format)
    sol = Solver.from_system(s, timing=True, **fmt)
    torch.cuda.synchronize()
    log(f"[bench] create (copy + device transpose) {time.perf_counter() - t0:.2f}s")
    dt = torch.from_numpy(s.dt).cuda()
    dm = torch.empty(s.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    if args.copy_calib:
        copy_calibration()

    for _ in range(args.warmup):
        sol.solve(dt, iters, dm=dm, history=False)
    torch.cuda.synchronize()
    fwd_ms = adj_ms = 0.0
    fwd_n = adj_n = 0
    per_step = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, _, info = sol.solve(dt, iters, dm=dm, history=False)
        per_step.append(time.perf_counter() - ts)
        ks = sol.kernel_stats()
        fwd_ms += ks["fwd_ms"]; adj_ms += ks["adj_ms"]
        fwd_n += ks["fwd_launches"]; adj_n += ks["adj_launches"]
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    gpu_ms = ev0.elapsed_time(ev1)
    assert info["iters"] == iters, info
    ms_per_step = wall * 1e3 / args.steps
    value = iters * args.steps / wall
    fwd_avg = fwd_ms / max(fwd_n, 1)
    adj_avg = adj_ms / max(adj_n, 1)
    fwd_gbs = ks["fwd_bytes"] / (fwd_avg * 1e-3) / 1e9
    adj_gbs = ks["adj_bytes"] / (adj_avg * 1e-3) / 1e9
    dom = "fwd" if fwd_ms >= adj_ms else "adj"
    dom_gbs = fwd_gbs if dom == "fwd" else adj_gbs
    # paper protocol: drop the slowest and fastest step, average the rest
    ps = sorted(per_step)
    trimmed = ps[1:-1] if len(ps) > 2 else ps
    log(f"[bench] {args.steps} steps: {ms_per_step:.2f} ms/step (events {gpu_ms / args.steps:.2f}), "
        f"{value:.1f} it/s; fwd {fwd_avg * 1e3:.1f} us {fwd_gbs:.0f} GB/s, adj {adj_avg * 1e3:.1f} us "
        f"{adj_gbs:.0f} GB/s")
    out = {
        "metric": METRIC, "value": value, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "m": s.m, "n": s.n, "nnz": s.nnz,
                   "iters_per_step": iters, "precision": "fp64", "precond": "none",
                   "row_format": args.row_format, "col_format": args.col_format},
        "roofline": {"bound": "hbm", "achieved": dom_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, f"{ks['row_format']}/{ks['col_format']}"),
                     "kernel": kernel_label(dom, ks)},
        "kernels": {"fwd": {"avg_us": fwd_avg * 1e3, "alg_bytes": ks["fwd_bytes"], "gbs": fwd_gbs},
                    "adj": {"avg_us": adj_avg * 1e3, "alg_bytes": ks["adj_bytes"], "gbs": adj_gbs}},
        "paper_protocol_ms_per_step": 1e3 * sum(trimmed) / len(trimmed),
    }
    sol.close()
    del sol
    if not args.no_extras:
        gold = golden_reference(s) if args.config == "cfg1" else None
        xstar = torch.from_numpy(gold["x_star"]).cuda() if gold is not None else None
        out["assembly"] = assembly_check(s, gen_s)
        out["fp32"] = fp32_rate(s, dt, iters, fmt, gold)
        out["time_to_tol"] = time_to_tol(s, dt, args.ttt_tol, fmt, args.model, xstar)
    if not args.no_batched and args.config == "cfg1":
        del dt, dm
        import torch
        torch.cuda.empty_cache()
        out["batched"] = batched_measure()
        log(f"[bench] batched: {out['batched']['value']:.0f} rhs-iters/s, matrix "
            f"{out['batched']['matrix_gbs']:.0f} GB/s")
    if not args.no_cpu:
        log("[bench] timing the CPU oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_iters, args.cpu_runs)
        log(f"[bench] cpu oracle {out['cpu_baseline']['value']:.3f} it/s on "
            f"{out['cpu_baseline']['cores']} threads ({out['cpu_baseline']['cpu_model']})")
        if args.config == "cfg1" and not args.no_scipy:
            out["scipy_lsqr"] = scipy_lsqr_context(s)
            log(f"[bench] scipy lsqr {out['scipy_lsqr']['value']:.3f} it/s (one thread)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
