"""Learned column-scaling preconditioner: model container, target search,
GPU training driver and the solve with the Jacobi fallback.

A small MLP (6 -> 64 -> 64 -> 1, GELU, softplus output) maps per-column
features to a multiplier of the Jacobi scale, d_j = d_j^Jacobi softplus(z_j).
Any d > 0 leaves the least-squares solution unchanged; only the iteration
count moves.  Features, inference (BF16) and training (FP32 forward/backward
and Adam) run in the library's kernels; this module orchestrates them.

Training targets come from a search per system over a low-dimensional family
of log multipliers, either per depth layer

    l_j(theta) = a_{iz(j)} + b (f2_j - mean f2) + c (f6_j - mean f6)

(nz + 2 parameters: one per depth layer, ray coverage, neighbour coverage) or
the linear-in-depth family a0 + a1 f3_j + b (...) + c (...): coordinate
descent over theta on a grid {-1, -1/2, 1/2, 1} x step, the step halved each
round, minimising LSQR iterations to the tolerance, capped at twice Jacobi's
count.  The target of column j is l_j at the best theta.

Fallback and judge: a learned scale that is not finite and positive is
replaced by Jacobi inside the library; a learned solve that has not reached
the tolerance within twice the Jacobi iteration count continues with Jacobi
(the library's fallback budget, opts.fallback_iters).
"""
from __future__ import annotations

import dataclasses
import json
import math
import time

import numpy as np

from .lsqr import LsqrError, Solver, Trainer

NPARAMS = 4673
H = 64
# features centred on each system's own mean (their level shifts with the size
# of the survey): log column norm, log ray coverage, log neighbour coverage
CENTRE = (1 << 0) | (1 << 1) | (1 << 5)


@dataclasses.dataclass
class ColumnScaleModel:
    params: np.ndarray          # float32 [NPARAMS]
    mean: np.ndarray            # float32 [6] feature standardisation
    std: np.ndarray             # float32 [6]
    meta: dict

    @property
    def centre(self):
        return int(self.meta.get("centre", 0))

    def save(self, path):
        np.savez(path, params=self.params.astype(np.float32), mean=self.mean.astype(np.float32),
                 std=self.std.astype(np.float32), meta=np.array(json.dumps(self.meta)))

    @classmethod
    def load(cls, path):
        z = np.load(path, allow_pickle=False)
        return cls(params=z["params"], mean=z["mean"], std=z["std"], meta=json.loads(str(z["meta"])))


def initial_params(seed=0):
    """He-normal hidden weights, zero hidden biases, small output weights and
    the output bias at softplus^-1(1) = log(e - 1): the untrained net is Jacobi."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(H * 6) * math.sqrt(2.0 / 6), np.zeros(H),
             rng.standard_normal(H * H) * math.sqrt(2.0 / H), np.zeros(H),
             rng.standard_normal(H) * math.sqrt(2.0 / H) * 0.1, [math.log(math.e - 1.0)]]
    return np.concatenate([np.asarray(p, dtype=np.float64) for p in parts]).astype(np.float32)


def family_log_multiplier(feat, theta, nz=None):
    """l_j(theta) for host features [n, 6]: per-depth family when theta has
    nz + 2 entries, else the linear-in-depth family (see the module docstring)."""
    f = np.asarray(feat, dtype=np.float64)
    cov = f[:, 1] - f[:, 1].mean()
    nbr = f[:, 5] - f[:, 5].mean()
    theta = np.asarray(theta, dtype=np.float64)
    if nz is not None and len(theta) == nz + 2:
        iz = np.arange(len(f)) % nz
        return theta[iz] + theta[nz] * cov + theta[nz + 1] * nbr
    a0, a1, b, c = theta
    return a0 + a1 * f[:, 2] + b * cov + c * nbr


def iterations_to_tol(system, col_scale, tol, cap, solver=None):
    """LSQR iterations to eta <= tol with the given scale (None: Jacobi);
    cap + 1 when the tolerance is not reached.  `solver` (created with Jacobi
    scaling) is reused when given: the scale is swapped in place."""
    if solver is None:
        kw = dict(precond="jacobi") if col_scale is None else dict(precond="user", col_scale=col_scale)
        with Solver.from_system(system, check_every=8, **kw) as sol:
            dm, _, info = sol.solve(system.dt, int(cap), tol=tol, history=False)
    else:
        solver.set_scale(solver.jacobi_scale if col_scale is None else col_scale)
        dm, _, info = solver.solve(system.dt, int(cap), tol=tol, history=False)
    return info["iters"] if info["istop"] == 1 else int(cap) + 1, info


def search_targets(system, tol=1e-6, family="depth", grid=(-1.0, -0.5, 0.5, 1.0), step=0.5,
                   rounds=2, log=None, progress=None):
    """Coordinate descent over theta; returns (features [n,6], targets [n],
    theta, Jacobi iterations, best iterations).  One solver context serves
    every candidate (the scale is swapped in place)."""
    with Solver.from_system(system, precond="jacobi", check_every=8) as sol:
        feat = sol.column_features().cpu().numpy().astype(np.float64)
        djac = sol.scale()
        sol.jacobi_scale = djac
        kj, _ = iterations_to_tol(system, None, tol, 20000, solver=sol)
        nz = int(system.nz)
        theta = np.zeros(nz + 2 if family == "depth" else 4)
        best = kj
        for rnd in range(rounds):
            h = step * 0.5 ** rnd
            for p in range(len(theta)):
                base = theta[p]
                for v in grid:
                    th = theta.copy()
                    th[p] = base + v * h
                    d = djac * np.exp(family_log_multiplier(feat, th, nz))
                    k, _ = iterations_to_tol(system, d, tol, min(2 * kj, best + 1), solver=sol)
                    if k < best:
                        best, theta = k, th
                if progress:
                    progress(f"    round {rnd + 1} parameter {p + 1}/{len(theta)}: best {best}")
    if log:
        log(f"  search: jacobi {kj} -> best {best} at theta {np.round(theta, 3).tolist()}")
    return feat, family_log_multiplier(feat, theta, nz), theta, kj, best


def centred(feat, centre=CENTRE, mean=None):
    """Features of one system with the flagged columns minus their mean over
    the system's columns (`mean`: those means, when feat holds a sample of
    the columns only)."""
    f = np.array(feat, dtype=np.float64)
    for k in range(f.shape[1]):
        if (centre >> k) & 1:
            f[:, k] -= f[:, k].mean() if mean is None else mean[k]
    return f


def train(feats, targets, epochs=60, batch=4096, lr=1e-3, seed=0, centre=CENTRE, log=None,
          means=None):
    """Fit the MLP on the GPU (the library's FP32 forward/backward and Adam).
    feats: per-system [n_s, 6] feature blocks (flagged columns are centred per
    system, as inference does; `means`: per-system feature means over all
    columns, for blocks that hold a sample of them)."""
    import torch
    X = np.concatenate([centred(f, centre, None if means is None else means[i])
                        for i, f in enumerate(feats)]).astype(np.float64)
    T = np.concatenate(targets).astype(np.float64)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std == 0] = 1.0
    Xs = torch.from_numpy(((X - mean) / std).astype(np.float32)).cuda()
    Tt = torch.from_numpy(T.astype(np.float32)).cuda()
    N = len(T)
    batch = min(batch, N)
    tr = Trainer(initial_params(seed), batch)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).cuda()
        for s0 in range(0, N - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            tr.step(Xs[idx].contiguous(), Tt[idx].contiguous(), lr)
        if ep % 10 == 9 or ep == epochs - 1:
            losses = [tr.grad(Xs[i:i + batch].contiguous(), Tt[i:i + batch].contiguous())[1]
                      for i in range(0, N - batch + 1, batch)]
            hist.append((ep + 1, float(np.mean(losses))))
            if log:
                log(f"  epoch {ep + 1}: loss {hist[-1][1]:.4e}")
    params = tr.params()
    tr.close()
    base = float(np.mean(T ** 2))       # loss of the untrained (Jacobi) multiplier
    return ColumnScaleModel(params=params, mean=mean.astype(np.float32), std=std.astype(np.float32),
                            meta={"samples": int(N), "epochs": epochs, "batch": batch, "lr": lr,
                                  "loss_history": hist, "loss_at_jacobi": base,
                                  "centre": int(centre)})


def learned_scale(system, model, solver=None):
    """Host float64 [n] learned column scale for a system."""
    import torch
    p = torch.from_numpy(np.ascontiguousarray(model.params, dtype=np.float32)).cuda()
    if solver is not None:
        return solver.mlp_scale(p, model.mean, model.std, centre=model.centre).cpu().numpy()
    with Solver.from_system(system) as sol:
        return sol.mlp_scale(p, model.mean, model.std, centre=model.centre).cpu().numpy()


def solve_learned(system, model, tol, k_jacobi=None, cap=20000, precision="fp64"):
    """Solve with the learned scale.  The Jacobi fallback runs inside the
    library (opts.fallback_iters = twice the Jacobi count when k_jacobi is
    given): a scale that is not finite and positive is rejected when it is
    set, and a learned solve that has not reached the tolerance within the
    budget continues from its current iterate with the Jacobi scale.  One
    context: features and inference on it, then the scale is swapped in."""
    t0 = time.perf_counter()
    fb = 2 * int(k_jacobi) if k_jacobi else 0
    with Solver.from_system(system, precond="jacobi", precision=precision, check_every=16,
                            fallback_iters=fb) as sol:
        d = learned_scale(system, model, solver=sol)
        try:
            sol.set_scale(d)             # rejected unless finite and > 0
            rejected = False
        except LsqrError:
            rejected = True
        dm, _, info = sol.solve(system.dt, int(cap), tol=tol, history=False)
        if rejected:
            info["fallback_used"] = 1
    info["iters_total"] = info["iters"]  # including a failed learned attempt
    info["seconds"] = time.perf_counter() - t0
    return dm, info
