"""Outer iterations of the inversion with synthetic re-linearisation.

The paper's inversion (theoretical-framework section) solves the linear
system of eq. (6) for a model perturbation, updates the model, rebuilds the
sensitivity matrix G from the updated model and repeats until the RMS of the
traveltime residuals falls below a threshold.  Sensitivity kernels need the
physics codes the paper uses, so this driver re-linearises a synthetic
nonlinear forward model around the current model instead:

    T(m) = G0 m + (beta / 2) (G0 m)^2          (elementwise square)
    J(m) = diag(1 + beta G0 m) G0              (its Jacobian: G0 row-scaled)

with G0 a generated sensitivity matrix and d_obs = T(m_true) (+ noise).
Outer step k forms the residual dd_k = d_obs - T(m_k) and the perturbed
matrix G_k = J(m_k) (a new context on the same structure), then either

* form "update" (eq. (6) as written): solves [G_k; w L; lambda I] dm ~
  [dd_k; 0; 0] and sets m_{k+1} = m_k + dm, or
* form "total": solves [G_k; w L; lambda I] m ~ [dd_k + G_k m_k; 0; 0] for
  m_{k+1} itself, started from x0 = m_k (lsqr_solve_x0) - or from zero,
  for the cold-start comparison.

Every product and solve runs in the library's kernels (G0 m by the plain
product of a context on G0); the host forms the row scales and the scaled
values.  The column scale of the previous step can be reused for the next
(Solver.set_scale) instead of recomputing Jacobi.
"""
from __future__ import annotations

import time

import numpy as np

from .lsqr import Solver


def _row_repeat(row_ptr, v):
    return np.repeat(np.asarray(v, dtype=np.float64), np.diff(row_ptr))


class SyntheticForward:
    """T(m) and its Jacobian for a generated system s (row_ptr, col, val)."""

    def __init__(self, s, beta, **solver_kw):
        self.s = s
        self.beta = float(beta)
        self.kw = dict(solver_kw)
        self.base = Solver.from_system(s)           # G0, no column scale: plain products

    def close(self):
        self.base.close()

    def g0m(self, m_model):
        import torch
        x = torch.from_numpy(np.ascontiguousarray(m_model, dtype=np.float64)).cuda()
        return self.base.apply(x)[:self.s.m].cpu().numpy()

    def travel(self, m_model):
        y = self.g0m(m_model)
        return y + 0.5 * self.beta * y * y

    def jacobian_solver(self, m_model, **kw):
        """A context on J(m) = diag(1 + beta G0 m) G0 (same structure)."""
        rs = 1.0 + self.beta * self.g0m(m_model)
        val = self.s.val * _row_repeat(self.s.row_ptr, rs)
        args = dict(self.kw)
        args.update(kw)
        args.setdefault("damp", self.s.damp)
        args.setdefault("smooth", self.s.smooth)
        return Solver(self.s.row_ptr, self.s.col, val, self.s.nx, self.s.ny, self.s.nz, **args)


def gauss_newton(fwd, d_obs, m0, outer=4, tol=1e-6, iters=20000, form="total", warm=True,
                 reuse_scale=False, rms_stop=0.0, log=None):
    """Outer iterations.  Returns dict(m, rms [outer+1], iters [outer],
    seconds [outer], eta [outer])."""
    m = np.asarray(m0, dtype=np.float64).copy()
    rms = [float(np.sqrt(np.mean((d_obs - fwd.travel(m)) ** 2)))]
    its, secs, etas = [], [], []
    d_prev = None
    for k in range(outer):
        if rms_stop > 0.0 and rms[-1] <= rms_stop:
            break
        dd = d_obs - fwd.travel(m)
        kw = {"precond": "user", "col_scale": d_prev} if (reuse_scale and d_prev is not None) \
            else {}
        sol = fwd.jacobian_solver(m, **kw)
        try:
            t0 = time.perf_counter()
            if form == "update":
                dm, _, info = sol.solve(dd, iters, tol=tol, history=False)
                m = m + dm
            else:
                # G_k m_k by the context's own product (apply multiplies by D)
                rhs = dd + _apply_data(sol, m)
                x0 = m if warm else None
                m_new, _, info = sol.solve(rhs, iters, tol=tol, history=False, x0=x0)
                m = m_new
            secs.append(time.perf_counter() - t0)
            its.append(int(info["iters"]))
            etas.append(float(info["eta"]))
            if reuse_scale:
                d_prev = sol.scale()
        finally:
            sol.close()
        rms.append(float(np.sqrt(np.mean((d_obs - fwd.travel(m)) ** 2))))
        if log:
            log(f"[outer] step {k + 1}: {its[-1]} iterations, {secs[-1]:.2f} s, "
                f"rms {rms[-2]:.4e} -> {rms[-1]:.4e}")
    return dict(m=m, rms=np.array(rms), iters=its, seconds=secs, eta=etas)


def _apply_data(sol, x):
    """G x for the context's data block (unscaled x)."""
    import torch
    d = sol.scale()
    z = torch.from_numpy(np.ascontiguousarray(x / d)).cuda()
    return sol.apply(z)[:sol.m].cpu().numpy()
