"""ORACLE — test infrastructure only.  FP64 NumPy reference of a warm-started
least-squares solve on the explicit block operator of the LSQR oracle,
A_D = [G; w L; lambda I] D (products by the oracle's C operator), right-hand
side bbar = [dt; 0; 0].

The paper's inversion solves its linear system again after every model
update and re-linearisation (theoretical-framework section, eq. (6)); a solve
that starts from an initial solution x0 works on the correction problem
A_D y ~ r0 = bbar - Abar x0 and returns x = x0 + D y.  Written from that
definition with the LSQR of Paige & Saunders (ACM TOMS 8, 1982) on a general
right-hand side: Golub-Kahan bidiagonalisation started from r0, a Givens
rotation per step, the iterate update; LSMR (oracle/lsmr.py) on the same
correction problem for the LSMR form.  The stopping test is taken
explicitly: eta_k = |Abar^T (bbar - Abar x_k)| / |Abar^T bbar| (unscaled
norms; the D-scaled ones for LSMR), re-computed with the operator after
every step, so the oracle does not depend on LSQR's own estimates.
"""
from __future__ import annotations

import math

import numpy as np


def _norm(x):
    return math.sqrt(float(np.dot(x, x)))


def bbar_of(op, dt):
    b = np.zeros(op.mbar)
    b[:op.m] = np.asarray(dt, dtype=np.float64)
    return b


def unscaled_apply(op, x):
    """Abar x for an unscaled x (op.apply multiplies by D first)."""
    return op.apply(x if op.d is None else x / op.d)


def normal_residual(op, b, x, scaled=False):
    """|Abar^T (b - Abar x)|, or |D Abar^T (b - Abar x)| when scaled."""
    r = b - unscaled_apply(op, x)
    g = op.apply_t(r)                                   # D Abar^T r
    if op.d is not None and not scaled:
        g = g / op.d
    return _norm(g)


def lsqr_rhs(op, rhs, iters, stop=None):
    """LSQR on A_D y ~ rhs (full length m + 2n), at most `iters` steps;
    stop(y) -> bool is asked after every step.  Returns (y, steps, istop):
    istop 0 when A_D^T rhs = 0 (y = 0), 1 when stop() held, 2 at the step
    limit, 3 at an exact breakdown (beta or alpha zero)."""
    n = op.n
    y = np.zeros(n)
    beta = _norm(rhs)
    if beta == 0.0:
        return y, 0, 0
    u = rhs / beta
    q = op.apply_t(u)
    alpha = _norm(q)
    if alpha == 0.0:
        return y, 0, 0
    v = q / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    for k in range(1, iters + 1):
        p = op.apply(v) - alpha * u
        beta = _norm(p)
        if beta > 0.0:
            u = p / beta
            q = op.apply_t(u) - beta * v
            alpha = _norm(q)
            if alpha > 0.0:
                v = q / alpha
        else:
            alpha = 0.0
        rho = math.sqrt(rhobar * rhobar + beta * beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        y = y + (phi / rho) * w
        w = v - (theta / rho) * w
        if stop is not None and stop(y):
            return y, k, 1
        if alpha == 0.0 or beta == 0.0:
            return y, k, 3
    return y, iters, 2


def warm(op, dt, x0, iters, tol=0.0, method="lsqr"):
    """Solve from x0: x = x0 + D y with y the method's iterate on the
    correction problem.  tol > 0 stops when the explicit eta <= tol.
    Returns dict(x, iters, istop, eta)."""
    from .lsmr import lsmr
    b = bbar_of(op, dt)
    x0 = np.asarray(x0, dtype=np.float64)
    scaled = method == "lsmr"
    nb = normal_residual(op, b, np.zeros(op.n), scaled)
    r0 = b - unscaled_apply(op, x0)
    ref = nb if nb > 0.0 else normal_residual(op, b, x0, scaled)
    d = np.ones(op.n) if op.d is None else op.d

    def eta_of(y):
        return normal_residual(op, b, x0 + d * y, scaled) / ref if ref > 0.0 else 0.0

    if normal_residual(op, b, x0, scaled) == 0.0:
        return dict(x=x0.copy(), iters=0, istop=1, eta=0.0)
    if method == "lsqr":
        y, k, istop = lsqr_rhs(op, r0, iters,
                               stop=(lambda yy: eta_of(yy) <= tol) if tol > 0.0 else None)
    else:
        # LSMR's own iteration on the correction problem, stepped one count at
        # a time so that the explicit test decides the stop
        k, istop, y = 0, 2, np.zeros(op.n)
        for k in range(1, iters + 1):
            out = lsmr(op, None, k, 0.0, b=r0)
            y = out["x"] / d if op.d is not None else out["x"]
            if tol > 0.0 and eta_of(y) <= tol:
                istop = 1
                break
            if out["istop"] == 3:
                istop = 3
                break
    return dict(x=x0 + d * y, iters=k, istop=istop, eta=eta_of(y))
