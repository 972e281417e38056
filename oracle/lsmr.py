"""ORACLE — test infrastructure only.  FP64 NumPy reference of LSMR (Fong &
Saunders 2011), the solver the paper's "Solver for the Large-scale Linear
System" section says DSurfTomo adopts, on the same explicit block operator
as the LSQR oracle: A_D = [G; w L; lambda I] D (products by the oracle's C
operator), right-hand side bbar = [dt; 0; 0], x = D y.

LSMR is MINRES applied to the normal equations A_D^T A_D y = A_D^T bbar:
after the Golub-Kahan bidiagonalisation (shared with LSQR) it applies two
chains of plane rotations, so that y_k minimises |A_D^T (bbar - A_D y)|
over the Krylov space K_k(A_D^T A_D, A_D^T bbar).  Written from the method's
definition in the paper of Fong & Saunders (SIAM J. Sci. Comput. 33, 2011):
the bidiagonalisation, the rotations P_k (on [alphabar_k, beta_{k+1}]) and
Pbar_k (on [cbar_{k-1} rho_k, theta_{k+1}]), the h / hbar recurrences, and
the estimate of |r_k| by a third rotation chain.  Damping is an explicit
operator block, so the internal damping of the method is zero.

History row k (k = 0 .. K): (|r_k| estimate, |A_D^T r_k| = |zetabar_{k+1}|,
eta_k = |zetabar_{k+1}| / (alpha_1 beta_1)); eta is the normal-equation
residual in the scaled variables, equal to |Abar^T r| / |Abar^T bbar| when
D = I.  Stop reasons as for the LSQR oracle (0 zero rhs, 1 eta <= tol,
2 iteration limit, 3 exact breakdown).
"""
from __future__ import annotations

import math

import numpy as np


def _norm(x):
    return math.sqrt(float(np.dot(x, x)))


def lsmr(op, dt, iters, tol=0.0, b=None):
    """LSMR on the oracle operator `op` (oracle.Operator).  b: optional full
    right-hand side [m + 2n] used instead of [dt; 0; 0].  Returns
    dict(x, hist [K+1, 3], istop, iters)."""
    m, n = op.m, op.n
    if b is None:
        b = np.zeros(op.mbar)
        b[:m] = np.asarray(dt, dtype=np.float64)
    else:
        b = np.asarray(b, dtype=np.float64)
    hist = np.full((iters + 1, 3), np.nan)
    beta = _norm(b)
    if beta == 0.0:
        hist[0] = (0.0, 0.0, 0.0)
        return dict(x=np.zeros(n), hist=hist[:1], istop=0, iters=0)
    u = b / beta
    q = op.apply_t(u)
    alpha = _norm(q)
    if alpha == 0.0:
        hist[0] = (beta, 0.0, 0.0)
        return dict(x=np.zeros(n), hist=hist[:1], istop=0, iters=0)
    v = q / alpha
    # rotation state
    alphabar, zetabar = alpha, alpha * beta
    rho, rhobar, cbar, sbar = 1.0, 1.0, 1.0, 0.0
    h = v.copy()
    hbar = np.zeros(n)
    y = np.zeros(n)
    arnorm0 = alpha * beta
    # |r_k| estimate state
    betadd, betad, rhodold, tautildeold, thetatilde, zeta = beta, 0.0, 1.0, 0.0, 0.0, 0.0
    hist[0] = (beta, arnorm0, 1.0)
    istop, k = 2, 0
    for k in range(1, iters + 1):
        # bidiagonalisation
        t = op.apply(v) - alpha * u
        beta = _norm(t)
        if beta > 0.0:
            u = t / beta
            q = op.apply_t(u) - beta * v
            alpha = _norm(q)
            if alpha > 0.0:
                v = q / alpha
        else:
            alpha = 0.0
        # rotation P_k: annihilates beta_{k+1} below alphabar_k
        rhoold = rho
        rho = math.sqrt(alphabar * alphabar + beta * beta)
        c = alphabar / rho
        s = beta / rho
        thetanew = s * alpha
        alphabar = c * alpha
        # rotation Pbar_k: annihilates theta_{k+1} in the normal-equation factor
        rhobarold = rhobar
        zetaold = zeta
        thetabar = sbar * rho
        rhotemp = cbar * rho
        rhobar = math.sqrt(rhotemp * rhotemp + thetanew * thetanew)
        cbar = rhotemp / rhobar
        sbar = thetanew / rhobar
        zeta = cbar * zetabar
        zetabar = -sbar * zetabar
        # h, hbar and the iterate
        hbar = h - (thetabar * rho / (rhoold * rhobarold)) * hbar
        y = y + (zeta / (rho * rhobar)) * hbar
        h = v - (thetanew / rho) * h
        # |r_k| by a third rotation chain
        betahat = c * betadd
        betadd = -s * betadd
        thetatildeold = thetatilde
        rhotildeold = math.sqrt(rhodold * rhodold + thetabar * thetabar)
        ctildeold = rhodold / rhotildeold
        stildeold = thetabar / rhotildeold
        thetatilde = stildeold * rhobar
        rhodold = ctildeold * rhobar
        betad = -stildeold * betad + ctildeold * betahat
        tautildeold = (zetaold - thetatildeold * tautildeold) / rhotildeold
        taud = (zeta - thetatilde * tautildeold) / rhodold
        normr = math.sqrt((betad - taud) ** 2 + betadd * betadd)
        normar = abs(zetabar)
        eta = normar / arnorm0
        hist[k] = (normr, normar, eta)
        if not all(map(math.isfinite, (rho, rhobar, zeta, normr))):
            raise FloatingPointError("LSMR scalar became non-finite")
        if tol > 0.0 and eta <= tol:
            istop = 1
            break
        if alpha == 0.0 or beta == 0.0:
            istop = 3
            break
    return dict(x=y if op.d is None else op.d * y, hist=hist[:k + 1], istop=istop, iters=k)
