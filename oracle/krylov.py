"""Krylov building blocks of the oracle (FP64, one vector at a time).

* ``cgs2_append``: classical Gram-Schmidt applied twice; the new direction is kept
  only if its norm after orthogonalisation exceeds a truncation threshold.  This is
  the single-column append of the global basis (Sec. 4.4: the new column's QR
  border [I, K^T z; 0, rho]) written for an orthonormal V, with the rank-revealing
  truncation read as "drop directions whose relative norm outside range(V) is
  below trunc".
* ``galerkin``: the outer projection.  The paper projects in the 2-norm of the
  residual (Sec. 4.1-4.2); in the CG form used here the initial guess on range(Q)
  is the A-Galerkin one, x0 = Q (Q^T A Q)^{-1} Q^T b, whose residual is orthogonal
  to range(Q) -- the analogue of r_j = (I - K K^T) b_j being orthogonal to K.
* ``deflated_cg``: CG on A g = r with the recycle space W deflated by A-orthogonal
  projection (Saad, Yeung, Erhel, Guyomarc'h 2000): the CG-form counterpart of
  MINRES on (I - K_j K_j^T) A (Sec. 4.2.1).  Its Galerkin start on range(W) plays
  the role of z in eq. (initialz).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla


def cgs2(Q: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Return v with its components along the orthonormal columns of Q removed, twice."""
    if Q.shape[1] == 0:
        return v.copy()
    w = v - Q @ (Q.T @ v)
    w = w - Q @ (Q.T @ w)
    return w


def cgs2_append(Q: np.ndarray, v: np.ndarray, trunc: float):
    """Normalise v, orthogonalise it against Q (CGS2); return (q or None, rho).

    rho is the norm of the orthogonalised unit vector: the relative size of the part
    of v outside range(Q).  The direction is kept only if rho > trunc.
    """
    nv = np.linalg.norm(v)
    if nv == 0.0:
        return None, 0.0
    w = cgs2(Q, v / nv)
    rho = float(np.linalg.norm(w))
    if rho > trunc:
        return w / rho, rho
    return None, rho


def galerkin(Q: np.ndarray, AQ: np.ndarray, b: np.ndarray):
    """A-Galerkin approximation on range(Q): x0 = Q G^{-1} Q^T b, G = Q^T A Q.

    AQ = A Q is passed in (the paper precomputes and borders it, Sec. 4.4).
    Returns (x0, r = b - A x0, c).
    """
    if Q.shape[1] == 0:
        return np.zeros_like(b), b.copy(), np.zeros(0)
    G = Q.T @ AQ
    G = 0.5 * (G + G.T)
    c = sla.cho_solve(sla.cho_factor(G, lower=True), Q.T @ b)
    x0 = Q @ c
    r = b - AQ @ c
    return x0, r, c


@dataclass
class CGResult:
    g: np.ndarray
    its: int
    resid: List[float] = field(default_factory=list)   # ||s_k|| per iteration
    breakdown: bool = False


def deflated_cg(A, r: np.ndarray, W: np.ndarray, tol_abs: float, maxit: int,
                AW: Optional[np.ndarray] = None) -> CGResult:
    """Deflated CG for A g = r with recycle space range(W).

    Start: g = W (W^T A W)^{-1} W^T r, s = r - A g, p = s - W (W^T A W)^{-1} (AW)^T s.
    Step:  w = A p, alpha = s^T s / p^T w, g += alpha p, s -= alpha w,
           stop when ||s|| <= tol_abs,
           beta = s_new^T s_new / s_old^T s_old,
           p = s + beta p - W (W^T A W)^{-1} (AW)^T s.
    """
    k = W.shape[1]
    if k:
        if AW is None:
            AW = A @ W
        GW = W.T @ AW
        GW = 0.5 * (GW + GW.T)
        fac = sla.cho_factor(GW, lower=True)
        y = sla.cho_solve(fac, W.T @ r)
        g = W @ y
        s = r - AW @ y
        p = s - W @ sla.cho_solve(fac, AW.T @ s)
    else:
        g = np.zeros_like(r)
        s = r.copy()
        p = s.copy()
    gamma = float(s @ s)
    res = CGResult(g=g, its=0, resid=[np.sqrt(gamma)])
    while np.sqrt(gamma) > tol_abs and res.its < maxit:
        w = A @ p
        pw = float(p @ w)
        if not (pw > 0.0) or not np.isfinite(pw):
            res.breakdown = True
            break
        alpha = gamma / pw
        g += alpha * p
        s -= alpha * w
        gamma_new = float(s @ s)
        res.its += 1
        res.resid.append(np.sqrt(gamma_new))
        if np.sqrt(gamma_new) <= tol_abs:
            gamma = gamma_new
            break
        beta = gamma_new / gamma
        gamma = gamma_new
        if k:
            p = s + beta * p - W @ sla.cho_solve(fac, AW.T @ s)
        else:
            p = s + beta * p
    res.g = g
    return res
