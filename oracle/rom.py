"""Full-order and reduced transfer functions at zero frequency (oracle).

* Full order (eq. (FullOrdTransFnc) rewritten in Sec. 3.1): Psi(p) = C~^T A(p)^{-1} B~,
  by a sparse direct solve, or column by column with full_solve on large grids.
* Reduced (eq. (newreduced)): E_r = V^T V, A_r(p) = V^T A(p) V, B_r = V^T B~,
  C_r = V^T C~, Psi_r(p) = C_r^T A_r(p)^{-1} B_r (omega = 0, so E_r does not enter).
* Jacobian column (eq. (newjac)): dPsi/dp_k = -C~^T A^{-1} Delta_k A^{-1} B~ with
  Delta_k = diag(d mu / d p_k); its reduced counterpart replaces A by A_r and
  Delta_k by V^T Delta_k V.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .krylov import deflated_cg


def full_transfer(A: sp.spmatrix, Bt: np.ndarray, Ct: np.ndarray) -> np.ndarray:
    """C~^T A^{-1} B~ by a sparse direct solve (n_det x n_src)."""
    lu = spla.splu(sp.csc_matrix(A))
    return Ct.T @ lu.solve(np.asarray(Bt, dtype=np.float64))


def full_solve(A: sp.spmatrix, b: np.ndarray, tol: float, maxit: int = 0) -> np.ndarray:
    """x = A^{-1} b to true relative residual ||b - A x|| <= tol ||b|| (Sec. 3: one
    full-order solve of eq. (blkeqn)), for grids too large for a direct solve: plain CG
    from zero, restarted from the true residual until the tolerance holds."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    maxit = maxit or 10 * A.shape[0]
    x = np.zeros_like(b)
    r = b.copy()
    its = 0
    empty = np.zeros((A.shape[0], 0))
    while np.linalg.norm(r) > tol * nb and its < maxit:
        cg = deflated_cg(A, r, empty, 0.5 * tol * nb, maxit - its)
        if cg.breakdown:
            raise ArithmeticError("CG breakdown: operator not SPD")
        its += cg.its
        x += cg.g
        r = b - A @ x
    return x


def reduced_matrices(V: np.ndarray, A: sp.spmatrix, Bt: np.ndarray, Ct: np.ndarray):
    """(A_r, B_r, C_r, E_r) of eq. (newreduced)."""
    Ar = V.T @ (A @ V)
    return Ar, V.T @ Bt, V.T @ Ct, V.T @ V


def reduced_transfer(Ar: np.ndarray, Br: np.ndarray, Cr: np.ndarray) -> np.ndarray:
    """C_r^T A_r^{-1} B_r (n_det x n_src)."""
    return Cr.T @ sla.solve(Ar, Br, assume_a="sym")


def full_jacobian_column(A: sp.spmatrix, Bt, Ct, dmu: np.ndarray) -> np.ndarray:
    """-C~^T A^{-1} diag(dmu) A^{-1} B~ (eq. (newjac))."""
    lu = spla.splu(sp.csc_matrix(A))
    Y = lu.solve(np.asarray(Bt, dtype=np.float64))
    Z = lu.solve(np.asarray(Ct, dtype=np.float64))
    return -Z.T @ (dmu[:, None] * Y)


def reduced_jacobian_column(V, Ar, Br, Cr, dmu: np.ndarray) -> np.ndarray:
    """-C_r^T A_r^{-1} (V^T diag(dmu) V) A_r^{-1} B_r."""
    Dr = V.T @ (dmu[:, None] * V)
    Yr = sla.solve(Ar, Br, assume_a="sym")
    Zr = sla.solve(Ar, Cr, assume_a="sym")
    return -Zr.T @ Dr @ Yr
