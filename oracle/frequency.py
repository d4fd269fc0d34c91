"""Nonzero modulation frequency (TEST INFRASTRUCTURE ONLY: used by tests/ and nothing else).

The frequency response of Sec. 2 with the symmetric rewriting of Sec. 3.1 is
Psi(omega; p) = C~^T (i omega/nu I + A(p))^{-1} B~, and the systems behind it are those of
eq. (solves): (A(p) + i sigma I) X = [B~, C~] with sigma = omega/nu.  Its reduced
counterpart (eq. (newreduced) and the transfer function right after it) is
Psi_r = C_r^T (i sigma E_r + A_r(p))^{-1} B_r with E_r = V^T V, A_r = V^T A V, B_r = V^T B~,
C_r = V^T C~.  The paper builds V at zero frequency only and leaves the construction at
nonzero frequency to later work; these are the definitions, written out with dense
complex solves (small grids only).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def shifted_solve(A, B: np.ndarray, sigma: float) -> np.ndarray:
    """X = (A + i sigma I)^{-1} B (complex, n x k) by a sparse direct solve."""
    n = A.shape[0]
    M = sp.csc_matrix(A, dtype=np.complex128) + 1j * sigma * sp.identity(n, format="csc")
    lu = spla.splu(M)
    return lu.solve(np.asarray(B, dtype=np.complex128))


def full_response(A, Bt: np.ndarray, Ct: np.ndarray, sigma: float) -> np.ndarray:
    """C~^T (A + i sigma I)^{-1} B~ (n_det x n_src, complex)."""
    return np.asarray(Ct).T @ shifted_solve(A, Bt, sigma)


def reduced_response(V: np.ndarray, A, Bt: np.ndarray, Ct: np.ndarray,
                     sigma: float) -> np.ndarray:
    """C_r^T (i sigma E_r + A_r)^{-1} B_r with the reduced matrices of V (any full-rank V)."""
    Er = V.T @ V
    Ar = V.T @ (A @ V)
    Br = V.T @ Bt
    Cr = V.T @ Ct
    M = Ar.astype(np.complex128) + 1j * sigma * Er
    return Cr.T @ np.linalg.solve(M, Br.astype(np.complex128))
