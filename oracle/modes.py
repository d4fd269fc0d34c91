"""Lowest eigenpairs of A(p) (TEST INFRASTRUCTURE ONLY: used by tests/ and nothing else).

U_0 of Algorithm 2 (Sec. 4.2.2) is a block of eigenvectors of the operator for its
smallest eigenvalues; the paper computes it offline.  The definition, written out: the
k smallest eigenvalues of the SPD matrix A and orthonormal eigenvectors for them, by a
dense symmetric eigendecomposition (small grids only).  Eigenvectors are unique only up to
sign, and only the invariant subspace of a cluster of equal eigenvalues is unique.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def lowest_modes(A, k: int):
    """(lambda[0..k), V n x k): the k smallest eigenpairs of the symmetric matrix A."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    lam, V = np.linalg.eigh(0.5 * (Ad + Ad.T))
    return lam[:k], V[:, :k]


def gershgorin_upper(A) -> float:
    """max_i sum_j |a_ij|, an upper bound of the spectrum of a symmetric A (sparse A stays
    sparse, so this also serves full-size grids)."""
    if sp.issparse(A):
        return float(np.asarray(abs(A).sum(axis=1)).max())
    return float(np.abs(np.asarray(A, dtype=np.float64)).sum(axis=1).max())
