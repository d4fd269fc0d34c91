"""Algorithm 2 of the paper (recycling and global basis construction), CG form.

The paper (Sec. 4.2-4.3, Algorithm 2) solves A_i X_i = B, B = [B~, C~] (eq. (blkeqn))
for a sequence of parameter points.  For every point and right-hand side it
  1. checks whether the global basis V already represents the solution (outer
     projection on range(V); no iteration if the relative residual <= tol),
  2. otherwise solves the correction equation A g_j = r_j (eq. (resi)) with a
     Krylov method recycling the small space U_j (Sec. 4.2.1),
  3. appends the new information to V and to U_j.
Initialisation (Sec. 4.2.2): U_0 = estimates of the low eigenvectors of A_0,
V = range([U_0, X_0]), U_j = [U_0, X_0(:, j)].

Readings taken here (the paper uses MINRES with 2-norm projections; this build
uses CG with A-orthogonal projections):
  * outer projection: A_i-Galerkin on range(Q), Q an orthonormal basis of V;
  * inner solve: deflated CG on A_i g = r_j with W = U_j; stop when the updated
    residual norm <= tol ||b_j||, then the true residual ||b_j - A_i x_j|| is
    recomputed and, if above tol ||b_j||, CG restarts from it (same W);
  * appended vector: the correction g (its new part equals that of the Krylov
    part y_m because g - y_m lies in range(U_j), a subset of range(V)), normalised
    and CGS2-orthogonalised against Q, kept iff its remaining norm > trunc and the
    basis is below its cap;
  * X_0 is produced by running the same loop at p_0 with Q = orth(U_0) and
    U_j = U_0 for every j; afterwards U_j = [U_0, X_0(:, j)];
  * U_j is stored orthonormal (U_0 part = the first columns of Q; each added
    column CGS2-orthogonalised against U_j); a correction joins U_j only if it
    joined V, so range(U_j) stays inside range(V).
  * uj_cap (None: unbounded, as in the paper): the most columns U_j may hold; a kept
    correction joins V but not U_j once U_j has uj_cap columns, and X_0(:, j) joins
    U_j only while k_u < uj_cap (the GPU library holds U_j in at most 64 columns);
  * group g (the batched form; g = 1 is the paper's order): the right-hand sides of
    a point are taken in consecutive groups of g.  Every member of a group is
    projected on the basis as it stands at the start of the group and solved
    without the other members' corrections; the group's corrections are then
    appended one by one in right-hand-side order, each exactly as for g = 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .krylov import cgs2_append, deflated_cg, galerkin


@dataclass
class Record:
    point: int
    rhs: int
    rho0: float          # initial relative residual after the outer projection
    its: int             # inner CG iterations (0 if skipped)
    solved: bool         # inner solve was run
    kept: bool           # correction appended to the global basis
    rho: float           # norm of the normalised correction outside range(Q) (nan if not solved)
    final_res: float     # true relative residual ||b - A x|| / ||b||
    m: int               # basis size after this right-hand side
    restarts: int = 0
    converged: bool = True


@dataclass
class SequenceResult:
    Q: np.ndarray
    X: List[np.ndarray]
    records: List[Record]
    W_extra: List[List[np.ndarray]]
    k_u: int


def _inner_solve(A, b, nb, x0, r, Wj, tol, maxit):
    """Deflated CG on A g = r with W = U_j, restarted from the true residual until
    ||b - A (x0 + g)|| <= tol ||b|| or maxit iterations."""
    AW = A @ Wj
    res = deflated_cg(A, r, Wj, tol * nb, maxit, AW=AW)
    g, its = res.g, res.its
    x = x0 + g
    rt = b - A @ x
    restarts = 0
    while np.linalg.norm(rt) > tol * nb and its < maxit and not res.breakdown:
        res = deflated_cg(A, rt, Wj, tol * nb, maxit - its, AW=AW)
        g = g + res.g
        its += res.its
        restarts += 1
        x = x0 + g
        rt = b - A @ x
    return g, x, its, restarts, float(np.linalg.norm(rt)) / nb


def solve_sequence(Astar: sp.csr_matrix, mus: List[np.ndarray], B: np.ndarray, U0: np.ndarray,
                   tol: float, trunc: float = 1e-8, cap: int = 0, maxit: Optional[int] = None,
                   keep_X: bool = True, group: int = 1,
                   uj_cap: Optional[int] = None) -> SequenceResult:
    n, n_rhs = B.shape
    if group < 1:
        raise ValueError("group must be >= 1")
    if maxit is None:
        maxit = n
    # V <- basis for range(U_0)
    Q = np.zeros((n, 0))
    for c in range(U0.shape[1]):
        q, _ = cgs2_append(Q, U0[:, c], trunc)
        if q is not None:
            Q = np.column_stack([Q, q])
    k_u = Q.shape[1]
    W_extra: List[List[np.ndarray]] = [[] for _ in range(n_rhs)]
    X: List[np.ndarray] = []
    records: List[Record] = []
    for i, mu in enumerate(mus):
        A = (Astar + sp.diags(mu)).tocsr()
        AQ = A @ Q
        Xi = np.zeros((n, n_rhs)) if keep_X or i == 0 else None
        for j0 in range(0, n_rhs, group):
            members = range(j0, min(j0 + group, n_rhs))
            solved = {}
            recs = {}
            # projections and solves against the basis as it stands at the group start
            for j in members:
                b = B[:, j]
                nb = float(np.linalg.norm(b))
                x0, r, _ = galerkin(Q, AQ, b)
                rho0 = float(np.linalg.norm(r)) / nb
                if rho0 <= tol:
                    recs[j] = Record(i, j, rho0, 0, False, False, float("nan"), rho0, Q.shape[1])
                    x = x0
                else:
                    Wj = np.column_stack([Q[:, :k_u]] + W_extra[j]) if (i > 0 and W_extra[j]) \
                        else Q[:, :k_u]
                    g, x, its, restarts, final = _inner_solve(A, b, nb, x0, r, Wj, tol, maxit)
                    solved[j] = (g, Wj)
                    recs[j] = Record(i, j, rho0, its, True, False, float("nan"), final, 0,
                                     restarts, converged=final <= tol)
                if Xi is not None:
                    Xi[:, j] = x
            # the group's corrections join V (and U_j) in right-hand-side order
            for j in members:
                rec = recs[j]
                if j in solved:
                    g, Wj = solved[j]
                    q, rho = cgs2_append(Q, g, trunc)
                    kept = q is not None and (cap == 0 or Q.shape[1] < cap)
                    if kept:
                        Q = np.column_stack([Q, q])
                        AQ = np.column_stack([AQ, A @ q])
                        if i > 0 and (uj_cap is None or Wj.shape[1] < uj_cap):
                            w, _ = cgs2_append(Wj, g, trunc)
                            if w is not None:
                                W_extra[j].append(w)
                    rec.kept, rec.rho = kept, rho
                rec.m = Q.shape[1]
                records.append(rec)
        if i == 0:
            for j in range(n_rhs):
                w, _ = cgs2_append(Q[:, :k_u], Xi[:, j], trunc)
                W_extra[j] = [w] if w is not None and (uj_cap is None or k_u < uj_cap) else []
        X.append(Xi)
    return SequenceResult(Q, X, records, W_extra, k_u)


def rhs_matrix(n: int, src_idx, src_scale, det_idx, det_scale) -> np.ndarray:
    """B = [B~, C~] as dense scaled identity columns, sources first (eq. (blkeqn))."""
    idx = np.concatenate([np.asarray(src_idx), np.asarray(det_idx)])
    sc = np.concatenate([np.asarray(src_scale, float), np.asarray(det_scale, float)])
    B = np.zeros((n, idx.size))
    B[idx, np.arange(idx.size)] = sc
    return B
