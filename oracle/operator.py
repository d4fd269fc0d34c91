"""Operator assembly for the zero-frequency DOT problem (oracle, FP64, CSR).

What is computed (paper Sec. 3, eq. (block1), eq. (sum)):
  * Finite differences of -div(D grad eta) + mu eta on the unit square/cube, second
    order centred in the interior, first order for the Robin condition
    eta + 2 A D d(eta)/d(xi) = 0 on the source/detector faces (eq. ModelPDE2),
    eta = 0 on the lateral faces (eq. ModelPDE3).
  * The Robin boundary unknowns are eliminated by a Schur complement
    F - D2 G^{-1} D1 (Sec. 3), which is SPD at zero frequency.  Eliminating the
    first-order Robin row eta_b (1 + 2AD/h) = eta_1 (2AD/h) from the adjacent
    interior row leaves, on the diagonal of that row, c * h/(h + 2AD) for the face
    (c = D/h^2) instead of the Dirichlet value c.
  * A(p) = A_* + diag(mu(p)) (eq. (sum)): the parameter enters only the diagonal.

Readings (the paper is silent): unit domain, interior nodes at (i+1)h, h = 1/(N+1);
the operator is not scaled by h^2; with a per-node D the coefficient of an
interior face is the harmonic mean of the two node values and a boundary face uses
the adjacent node's value; the RBF is the Wendland C2 function (1-t)^4 (4t+1).

The module also assembles the *unreduced* boundary-node system of eq. (block1)
(boundary unknowns kept, no elimination anywhere) so that tests can check the
Schur form against it.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np
import scipy.sparse as sp

DIRICHLET = 0
ROBIN = 1


def _strides(N):
    return (1, N[0], N[0] * N[1])


def _D_nodes(D, n):
    if np.isscalar(D):
        return np.full(n, float(D))
    D = np.asarray(D, dtype=np.float64)
    assert D.shape == (n,)
    return D


def _multi_index(N, n):
    idx = np.arange(n)
    return idx % N[0], (idx // N[0]) % N[1], idx // (N[0] * N[1])


def assemble_Astar(dim: int, N, bc, D, robin_A: float) -> sp.csr_matrix:
    """The parameter-free part A_* of eq. (sum) as CSR (n x n)."""
    N = tuple(N)
    n = N[0] * N[1] * N[2]
    Dn = _D_nodes(D, n)
    coord = _multi_index(N, n)
    st = _strides(N)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for a in range(dim):
        h = 1.0 / (N[a] + 1)
        i = coord[a]
        # interior faces between node k and k + stride
        has_plus = i < N[a] - 1
        k = np.nonzero(has_plus)[0]
        kp = k + st[a]
        if np.isscalar(D):
            Dface = np.full(k.shape, float(D))
        else:
            Dface = 2.0 * Dn[k] * Dn[kp] / (Dn[k] + Dn[kp])
        c = Dface / h ** 2
        rows += [k, kp]
        cols += [kp, k]
        vals += [-c, -c]
        np.add.at(diag, k, c)
        np.add.at(diag, kp, c)
        # boundary faces (missing neighbour across the face)
        for side, on_face in ((0, i == 0), (1, i == N[a] - 1)):
            kb = np.nonzero(on_face)[0]
            cb = Dn[kb] / h ** 2
            if bc[2 * a + side] == ROBIN:
                beta = h / (h + 2.0 * robin_A * Dn[kb])
            else:
                beta = np.ones_like(cb)
            np.add.at(diag, kb, cb * beta)
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def wendland(t):
    """Compactly supported Wendland C2 function psi(t) = (1-t)^4 (4t+1) for t < 1."""
    t = np.asarray(t, dtype=np.float64)
    return np.where(t < 1.0, (1.0 - t) ** 4 * (4.0 * t + 1.0), 0.0)


def node_coords(dim: int, N) -> np.ndarray:
    n = N[0] * N[1] * N[2]
    coord = _multi_index(N, n)
    return np.stack([(coord[a] + 1.0) / (N[a] + 1) for a in range(dim)], axis=1)


def mu_field(dim: int, N, mu0: float, centers, radii, amps) -> np.ndarray:
    """mu(x; p) = mu0 + sum_b a_b psi(|x - c_b| / r_b) at every unknown (Sec. 2.1, Sec. 5)."""
    X = node_coords(dim, N)
    mu = np.full(X.shape[0], float(mu0))
    for c, r, a in zip(np.asarray(centers), np.asarray(radii), np.asarray(amps)):
        dist = np.sqrt(((X - c[None, :]) ** 2).sum(axis=1))
        mu += a * wendland(dist / r)
    return mu


def mu_gradient(dim: int, N, centers, radii, amps) -> np.ndarray:
    """d mu / d p_k at every unknown for the bump parameters, per bump b in the order
    (a_b, r_b, c_b[0], .., c_b[dim-1]): rows b (dim + 2) + (0, 1, 2 + d).

    With t = |x - c| / r and psi(t) = (1-t)^4 (4t+1), psi'(t) = -20 t (1-t)^3 (zero for
    t >= 1), so
      d mu / d a = psi(t),
      d mu / d r = a psi'(t) (-t / r)            = 20 a t^2 (1-t)^3 / r,
      d mu / d c_d = a psi'(t) (-(x_d - c_d) / (r |x - c|)) = 20 a (1-t)^3 (x_d - c_d) / r^2.
    (the Jacobian columns of eq. (newjac) take Delta_k = diag of these)."""
    X = node_coords(dim, N)
    centers = np.asarray(centers, dtype=np.float64)
    out = []
    for c, r, a in zip(centers, np.asarray(radii, dtype=np.float64),
                       np.asarray(amps, dtype=np.float64)):
        diff = X - c[None, :]
        t = np.sqrt((diff ** 2).sum(axis=1)) / r
        inside = t < 1.0
        u3 = np.where(inside, (1.0 - t) ** 3, 0.0)
        out.append(wendland(t))
        out.append(20.0 * a * t * t * u3 / r)
        for d in range(dim):
            out.append(20.0 * a * u3 * diff[:, d] / (r * r))
    return np.array(out).reshape(-1, X.shape[0])


def assemble_A(Astar: sp.csr_matrix, mu: np.ndarray) -> sp.csr_matrix:
    """A(p) = A_* + diag(mu(p)) (eq. (sum))."""
    return (Astar + sp.diags(mu)).tocsr()


# --------------------------------------------------------------------------------------
# The unreduced system of eq. (block1), boundary unknowns first.


def full_boundary_system(dim: int, N, bc, D, robin_A: float, mu: np.ndarray):
    """Assemble the unsymmetric boundary-node system of eq. (block1) at omega = 0.

    Unknowns: the Robin boundary nodes (one per boundary face of a node on a Robin
    face, located at distance h outside it) followed by the interior nodes.  Rows:
      * interior node: sum over its faces of c (eta_i - eta_nbr) + mu_i eta_i with
        eta_nbr = 0 across a Dirichlet face and eta_nbr a boundary unknown across a
        Robin face;
      * Robin boundary node b next to interior node i (first-order difference of
        the outward derivative): eta_b + 2 A D_i (eta_b - eta_i)/h = 0.
    Returns (M, nb_bnd, bnd_of) where M is dense (n_b + n) x (n_b + n) ordered
    [boundary; interior] and bnd_of maps (interior node, face) -> boundary slot.
    """
    N = tuple(N)
    n = N[0] * N[1] * N[2]
    Dn = _D_nodes(D, n)
    coord = _multi_index(N, n)
    st = _strides(N)
    bnd_of: Dict[Tuple[int, int], int] = {}
    for a in range(dim):
        for side in (0, 1):
            if bc[2 * a + side] != ROBIN:
                continue
            on = np.nonzero(coord[a] == (0 if side == 0 else N[a] - 1))[0]
            for k in on:
                bnd_of[(int(k), 2 * a + side)] = len(bnd_of)
    nbnd = len(bnd_of)
    M = np.zeros((nbnd + n, nbnd + n))
    for k in range(n):
        row = nbnd + k
        M[row, row] += mu[k]
        for a in range(dim):
            h = 1.0 / (N[a] + 1)
            for side, step in ((0, -1), (1, +1)):
                j = coord[a][k] + step
                if 0 <= j < N[a]:
                    kn = k + step * st[a]
                    if np.isscalar(D):
                        Df = float(D)
                    else:
                        Df = 2 * Dn[k] * Dn[kn] / (Dn[k] + Dn[kn])
                    c = Df / h ** 2
                    M[row, row] += c
                    M[row, nbnd + kn] -= c
                else:
                    c = Dn[k] / h ** 2
                    M[row, row] += c
                    if bc[2 * a + side] == ROBIN:
                        M[row, bnd_of[(k, 2 * a + side)]] -= c
    for (k, face), s in bnd_of.items():
        a = face // 2
        h = 1.0 / (N[a] + 1)
        g = 2.0 * robin_A * Dn[k] / h
        M[s, s] = 1.0 + g
        M[s, nbnd + k] = -g
    return M, nbnd, bnd_of
