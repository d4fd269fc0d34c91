"""Pins for the lowest-eigenpair oracle (U_0 of Algorithm 2): the closed-form spectrum
and an exact sine eigenvector of the all-Dirichlet constant-coefficient operator, the
eigen-residual and orthonormality on a variable-coefficient operator with absorption
bumps, the Ky Fan minimum (no orthonormal block has a smaller Rayleigh-quotient trace),
and the Gershgorin bound above the largest eigenvalue."""
import numpy as np

import phantoms as ph
from oracle import modes
from oracle import operator as op


def test_closed_form_lowest_eigenvalues():
    dim, N, D = 3, (6, 5, 4), 0.04
    A = op.assemble_Astar(dim, N, (0,) * 6, D, 1.0)
    lam, V = modes.lowest_modes(A, 7)
    axes = []
    for a in range(dim):
        h = 1.0 / (N[a] + 1)
        kk = np.arange(1, N[a] + 1)
        axes.append(4 * D / h ** 2 * np.sin(kk * np.pi / (2 * (N[a] + 1))) ** 2)
    ref = np.sort(np.add.outer(np.add.outer(axes[2], axes[1]), axes[0]).reshape(-1))[:7]
    np.testing.assert_allclose(lam, ref, rtol=1e-12)
    # the lowest mode is the product of first sines (simple eigenvalue): equal up to sign
    v = np.ones(1)
    for a in range(dim):
        i = np.arange(N[a]) + 1
        va = np.sin(np.pi * i / (N[a] + 1))
        v = np.multiply.outer(va, v) if a else va
    v = v.reshape(-1) / np.linalg.norm(v)
    assert abs(abs(v @ V[:, 0]) - 1.0) <= 1e-12


def test_invariants_variable_operator():
    wl = ph.small(3, (7, 6, 5), D="lognormal")
    A = op.assemble_A(op.assemble_Astar(wl.dim, wl.N, wl.bc, ph.diffusion_field(wl), wl.robin_A),
                      op.mu_field(wl.dim, wl.N, 0.01, [[0.4, 0.5, 0.6]], [0.3], [0.02]))
    lam, V = modes.lowest_modes(A, 10)
    assert np.all(np.diff(lam) >= 0)
    assert np.abs(V.T @ V - np.eye(10)).max() <= 1e-12
    R = A @ V - V * lam
    assert np.abs(R).max() <= 1e-12 * modes.gershgorin_upper(A)
    # Ky Fan: trace(Q^T A Q) >= sum of the 10 smallest for every orthonormal Q
    rng = np.random.default_rng(3)
    for _ in range(5):
        Q, _ = np.linalg.qr(V + 0.1 * rng.standard_normal(V.shape))
        assert np.trace(Q.T @ (A @ Q)) >= lam.sum() - 1e-12 * abs(lam.sum())
    # a planted mistake (the 10 largest instead) breaks the minimum
    lam_all = np.linalg.eigvalsh(A.toarray())
    assert lam_all[-10:].sum() > lam.sum() * (1 + 1e-3)
    assert modes.gershgorin_upper(A) >= lam_all[-1]
