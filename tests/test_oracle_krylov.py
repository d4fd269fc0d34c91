"""Pins for the oracle's Krylov building blocks (CGS2 append, Galerkin start, deflated CG)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import phantoms as ph
from oracle import krylov as kr
from oracle import operator as op


def _operator(wl, seed=0):
    D = ph.diffusion_field(wl)
    As = op.assemble_Astar(wl.dim, wl.N, wl.bc, D, wl.robin_A)
    p = ph.parameter_points(wl, K=1)[0]
    mu = op.mu_field(wl.dim, wl.N, p.mu0, p.centers, p.radii, p.amps)
    return op.assemble_A(As, mu)


def test_cgs2_orthonormal_and_truncation():
    rng = np.random.default_rng(0)
    n = 500
    Q = np.zeros((n, 0))
    for _ in range(60):
        q, rho = kr.cgs2_append(Q, rng.standard_normal(n) + 1e3 * Q @ rng.standard_normal(Q.shape[1]), 1e-8)
        assert q is not None
        Q = np.column_stack([Q, q])
    assert np.abs(Q.T @ Q - np.eye(60)).max() < 1e-13
    # exact duplicate (up to scale) is dropped
    v = Q @ rng.standard_normal(60)
    q, rho = kr.cgs2_append(Q, 3.0 * v, 1e-8)
    assert q is None and rho < 1e-14
    # a 1e-6 relative perturbation outside range(Q) is kept; rho equals the distance
    # of the unit vector from range(Q) (least squares via a library routine)
    e = rng.standard_normal(n)
    w = v / np.linalg.norm(v) + 1e-6 * e / np.linalg.norm(e)
    q, rho = kr.cgs2_append(Q, w, 1e-8)
    u = w / np.linalg.norm(w)
    coef = np.linalg.lstsq(Q, u, rcond=None)[0]
    dist = np.linalg.norm(u - Q @ coef)
    assert q is not None and abs(rho - dist) < 1e-9 * dist


def test_galerkin_properties():
    wl = ph.small(3, (6, 5, 7))
    A = _operator(wl)
    n = wl.n
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((n, 12)))
    b = rng.standard_normal(n)
    AQ = A @ Q
    x0, r, c = kr.galerkin(Q, AQ, b)
    # residual orthogonal to range(Q), x0 in range(Q)
    assert np.abs(Q.T @ r).max() < 1e-12 * np.linalg.norm(b)
    np.testing.assert_allclose(Q @ (Q.T @ x0), x0, atol=1e-13 * np.linalg.norm(x0))
    # A-norm optimality against random perturbations inside range(Q)
    xs = spla.spsolve(A.tocsc(), b)
    Ad = A.toarray()
    e0 = (x0 - xs) @ Ad @ (x0 - xs)
    for _ in range(20):
        d = Q @ rng.standard_normal(12) * 1e-3
        e = (x0 + d - xs) @ Ad @ (x0 + d - xs)
        assert e >= e0
    # full space -> exact solution
    Qf, _ = np.linalg.qr(rng.standard_normal((n, n)))
    xf, rf, _ = kr.galerkin(Qf, A @ Qf, b)
    np.testing.assert_allclose(xf, xs, rtol=1e-9, atol=1e-12 * np.abs(xs).max())


def test_galerkin_catches_missing_gram():
    """Planted mistake: c = Q^T b without the Gram solve breaks orthogonality of r."""
    wl = ph.small(2, (10, 10))
    A = _operator(wl)
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((wl.n, 6)))
    b = rng.standard_normal(wl.n)
    c = Q.T @ b
    r = b - A @ (Q @ c)
    assert np.abs(Q.T @ r).max() > 1e-3 * np.linalg.norm(b)


def _scipy_cg_iterations(A, b, rtol):
    its = [0]

    def cb(xk):
        its[0] += 1
    x, info = spla.cg(A, b, rtol=rtol, atol=0.0, maxiter=10 * A.shape[0], callback=cb)
    return x, its[0]


@pytest.mark.parametrize("wl", [ph.small(2, (24, 24)), ph.small(3, (10, 9, 11))])
def test_empty_W_is_textbook_cg(wl):
    A = _operator(wl)
    b = np.random.default_rng(3).standard_normal(wl.n)
    tol = 1e-10
    res = kr.deflated_cg(A, b, np.zeros((wl.n, 0)), tol * np.linalg.norm(b), 10 * wl.n)
    xs = spla.spsolve(A.tocsc(), b)
    x_sc, its_sc = _scipy_cg_iterations(A, b, tol)
    assert abs(res.its - its_sc) <= 1
    assert np.linalg.norm(res.g - xs) <= 1e-7 * np.linalg.norm(xs)
    assert np.linalg.norm(b - A @ res.g) <= 1.01 * tol * np.linalg.norm(b)


def test_deflation_with_exact_eigenvectors():
    """W = exact low eigenvectors: the iteration is CG on the complementary invariant
    subspace, so it needs no more steps than CG on the deflated spectrum, and the
    residual stays orthogonal to W."""
    wl = ph.small(2, (20, 20))
    A = _operator(wl)
    Ad = A.toarray()
    lam, V = np.linalg.eigh(Ad)
    k = 8
    W = V[:, :k]
    b = np.random.default_rng(4).standard_normal(wl.n)
    tol = 1e-10
    res = kr.deflated_cg(A, b, W, tol * np.linalg.norm(b), 10 * wl.n)
    xs = np.linalg.solve(Ad, b)
    assert np.linalg.norm(res.g - xs) <= 1e-7 * np.linalg.norm(xs)
    s = b - A @ res.g
    assert np.abs(W.T @ s).max() <= 1e-12 * np.linalg.norm(b)
    # textbook CG on the complement-projected problem takes the same number of steps
    P = np.eye(wl.n) - W @ W.T
    bc = P @ b
    _, its_c = _scipy_cg_iterations(sp.csr_matrix(Ad), bc, tol * np.linalg.norm(b) / np.linalg.norm(bc))
    assert abs(res.its - its_c) <= 1
    # and fewer than undeflated CG
    _, its_full = _scipy_cg_iterations(A, b, tol)
    assert res.its < its_full


def test_deflated_cg_general_W_invariants():
    wl = ph.small(3, (8, 8, 8))
    A = _operator(wl)
    rng = np.random.default_rng(5)
    W = ph.smooth_modes(wl)
    b = rng.standard_normal(wl.n)
    tol = 1e-10
    res = kr.deflated_cg(A, b, W, tol * np.linalg.norm(b), 10 * wl.n)
    s = b - A @ res.g
    assert np.linalg.norm(s) <= 1.01 * tol * np.linalg.norm(b)
    # deflated CG keeps the residual orthogonal to W (Galerkin on range(W))
    assert np.abs(W.T @ s).max() <= 1e-9 * np.linalg.norm(b)
    # residual history non-increasing in the A^{-1}-norm is not guaranteed for ||s||,
    # but the error A-norm is: check the recorded residuals end below tol
    assert res.resid[-1] <= tol * np.linalg.norm(b)


def test_deflated_cg_catches_missing_projection():
    """Planted mistake: dropping the deflation term from the direction update leaves
    the method convergent but loses W^T s = 0; the invariant test must see it."""
    wl = ph.small(3, (8, 8, 8))
    A = _operator(wl)
    W = ph.smooth_modes(wl)
    b = np.random.default_rng(5).standard_normal(wl.n)
    tol = 1e-10
    # mutated copy: plain CG started from the Galerkin point of range(W)
    AW = A @ W
    GW = W.T @ AW
    y = np.linalg.solve(GW, W.T @ b)
    g = W @ y
    s = b - AW @ y
    p = s.copy()
    gam = s @ s
    for _ in range(5):
        w = A @ p
        al = gam / (p @ w)
        g += al * p
        s -= al * w
        gn = s @ s
        p = s + gn / gam * p
        gam = gn
    assert np.abs(W.T @ s).max() > 1e-6 * np.linalg.norm(b)


@pytest.mark.parametrize("wl", [ph.small(3, (12, 11, 10), n_src=2, n_det=2),
                                ph.small(3, (9, 10, 8), n_src=2, n_det=2, D="lognormal")])
def test_full_solve_matches_direct(wl):
    """The large-grid reference solve reaches the sparse LU solution to its tolerance:
    ||x - x_LU|| <= ||A^{-1}|| ||b - A x|| <= tol ||b|| / lambda_min."""
    from oracle import rom as orom
    As = op.assemble_Astar(wl.dim, wl.N, wl.bc, ph.diffusion_field(wl), wl.robin_A)
    p = ph.parameter_points(wl)[1]
    A = op.assemble_A(As, op.mu_field(wl.dim, wl.N, p.mu0, p.centers, p.radii, p.amps))
    lam = spla.eigsh(A, k=1, which="SA", return_eigenvectors=False)[0]
    rng = np.random.default_rng(5)
    for tol in (1e-6, 1e-12):
        b = np.zeros(wl.n)
        b[rng.integers(wl.n)] = 1.0
        x = orom.full_solve(A, b, tol)
        assert np.linalg.norm(b - A @ x) <= tol
        x_lu = spla.splu(sp.csc_matrix(A)).solve(b)
        assert np.linalg.norm(x - x_lu) <= 1.01 * tol / lam + 1e-15
