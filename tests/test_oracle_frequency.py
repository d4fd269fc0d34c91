"""Pins for the nonzero-frequency oracle (eq. (solves) and the reduced transfer function of
eq. (newreduced)): the closed form of a constant-coefficient all-Dirichlet operator from
its sine eigenpairs; zero frequency against the zero-frequency transfer functions;
conjugate symmetry in sigma and complex symmetry for B = C; invariance of the reduced
response under a change of basis (which needs E_r = V^T V); Galerkin exactness and
Hermite interpolation in sigma when V spans the real and imaginary parts of the forward
and adjoint solutions at sigma; and the large-sigma expansion."""
import numpy as np

import phantoms as ph
from oracle import frequency as fq
from oracle import operator as op
from oracle import rom


def _problem(dim=2, N=(11, 9, 1), seed=3):
    wl = ph.small(dim, N[:dim], n_src=3, n_det=4, K=1, nb=2, D="lognormal")
    D = ph.diffusion_field(wl)
    As = op.assemble_Astar(wl.dim, wl.N, wl.bc, D, wl.robin_A)
    p = ph.parameter_points(wl)[0]
    A = op.assemble_A(As, op.mu_field(wl.dim, wl.N, p.mu0, p.centers, p.radii, p.amps))
    rng = np.random.default_rng(seed)
    n = A.shape[0]
    Bt = np.zeros((n, 3))
    Ct = np.zeros((n, 4))
    for j, i in enumerate(rng.choice(n, 3, replace=False)):
        Bt[i, j] = rng.uniform(0.5, 2.0)
    for j, i in enumerate(rng.choice(n, 4, replace=False)):
        Ct[i, j] = rng.uniform(0.5, 2.0)
    return A, Bt, Ct


def test_closed_form_sine_eigenbasis():
    # constant D, all-Dirichlet, constant mu0: A = sum_k lambda_k phi_k phi_k^T with
    # phi_(a,b)(i,j) = (2/(N+1)) sin(a pi (i+1) h) sin(b pi (j+1) h)
    Nx, Ny, D, mu0 = 9, 7, 0.05, 0.2
    As = op.assemble_Astar(2, (Nx, Ny, 1), (0,) * 6, D, 1.0)
    n = Nx * Ny
    A = op.assemble_A(As, np.full(n, mu0))
    hx, hy = 1.0 / (Nx + 1), 1.0 / (Ny + 1)
    ix, iy = np.arange(Nx), np.arange(Ny)
    rng = np.random.default_rng(5)
    Bt, Ct = rng.standard_normal((n, 2)), rng.standard_normal((n, 3))
    for sigma in (0.0, 0.7, 40.0, -3.0):
        ref = np.zeros((3, 2), dtype=complex)
        for a in range(1, Nx + 1):
            for b in range(1, Ny + 1):
                lam = (4 * D / hx ** 2 * np.sin(a * np.pi * hx / 2) ** 2
                       + 4 * D / hy ** 2 * np.sin(b * np.pi * hy / 2) ** 2 + mu0)
                phi = np.outer(np.sin(b * np.pi * (iy + 1) * hy),
                               np.sin(a * np.pi * (ix + 1) * hx)).reshape(-1)
                phi *= np.sqrt(2 * hx) * np.sqrt(2 * hy)
                ref += np.outer(Ct.T @ phi, Bt.T @ phi) / (lam + 1j * sigma)
        got = fq.full_response(A, Bt, Ct, sigma)
        np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def test_zero_frequency_and_symmetries():
    A, Bt, Ct = _problem()
    np.testing.assert_allclose(fq.full_response(A, Bt, Ct, 0.0), rom.full_transfer(A, Bt, Ct),
                               rtol=1e-12, atol=1e-15)
    V, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((A.shape[0], 20)))
    Ar, Br, Cr, _ = rom.reduced_matrices(V, A, Bt, Ct)
    np.testing.assert_allclose(fq.reduced_response(V, A, Bt, Ct, 0.0),
                               rom.reduced_transfer(Ar, Br, Cr), rtol=1e-11, atol=1e-15)
    for sigma in (0.3, 5.0):
        P, M = fq.full_response(A, Bt, Ct, sigma), fq.full_response(A, Bt, Ct, -sigma)
        np.testing.assert_allclose(M, np.conj(P), rtol=1e-12, atol=1e-15)
        assert np.abs(P.imag).max() > 1e-3 * np.abs(P).max()   # a genuinely complex response
        S = fq.full_response(A, Bt, Bt, sigma)
        np.testing.assert_allclose(S, S.T, rtol=1e-12, atol=1e-15)
        # a planted sign error (A - i sigma I) is caught by the symmetry in sigma
        assert np.abs(fq.full_response(A, Bt, Ct, -sigma) - P).max() > 1e-3 * np.abs(P).max()


def test_reduced_response_basis_invariance():
    A, Bt, Ct = _problem()
    rng = np.random.default_rng(2)
    V, _ = np.linalg.qr(rng.standard_normal((A.shape[0], 15)))
    S = rng.standard_normal((15, 15)) + 4 * np.eye(15)
    for sigma in (0.5, 8.0):
        a = fq.reduced_response(V, A, Bt, Ct, sigma)
        b = fq.reduced_response(V @ S, A, Bt, Ct, sigma)
        np.testing.assert_allclose(b, a, rtol=1e-9, atol=1e-12 * np.abs(a).max())
        # with E_r taken as I the skewed basis gives another (wrong) response
        W = V @ S
        Ar, Br, Cr = W.T @ (A @ W), W.T @ Bt, W.T @ Ct
        wrong = Cr.T @ np.linalg.solve(Ar + 1j * sigma * np.eye(15), Br)
        assert np.abs(wrong - a).max() > 1e-3 * np.abs(a).max()


def test_galerkin_exact_and_hermite_in_sigma():
    A, Bt, Ct = _problem(3, (7, 6, 5))
    sigma = 2.5
    X = fq.shifted_solve(A, np.hstack([Bt, Ct]), sigma)
    V, _ = np.linalg.qr(np.hstack([X.real, X.imag]))
    full = fq.full_response(A, Bt, Ct, sigma)
    red = fq.reduced_response(V, A, Bt, Ct, sigma)
    np.testing.assert_allclose(red, full, rtol=1e-10, atol=1e-12 * np.abs(full).max())
    # first derivative in sigma matches too (forward and adjoint solutions both in V)
    h = 1e-4
    dfull = (fq.full_response(A, Bt, Ct, sigma + h) - fq.full_response(A, Bt, Ct, sigma - h)) / (2 * h)
    dred = (fq.reduced_response(V, A, Bt, Ct, sigma + h)
            - fq.reduced_response(V, A, Bt, Ct, sigma - h)) / (2 * h)
    np.testing.assert_allclose(dred, dfull, rtol=1e-5, atol=1e-7 * np.abs(dfull).max())
    # away from sigma the reduced response is an approximation, not the full one
    far = 40.0
    err = np.abs(fq.reduced_response(V, A, Bt, Ct, far) - fq.full_response(A, Bt, Ct, far)).max()
    assert err > 1e-8 * np.abs(fq.full_response(A, Bt, Ct, far)).max()


def test_large_sigma_expansion():
    A, Bt, Ct = _problem()
    rng = np.random.default_rng(4)
    Bd, Cd = rng.standard_normal(Bt.shape), rng.standard_normal(Ct.shape)
    sigma = 1e4
    s = 1j * sigma
    approx = Cd.T @ Bd / s - Cd.T @ (A @ Bd) / s ** 2
    got = fq.full_response(A, Bd, Cd, sigma)
    third = np.abs(Cd.T @ (A @ (A @ Bd))).max() / sigma ** 3
    assert np.abs(got - approx).max() <= 2 * third
