"""Pins for the reduced Jacobian (eq. (newjac)) and the bump-parameter derivatives it
uses: d mu / d p against central differences of mu itself; the full-order Jacobian
column against central differences of the full transfer function; the reduced column
against central differences of the reduced transfer function (any basis, any point);
and, at the sample points of a generated basis, the reduced columns equal the full ones
for every parameter (the interpolation theorem of the section on generating the ROM)."""
import numpy as np
import pytest

import phantoms as ph
from oracle import operator as op
from oracle import rom
from oracle import sequence as seq


def _params(rng, nb, dim):
    return (rng.uniform(0.3, 0.7, (nb, dim)), rng.uniform(0.2, 0.35, nb),
            rng.uniform(0.01, 0.03, nb))


def _perturbed(c, r, a, k, dim, h):
    c, r, a = c.copy(), r.copy(), a.copy()
    b, j = divmod(k, dim + 2)
    if j == 0:
        a[b] += h
    elif j == 1:
        r[b] += h
    else:
        c[b, j - 2] += h
    return c, r, a


def test_mu_gradient_matches_central_differences():
    rng = np.random.default_rng(11)
    for dim, N in ((2, (17, 13, 1)), (3, (9, 8, 7))):
        c, r, a = _params(rng, 3, dim)
        G = op.mu_gradient(dim, N, c, r, a)
        assert G.shape == (3 * (dim + 2), N[0] * N[1] * N[2])
        h = 1e-6
        for k in range(G.shape[0]):
            fp = op.mu_field(dim, N, 0.01, *_perturbed(c, r, a, k, dim, h))
            fm = op.mu_field(dim, N, 0.01, *_perturbed(c, r, a, k, dim, -h))
            fd = (fp - fm) / (2 * h)
            assert np.abs(fd - G[k]).max() <= 1e-6 * max(np.abs(G[k]).max(), 1e-3), k


def test_mu_gradient_catches_a_wrong_power():
    """A plausible slip (r instead of r^2 in the centre derivative) fails the same check."""
    rng = np.random.default_rng(12)
    dim, N = 2, (15, 15, 1)
    c, r, a = _params(rng, 1, dim)
    G = op.mu_gradient(dim, N, c, r, a)
    bad = G[2] * r[0]          # the centre derivative with one factor 1/r dropped
    h = 1e-6
    fd = (op.mu_field(dim, N, 0.01, *_perturbed(c, r, a, 2, dim, h))
          - op.mu_field(dim, N, 0.01, *_perturbed(c, r, a, 2, dim, -h))) / (2 * h)
    assert np.abs(fd - G[2]).max() <= 1e-6 * np.abs(G[2]).max()
    assert np.abs(fd - bad).max() > 1e-2 * np.abs(G[2]).max()


@pytest.fixture(scope="module")
def small2d():
    wl = ph.small(2, (14, 12), n_src=3, n_det=3, K=2, nb=2)
    D = ph.diffusion_field(wl)
    As = op.assemble_Astar(wl.dim, wl.N, wl.bc, D, wl.robin_A)
    si, di = ph.rhs_nodes(wl)
    ss, ds = ph.rhs_scales(wl)
    B = seq.rhs_matrix(wl.n, si, ss, di, ds)
    return wl, As, B


def _psi(As, B, ns, dim, N, c, r, a, V=None):
    A = op.assemble_A(As, op.mu_field(dim, N, 0.01, c, r, a))
    if V is None:
        return rom.full_transfer(A, B[:, :ns], B[:, ns:])
    return rom.reduced_transfer(*rom.reduced_matrices(V, A, B[:, :ns], B[:, ns:])[:3])


def test_full_jacobian_matches_central_differences(small2d):
    wl, As, B = small2d
    rng = np.random.default_rng(13)
    c, r, a = _params(rng, 2, wl.dim)
    A = op.assemble_A(As, op.mu_field(wl.dim, wl.N, 0.01, c, r, a))
    G = op.mu_gradient(wl.dim, wl.N, c, r, a)
    ns = wl.n_src
    h = 1e-5
    for k in range(G.shape[0]):
        J = rom.full_jacobian_column(A, B[:, :ns], B[:, ns:], G[k])
        fd = (_psi(As, B, ns, wl.dim, wl.N, *_perturbed(c, r, a, k, wl.dim, h))
              - _psi(As, B, ns, wl.dim, wl.N, *_perturbed(c, r, a, k, wl.dim, -h))) / (2 * h)
        assert np.abs(fd - J).max() <= 1e-5 * np.abs(J).max(), k


def test_reduced_jacobian_matches_central_differences(small2d):
    """Any basis, any point: the reduced column is the derivative of the reduced model."""
    wl, As, B = small2d
    rng = np.random.default_rng(14)
    V, _ = np.linalg.qr(rng.standard_normal((wl.n, 20)))
    c, r, a = _params(rng, 2, wl.dim)
    A = op.assemble_A(As, op.mu_field(wl.dim, wl.N, 0.01, c, r, a))
    G = op.mu_gradient(wl.dim, wl.N, c, r, a)
    ns = wl.n_src
    Ar, Br, Cr, _ = rom.reduced_matrices(V, A, B[:, :ns], B[:, ns:])
    h = 1e-5
    for k in range(G.shape[0]):
        Jr = rom.reduced_jacobian_column(V, Ar, Br, Cr, G[k])
        fd = (_psi(As, B, ns, wl.dim, wl.N, *_perturbed(c, r, a, k, wl.dim, h), V=V)
              - _psi(As, B, ns, wl.dim, wl.N, *_perturbed(c, r, a, k, wl.dim, -h), V=V)) / (2 * h)
        assert np.abs(fd - Jr).max() <= 1e-5 * np.abs(Jr).max(), k


def test_reduced_jacobian_equals_full_at_samples(small2d):
    """With the basis of Algorithm 2 (every solution for B~ and C~ at every p_i in
    range(V)), every reduced Jacobian column equals the full one at each p_i."""
    wl, As, B = small2d
    pts = ph.parameter_points(wl)
    mus = [op.mu_field(wl.dim, wl.N, p.mu0, p.centers, p.radii, p.amps) for p in pts]
    res = seq.solve_sequence(As, mus, B, ph.smooth_modes(wl), 1e-12, wl.trunc)
    V = res.Q
    ns = wl.n_src
    for p, mu in zip(pts, mus):
        A = op.assemble_A(As, mu)
        Ar, Br, Cr, _ = rom.reduced_matrices(V, A, B[:, :ns], B[:, ns:])
        G = op.mu_gradient(wl.dim, wl.N, p.centers, p.radii, p.amps)
        for k in range(G.shape[0]):
            J = rom.full_jacobian_column(A, B[:, :ns], B[:, ns:], G[k])
            Jr = rom.reduced_jacobian_column(V, Ar, Br, Cr, G[k])
            assert np.abs(Jr - J).max() <= 1e-6 * np.abs(J).max(), k
