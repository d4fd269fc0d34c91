"""Pins for the oracle's operator assembly (paper Sec. 3, eq. (block1), eq. (sum))."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import phantoms as ph
from oracle import operator as op

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_fixture(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(x) for x in line.split()])
    return rows


def test_golden_2x2_robin():
    rows = _read_fixture("stencil_2d_2x2_robin_y.txt")
    dim, n0, n1, D, A = rows[0]
    M = np.array(rows[1:])
    bc = ph.face_kinds(2)
    As = op.assemble_Astar(2, (int(n0), int(n1), 1), bc, D, A).toarray()
    np.testing.assert_allclose(As, M, rtol=0, atol=1e-13)


def test_golden_varD_harmonic():
    rows = _read_fixture("stencil_2d_1x3_varD.txt")
    dim, n0, n1, A = rows[0]
    Dv = np.array(rows[1])
    M = np.array(rows[2:])
    bc = ph.face_kinds(2)
    As = op.assemble_Astar(2, (int(n0), int(n1), 1), bc, Dv, A).toarray()
    np.testing.assert_allclose(As, M, rtol=0, atol=1e-12)


def _schur_pin(assemble, dim, N, D, A, seed=0):
    """The assembled operator equals the Schur complement of eq. (block1) and the
    transfer function C1^T M^{-1} B1 of the full system equals C~^T A~^{-1} B~."""
    bc = ph.face_kinds(dim)
    n = N[0] * N[1] * N[2]
    rng = np.random.default_rng(seed)
    mu = 0.01 + 0.05 * rng.random(n)
    M, nb, bnd_of = op.full_boundary_system(dim, N, bc, D, A, mu)
    G = M[:nb, :nb]
    D1 = M[:nb, nb:]
    D2 = M[nb:, :nb]
    F = M[nb:, nb:]
    assert np.count_nonzero(G - np.diag(np.diag(G))) == 0          # G diagonal
    assert (np.count_nonzero(D1, axis=1) <= 1).all()                 # <= 1 nnz per row
    assert ((D2 != 0) == (D1.T != 0)).all()                          # pattern of D1^T
    S = F - D2 @ np.diag(1.0 / np.diag(G)) @ D1
    At = assemble(dim, N, bc, D, A).toarray() + np.diag(mu)
    err_S = np.abs(S - At).max() / np.abs(At).max()
    # sources on the low Robin face, detectors on the high one (not co-located)
    lo_face = [s for (k, f), s in bnd_of.items() if f == 2 * (dim - 1)]
    hi_face = [s for (k, f), s in bnd_of.items() if f == 2 * (dim - 1) + 1]
    src = lo_face[:: max(1, len(lo_face) // 3)][:3]
    det = hi_face[:: max(1, len(hi_face) // 3)][:3]
    B1 = np.zeros((nb + n, len(src)))
    C1 = np.zeros((nb + n, len(det)))
    B1[src, np.arange(len(src))] = 1.0
    C1[det, np.arange(len(det))] = 1.0
    assert np.abs(C1.T @ B1).max() == 0.0
    psi_full = C1.T @ np.linalg.solve(M, B1)
    Bt = D2 @ np.diag(1.0 / np.diag(G)) @ B1[:nb]
    Ct = (C1[:nb].T @ np.diag(1.0 / np.diag(G)) @ D1).T
    # effective sources/receivers are scaled identity columns (Sec. 3.1)
    assert (np.count_nonzero(Bt, axis=0) == 1).all() and (np.count_nonzero(Ct, axis=0) == 1).all()
    psi_schur = Ct.T @ np.linalg.solve(At, Bt)
    err_psi = np.abs(psi_full - psi_schur).max() / np.abs(psi_full).max()
    return err_S, err_psi


@pytest.mark.parametrize("dim,N,D", [(2, (6, 5, 1), 0.03), (2, (4, 7, 1), "var"),
                                     (3, (4, 3, 5), 0.03), (3, (3, 4, 4), "var")])
def test_schur_identity(dim, N, D):
    n = N[0] * N[1] * N[2]
    if D == "var":
        D = 0.03 * np.exp(0.3 * np.random.default_rng(3).standard_normal(n))
    err_S, err_psi = _schur_pin(op.assemble_Astar, dim, N, D, 0.7)
    assert err_S < 1e-13
    assert err_psi < 1e-11


def test_schur_pin_catches_dirichlet_robin_mixup():
    """Planted mistake: treating the Robin face like a Dirichlet one must fail the pin."""
    def wrong(dim, N, bc, D, A):
        return op.assemble_Astar(dim, N, (0,) * 6, D, A)
    err_S, err_psi = _schur_pin(wrong, 2, (5, 5, 1), 0.03, 1.0)
    assert err_S > 1e-3 and err_psi > 1e-3


def test_schur_pin_catches_missing_beta():
    """Planted mistake: dropping the Robin diagonal correction altogether."""
    def wrong(dim, N, bc, D, A):
        # beta -> 0 is what a very large Robin constant produces
        return op.assemble_Astar(dim, N, bc, D, 1e12)
    err_S, err_psi = _schur_pin(wrong, 3, (3, 3, 4), 0.03, 1.0)
    assert err_S > 1e-3 and err_psi > 1e-3


@pytest.mark.parametrize("dim,N", [(2, (7, 5, 1)), (3, (4, 5, 3))])
def test_dirichlet_closed_form_spectrum(dim, N):
    """All-Dirichlet, constant D: eigenvalues are sums of 4 D/h^2 sin^2(k pi / (2(N+1)))."""
    D = 0.05
    As = op.assemble_Astar(dim, N, (0,) * 6, D, 1.0).toarray()
    lam = np.linalg.eigvalsh(As)
    axes = []
    for a in range(dim):
        h = 1.0 / (N[a] + 1)
        k = np.arange(1, N[a] + 1)
        axes.append(4 * D / h ** 2 * np.sin(k * np.pi / (2 * (N[a] + 1))) ** 2)
    ref = axes[0]
    for a in range(1, dim):
        ref = np.add.outer(axes[a], ref).reshape(-1)
    np.testing.assert_allclose(np.sort(lam), np.sort(ref), rtol=1e-12)


def test_dirichlet_closed_form_eigenvector():
    """The discrete sine product is an exact eigenvector (pins the index strides)."""
    N = (5, 4, 3)
    D = 0.02
    As = op.assemble_Astar(3, N, (0,) * 6, D, 1.0)
    ks = (2, 1, 3)
    v = np.ones(1)
    lam = 0.0
    for a in range(3):
        i = np.arange(N[a]) + 1
        va = np.sin(ks[a] * np.pi * i / (N[a] + 1))
        v = np.multiply.outer(va, v) if a else va
        h = 1.0 / (N[a] + 1)
        lam += 4 * D / h ** 2 * np.sin(ks[a] * np.pi / (2 * (N[a] + 1))) ** 2
    v = v.reshape(-1)
    np.testing.assert_allclose(As @ v, lam * v, atol=1e-12 * lam)


@pytest.mark.parametrize("wl", [ph.small(2, (9, 8)), ph.small(3, (5, 6, 4), D="lognormal")])
def test_spd_stieltjes(wl):
    D = ph.diffusion_field(wl)
    As = op.assemble_Astar(wl.dim, wl.N, wl.bc, D, wl.robin_A)
    Ad = As.toarray()
    assert np.array_equal(Ad, Ad.T)
    off = Ad - np.diag(np.diag(Ad))
    assert (off <= 0).all() and (np.diag(Ad) > 0).all()
    # weakly diagonally dominant with strict rows at the boundary -> SPD
    assert (np.diag(Ad) + off.sum(axis=1) >= -1e-12).all()
    assert np.linalg.eigvalsh(Ad).min() > 0
    # Stieltjes => entrywise positive inverse (irreducible)
    assert (np.linalg.inv(Ad) > 0).all()


def test_constant_field_equals_scalar_D():
    wl = ph.small(3, (4, 5, 6))
    a = op.assemble_Astar(3, wl.N, wl.bc, 0.03, 1.0).toarray()
    b = op.assemble_Astar(3, wl.N, wl.bc, np.full(wl.n, 0.03), 1.0).toarray()
    np.testing.assert_allclose(a, b, rtol=1e-14)


def test_wendland_closed_form():
    t = np.array([0.0, 0.25, 0.5, 0.75, 1.0, 1.5])
    ref = np.array([1.0, 0.75 ** 4 * 2.0, 0.5 ** 4 * 3.0, 0.25 ** 4 * 4.0, 0.0, 0.0])
    np.testing.assert_allclose(op.wendland(t), ref, rtol=1e-15)
    # C2 at the support edge: value, slope and curvature vanish at t = 1
    eps = 1e-4
    f = op.wendland(np.array([1 - 2 * eps, 1 - eps, 1.0]))
    assert abs(f[2]) == 0 and abs(f[1]) < 1e-14 and abs(f[0]) < 1e-13


def test_mu_field_bumps():
    wl = ph.small(2, (19, 19))
    c = np.array([[0.5, 0.5]])
    mu = op.mu_field(2, wl.N, 0.01, c, np.array([0.2]), np.array([0.03]))
    X = op.node_coords(2, wl.N)
    k = np.argmin(((X - c) ** 2).sum(1))
    assert abs(mu[k] - 0.04) < 1e-15                      # centre node sits at (0.5, 0.5)
    far = np.sqrt(((X - c) ** 2).sum(1)) >= 0.2
    assert np.all(mu[far] == 0.01)
    assert np.all(mu >= 0.01)
    # radial: equal distance -> equal value
    d = np.round(np.sqrt(((X - c) ** 2).sum(1)), 12)
    for val in np.unique(d)[:6]:
        assert np.ptp(mu[d == val]) < 1e-15


def test_generator_shapes():
    wl = ph.WORKLOADS["cube64"]
    s, d = ph.rhs_nodes(wl)
    assert s.shape == (32,) and d.shape == (32,)
    N = wl.N
    assert np.all(s // (N[0] * N[1]) == 0) and np.all(d // (N[0] * N[1]) == N[2] - 1)
    assert len(set(s.tolist())) == 32 and len(set(d.tolist())) == 32
    wl1 = ph.WORKLOADS["slab2d_32"]
    s1, d1 = ph.rhs_nodes(wl1)
    assert np.all(s1 // 32 == 31) and np.all(d1 // 32 == 0)
    U0 = ph.smooth_modes(ph.small(3, (10, 11, 12)))
    assert U0.shape == (1320, 10)
    np.testing.assert_allclose(np.linalg.norm(U0, axis=0), 1.0)
    pts = ph.parameter_points(wl)
    assert len(pts) == 16 and pts[0].centers.shape == (8, 3)
    pts2 = ph.parameter_points(wl)
    np.testing.assert_array_equal(pts[5].radii, pts2[5].radii)
