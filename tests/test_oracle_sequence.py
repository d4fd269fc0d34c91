"""Pins for the oracle's Algorithm 2 (CG form) and the reduced model (eq. (newreduced))."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import phantoms as ph
from oracle import operator as op
from oracle import rom
from oracle import sequence as seq


def _setup(wl, mode="independent"):
    D = ph.diffusion_field(wl)
    As = op.assemble_Astar(wl.dim, wl.N, wl.bc, D, wl.robin_A)
    pts = ph.parameter_points(wl, mode=mode)
    mus = [op.mu_field(wl.dim, wl.N, p.mu0, p.centers, p.radii, p.amps) for p in pts]
    si, di = ph.rhs_nodes(wl)
    ss, ds = ph.rhs_scales(wl)
    B = seq.rhs_matrix(wl.n, si, ss, di, ds)
    U0 = ph.smooth_modes(wl)
    return As, mus, B, U0


@pytest.fixture(scope="module")
def slab2d_32():
    wl = ph.WORKLOADS["slab2d_32"]
    As, mus, B, U0 = _setup(wl)
    res = seq.solve_sequence(As, mus, B, U0, wl.tol, wl.trunc)
    return wl, As, mus, B, U0, res


def test_slab2d_32_solutions_match_dense_cholesky(slab2d_32):
    wl, As, mus, B, U0, res = slab2d_32
    for i, mu in enumerate(mus):
        Ad = As.toarray() + np.diag(mu)
        Xc = sla.cho_solve(sla.cho_factor(Ad), B)
        err = np.linalg.norm(res.X[i] - Xc, axis=0) / np.linalg.norm(Xc, axis=0)
        assert err.max() < 1e-7
        # entrywise positive (Stieltjes inverse applied to non-negative columns)
        assert (Xc > 0).all()


def test_slab2d_32_invariants(slab2d_32):
    wl, As, mus, B, U0, res = slab2d_32
    Q = res.Q
    m = Q.shape[1]
    assert np.abs(Q.T @ Q - np.eye(m)).max() < 1e-12
    kept = sum(r.kept for r in res.records)
    assert m == res.k_u + kept
    for i in range(len(mus)):
        assert sum(r.kept for r in res.records if r.point == i) <= B.shape[1]
    for r in res.records:
        assert r.final_res <= wl.tol * (1 + 1e-9)
        assert r.its == 0 or r.solved
    # every solution lies in range(Q) (x0 in range(Q), correction appended)
    for Xi in res.X:
        P = Q @ (Q.T @ Xi)
        assert np.linalg.norm(Xi - P) <= 1e-9 * np.linalg.norm(Xi)


def test_slab2d_32_reciprocity(slab2d_32):
    """B^T X_i is symmetric (A_i symmetric): forward and adjoint halves agree."""
    wl, As, mus, B, U0, res = slab2d_32
    for Xi in res.X:
        S = B.T @ Xi
        assert np.abs(S - S.T).max() <= 1e-8 * np.abs(S).max()


def test_interpolation_theorem(slab2d_32):
    """Theorem of Sec. 3.4: with A(p_i)^{-1}B and (C A(p_i)^{-1})^T in range(V) the
    reduced transfer function and its gradient match the full ones at p_i."""
    wl, As, mus, B, U0, res = slab2d_32
    ns = wl.n_src
    Bt, Ct = B[:, :ns], B[:, ns:]
    Q = res.Q
    pts = ph.parameter_points(wl)
    for i, mu in enumerate(mus):
        A = op.assemble_A(As, mu)
        psi = rom.full_transfer(A, Bt, Ct)
        Ar, Br, Cr, Er = rom.reduced_matrices(Q, A, Bt, Ct)
        psir = rom.reduced_transfer(Ar, Br, Cr)
        assert np.abs(psir - psi).max() <= 1e-8 * np.abs(psi).max()
        np.testing.assert_allclose(Er, np.eye(Q.shape[1]), atol=1e-12)
        assert np.abs(Ar - Ar.T).max() <= 1e-12 * np.abs(Ar).max()
        # gradient w.r.t. the amplitude of bump 0 (d mu / d a_0 = psi(|x-c|/r))
        X = op.node_coords(wl.dim, wl.N)
        p = pts[i]
        dmu = op.wendland(np.sqrt(((X - p.centers[0]) ** 2).sum(1)) / p.radii[0])
        J = rom.full_jacobian_column(A, Bt, Ct, dmu)
        Jr = rom.reduced_jacobian_column(Q, Ar, Br, Cr, dmu)
        assert np.abs(Jr - J).max() <= 1e-6 * np.abs(J).max()


def test_reduced_transfer_rotation_invariant(slab2d_32):
    wl, As, mus, B, U0, res = slab2d_32
    ns = wl.n_src
    Q = res.Q
    O, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((Q.shape[1],) * 2))
    mu = op.mu_field(wl.dim, wl.N, 0.01, [[0.4, 0.6]], [0.2], [0.02])   # off the samples
    A = op.assemble_A(As, mu)
    a = rom.reduced_transfer(*rom.reduced_matrices(Q, A, B[:, :ns], B[:, ns:])[:3])
    b = rom.reduced_transfer(*rom.reduced_matrices(Q @ O, A, B[:, :ns], B[:, ns:])[:3])
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_transfer_monotone_in_absorption():
    """Stieltjes operator: more absorption -> entrywise smaller transfer function."""
    wl = ph.small(2, (14, 14))
    D = ph.diffusion_field(wl)
    As = op.assemble_Astar(wl.dim, wl.N, wl.bc, D, wl.robin_A)
    si, di = ph.rhs_nodes(wl)
    B = seq.rhs_matrix(wl.n, si, np.ones(4), di, np.ones(4))
    c = [[0.5, 0.5]]
    p1 = rom.full_transfer(op.assemble_A(As, op.mu_field(2, wl.N, 0.01, c, [0.2], [0.01])), B[:, :4], B[:, 4:])
    p2 = rom.full_transfer(op.assemble_A(As, op.mu_field(2, wl.N, 0.01, c, [0.2], [0.03])), B[:, :4], B[:, 4:])
    assert (p2 < p1).all()


def test_no_recycling_special_case():
    """No U_0, one point: every right-hand side starts from the Galerkin point of the
    basis built so far; the first one is textbook CG from zero."""
    wl = ph.small(2, (16, 16), n_src=3, n_det=3, K=1)
    As, mus, B, _ = _setup(wl)
    res = seq.solve_sequence(As, mus, B, np.zeros((wl.n, 0)), 1e-10)
    A = op.assemble_A(As, mus[0])
    its = [0]

    def cb(xk):
        its[0] += 1
    spla.cg(A, B[:, 0], rtol=1e-10, atol=0.0, maxiter=10000, callback=cb)
    assert abs(res.records[0].its - its[0]) <= 1
    assert res.k_u == 0


def test_drift_mode_and_truncation_cap():
    wl = ph.small(3, (8, 8, 8), n_src=4, n_det=4, K=4, tol=1e-8)
    As, mus, B, U0 = _setup(wl, mode="drift")
    res = seq.solve_sequence(As, mus, B, U0, wl.tol, 1e-8, cap=20)
    assert res.Q.shape[1] <= 20
    for r in res.records:
        assert r.final_res <= wl.tol * (1 + 1e-9)
    dropped_by_cap = [r for r in res.records if r.solved and not r.kept and r.rho > 1e-8]
    assert len(dropped_by_cap) > 0


def test_skip_when_in_basis():
    """A right-hand side whose solution is already in range(V) needs no iteration:
    repeating a point reproduces rho0 <= tol for every column."""
    wl = ph.small(2, (12, 12), n_src=3, n_det=3, K=1, tol=1e-10)
    As, mus, B, U0 = _setup(wl)
    res = seq.solve_sequence(As, [mus[0], mus[0]], B, U0, 1e-10)
    second = [r for r in res.records if r.point == 1]
    assert all(r.its == 0 and not r.solved for r in second)
    assert all(r.rho0 <= 1e-10 for r in second)


@pytest.mark.parametrize("group", [3, 16])
def test_grouped_sequence_invariants(slab2d_32, group):
    """The batched reading (RHS in groups sharing one projection): every solution still
    meets the dense Cholesky solution, the basis stays orthonormal and contains every
    solution, so the reduced transfer function interpolates at every sample point."""
    wl, As, mus, B, U0, res1 = slab2d_32
    res = seq.solve_sequence(As, mus, B, U0, wl.tol, wl.trunc, group=group)
    Q = res.Q
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-12
    assert Q.shape[1] == res.k_u + sum(r.kept for r in res.records)
    assert [(r.point, r.rhs) for r in res.records] == [(r.point, r.rhs) for r in res1.records]
    ns = wl.n_src
    for i, mu in enumerate(mus):
        Ad = As.toarray() + np.diag(mu)
        Xc = sla.cho_solve(sla.cho_factor(Ad), B)
        err = np.linalg.norm(res.X[i] - Xc, axis=0) / np.linalg.norm(Xc, axis=0)
        assert err.max() < 1e-7
        assert np.linalg.norm(res.X[i] - Q @ (Q.T @ res.X[i])) <= 1e-9 * np.linalg.norm(res.X[i])
        A = op.assemble_A(As, mu)
        Ar, Br, Cr, _ = rom.reduced_matrices(Q, A, B[:, :ns], B[:, ns:])
        psi = B[:, ns:].T @ Xc[:, :ns]
        assert np.abs(rom.reduced_transfer(Ar, Br, Cr) - psi).max() <= 1e-9 * np.abs(psi).max()
    # members of a group see the basis of the group start: with one group per point,
    # every right-hand side at p_0 is projected on orth(U_0) alone
    resall = seq.solve_sequence(As, mus[:1], B, U0, wl.tol, wl.trunc, group=B.shape[1])
    A0 = op.assemble_A(As, mus[0])
    U, _ = np.linalg.qr(U0)
    for r in resall.records:
        b = B[:, r.rhs]
        c = np.linalg.solve(U.T @ (A0 @ U), U.T @ b)
        assert abs(r.rho0 - np.linalg.norm(b - A0 @ (U @ c)) / np.linalg.norm(b)) <= 1e-12


def test_group_one_is_the_sequential_order(slab2d_32):
    wl, As, mus, B, U0, res1 = slab2d_32
    res = seq.solve_sequence(As, mus[:2], B, U0, wl.tol, wl.trunc, group=1)
    for a, b in zip(res.records, res1.records):
        assert (a.point, a.rhs, a.its, a.kept, a.m) == (b.point, b.rhs, b.its, b.kept, b.m)


def test_uj_cap_bounds_recycle_spaces(slab2d_32):
    """uj_cap: U_j never holds more than uj_cap columns (k_u + extra corrections), every
    solution still meets tol, V is unchanged by the cap (the cap only limits the recycle
    spaces), and uj_cap=None or a cap above every U_j reproduces the unbounded sequence."""
    wl, As, mus, B, U0, res = slab2d_32
    k_u = res.k_u
    widest = max(len(w) for w in res.W_extra)
    assert widest >= 2
    same = seq.solve_sequence(As, mus, B, U0, wl.tol, wl.trunc, uj_cap=k_u + widest)
    assert [r.its for r in same.records] == [r.its for r in res.records]
    assert np.array_equal(same.Q, res.Q)
    capped = seq.solve_sequence(As, mus, B, U0, wl.tol, wl.trunc, uj_cap=k_u + 1)
    assert max(len(w) for w in capped.W_extra) == 1
    for r in capped.records:
        assert r.final_res <= wl.tol * (1 + 1e-9)
    none = seq.solve_sequence(As, mus, B, U0, wl.tol, wl.trunc, uj_cap=k_u)
    assert all(len(w) == 0 for w in none.W_extra)
    # the recycle space only changes the inner solves, never what V must represent:
    # every capped run's solutions lie in range(V)
    for run in (capped, none):
        for Xi in run.X:
            P = run.Q @ (run.Q.T @ Xi)
            assert np.linalg.norm(Xi - P) <= 1e-9 * np.linalg.norm(Xi)
