"""GPU parity of the lowest eigenpairs of A(p) (rom_lowest_modes, the U_0 of Algorithm 2,
Sec. 4.2.2) against the oracle's dense eigendecomposition.

Bounds used (A symmetric, each returned pair (theta_i, u_i) with residual r_i):
  - every theta_i lies within ||r_i|| of an eigenvalue, and Rayleigh-Ritz values sit above
    the matching eigenvalue (Courant-Fischer), so |theta_i - lambda_i| <= ||r_i|| once the
    pairs are ordered; the iteration stops at ||r_i|| <= tol * b (b: Gershgorin bound);
  - the largest sine of the principal angles between range(U) and the oracle's eigenvectors,
    ||(I - V V^T) U||_2, is at most ||R||_F / gap (Davis-Kahan), gap = lambda_k -
    theta_{k-1}, checked at twice that;
  - orthonormality of U to 1e-12 (Cholesky QR twice).
A degenerate spectrum (constant coefficients, all-Dirichlet square) checks a double
eigenvalue against the closed form and its 2D invariant subspace rather than vectors."""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem, principal_cosines
from oracle import modes
from oracle import operator as op

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def drv(gpu):
    from paper_1602_00138_amd import driver
    return driver


def _check_pairs(A, U, lam, k, tol):
    b = modes.gershgorin_upper(A)
    lam_ref, V_ref = modes.lowest_modes(A, k + 1)
    assert U.shape == (A.shape[0], k)
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-12
    assert np.all(np.diff(lam) >= -1e-12 * b)
    R = A @ U - U * lam
    res = np.linalg.norm(R, axis=0)
    assert res.max() <= tol * b * (1 + 1e-6), res.max() / b
    np.testing.assert_allclose(lam, lam_ref[:k], rtol=0, atol=res.max() + 1e-12 * b)
    gap = lam_ref[k] - lam[k - 1]
    if gap > 1e-6 * b:
        # largest sine = ||(I - V V^T) U||_2 (accurate where 1 - cos^2 would cancel)
        Vk = V_ref[:, :k]
        sine = np.linalg.norm(U - Vk @ (Vk.T @ U), 2)
        assert sine <= 2 * np.linalg.norm(R) / gap + 1e-12
    return res


@pytest.mark.parametrize("wl,k,kx", [
    (ph.small(2, (17, 13), K=2, nb=2), 8, 12),
    (ph.small(3, (11, 10, 9), K=2, nb=3, D="lognormal"), 10, 16),
    (ph.small(3, (9, 8, 7), K=2, nb=2, D="lognormal"), 24, 32),    # the largest block
    (ph.small(2, (12, 11), K=2, nb=1), 1, 4),
    (ph.small(3, (12, 10, 9), K=2, nb=2, D="lognormal"), 10, 16),   # even nx: two-node filter
])
def test_lowest_modes_parity(drv, wl, k, kx):
    orc = OracleProblem(wl)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    X0 = np.ascontiguousarray(ph.smooth_modes(wl, kx).T)
    tol = 1e-9
    for i, p in enumerate(pts):
        U, lam, sweeps = prob.lowest_modes(p, k, torch_from(X0), tol=tol, maxit=400)
        assert 1 <= sweeps < 400
        _check_pairs(orc.A(i), U.cpu().numpy().T, lam, k, tol)


def test_lowest_modes_degenerate_closed_form(drv):
    """Constant D, all-Dirichlet 15 x 15: lambda_(a,b) = 4D/h^2 (sin^2(a pi h/2) +
    sin^2(b pi h/2)); (1,2) and (2,1) form a double eigenvalue, as do (1,3)/(3,1)."""
    from paper_1602_00138_amd import driver
    wl = ph.small(2, (15, 15), K=1, nb=1)
    D, n = 0.04, 15
    s, d = ph.rhs_nodes(wl)
    ss, ds = ph.rhs_scales(wl)
    prob = driver.Problem(2, wl.N, (0,) * 6, 1.0, D, s, ss, d, ds, ph.smooth_modes(wl, 4))
    from paper_1602_00138_amd import rom as R
    p = R.MuParams(0.0, np.array([[0.5, 0.5]]), np.array([0.1]), np.array([0.0]))
    k = 6
    X0 = np.random.default_rng(11).standard_normal((10, n * n))
    U, lam, _ = prob.lowest_modes(p, k, torch_from(X0), tol=1e-10, maxit=600)
    h = 1.0 / (n + 1)
    one = 4 * D / h ** 2 * np.sin(np.arange(1, n + 1) * np.pi * h / 2) ** 2
    ref = np.sort(np.add.outer(one, one).reshape(-1))[:k]
    b = 8 * D / h ** 2 * 2
    np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-9 * b)
    A = op.assemble_A(op.assemble_Astar(2, wl.N, (0,) * 6, D, 1.0), np.zeros(n * n))
    U = U.cpu().numpy().T
    lam_ref, V_ref = modes.lowest_modes(A, 7)
    # the double eigenvalue's subspace: columns 1..2 span the same plane as the oracle's
    cos = principal_cosines(U[:, 1:3], V_ref[:, 1:3])
    assert cos.min() >= 1 - 1e-12


def test_lowest_modes_errors(drv):
    from paper_1602_00138_amd import rom as R
    wl = ph.small(2, (9, 8), K=1, nb=1)
    prob = drv.problem_from_workload(wl)
    p = drv.points_from_workload(wl)[0]
    X0 = torch_from(np.ascontiguousarray(ph.smooth_modes(wl, 8).T))
    for k in (0, 9):
        with pytest.raises(R.RomError):
            prob.lowest_modes(p, k, X0)
    with pytest.raises(R.RomError):
        prob.lowest_modes(p, 4, torch_from(np.zeros((33, wl.n))))
    with pytest.raises(R.RomError):
        R.rom_lowest_modes_bytes(prob.op, 33)
    # maxit reached: ENOCONV after exactly maxit sweeps, with a valid block
    with pytest.raises(R.RomError) as e:
        prob.lowest_modes(p, 4, X0, tol=1e-30, maxit=3)
    assert e.value.status == R.ROM_ENOCONV
    U, lam, sweeps, st = prob.lowest_modes(p, 4, X0, tol=1e-30, maxit=3, allow_noconv=True)
    assert sweeps == 3 and st == R.ROM_ENOCONV
    Uh = U.cpu().numpy().T
    assert np.abs(Uh.T @ Uh - np.eye(4)).max() <= 1e-12


def torch_from(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float64))


def test_sequence_seeded_with_computed_modes(drv):
    """U_0 of Algorithm 2 from rom_lowest_modes (the eigenvectors of A(p_0) the paper takes
    offline) instead of the analytic smooth modes: the sequence passes the parity gates
    against the oracle run on its own dense eigenvectors of A(p_0) (the two U_0 span the
    same invariant subspace to the eigen-residual 1e-9 b), and both seeds' iteration
    counts are reported."""
    import torch
    from oracle import sequence as oseq
    from test_gpu_parity import _check_sequence
    wl = ph.small(3, (13, 11, 10), n_src=4, n_det=4, K=3, D="lognormal")
    orc = OracleProblem(wl)
    lam_ref, V_ref = modes.lowest_modes(orc.A(0), 11)
    assert lam_ref[10] - lam_ref[9] > 1e-3 * lam_ref[9]     # U_0 is well defined
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    X0 = torch.from_numpy(np.ascontiguousarray(ph.smooth_modes(wl, 16).T))
    U, lam, sweeps = prob.lowest_modes(pts[0], 10, X0, tol=1e-9, maxit=400)
    analytic = prob.solve(pts, wl.tol, wl.trunc, keep_X=False)
    prob.set_U0(U)
    res = prob.solve(pts, wl.tol, wl.trunc)
    ores = oseq.solve_sequence(orc.As, orc.mus, orc.B, V_ref[:, :10], wl.tol, wl.trunc)
    _check_sequence(wl, orc, ores, res, prob, pts)
    its = lambda r: sum(x["its"] for x in r.records)
    print(f"\nU_0 from {sweeps} filter sweeps: iterations with eigenvectors {its(res)} "
          f"(oracle {sum(r.its for r in ores.records)}), with the analytic modes {its(analytic)}")
    res.close()
    analytic.close()
    prob.close()
