"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Tolerances (stated per check): the stencil product agrees to rounding (1e-14
relative); solutions to 1e-7 relative and reduced transfer-function entries to
1e-6 relative at solver tolerance 1e-10; CG iteration counts within 2 and the
skip/append decisions equal wherever the oracle's decision is not within 1% of
its threshold; bases equal as subspaces (principal-angle cosines >= 1 - 1e-8).
"""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem, principal_cosines
from oracle import rom as orom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def drv(gpu):
    from paper_1602_00138_amd import driver
    return driver


def _gpu_run(drv, wl, K=None, mode="independent", k_u=None, **kw):
    prob = drv.problem_from_workload(wl, k_u=k_u)
    pts = drv.points_from_workload(wl, K=K, mode=mode)
    res = prob.solve(pts, kw.pop("tol", wl.tol), kw.pop("trunc", wl.trunc), **kw)
    return prob, pts, res


# odd nx: one node per thread; even nx: the two-node SpMM (16-byte loads and stores,
# two or four columns per thread)
@pytest.mark.parametrize("wl", [ph.small(2, (17, 13)), ph.small(3, (9, 8, 7)),
                                ph.small(3, (11, 6, 9), D="lognormal"),
                                ph.small(2, (18, 13)), ph.small(2, (16, 11), D="lognormal"),
                                ph.small(3, (10, 8, 7)), ph.small(3, (12, 6, 9), D="lognormal")])
def test_apply_operator_matches_oracle(drv, wl):
    import torch
    orc = OracleProblem(wl)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    rng = np.random.default_rng(0)
    # 1, 3 and 9 columns: single columns, and full and partial groups of the SpMM's
    # columns-per-thread grouping
    for k in (1, 3, 9):
        X = rng.standard_normal((k, wl.n))
        Y = prob.apply(pts[1], torch.as_tensor(X, device="cuda")).cpu().numpy()
        ref = (orc.A(1) @ X.T).T
        assert np.abs(Y - ref).max() <= 1e-14 * np.abs(ref).max(), k
    prob.close()


def _check_sequence(wl, orc, ores, res, prob, pts, sol_tol=1e-7, psi_tol=1e-6, interpolates=True,
                    trunc=None):
    """interpolates: every solution lies in range(V) (no cap), so the reduced transfer
    function equals the full one at the sample points (Theorem of Sec. 3.4).  A skip
    decision within 1% of tol, or a keep decision within rounding (1e-6) of trunc, may
    differ."""
    n_rhs = wl.n_rhs
    trunc = wl.trunc if trunc is None else trunc
    # decisions and counts
    assert len(res.records) == len(ores.records)
    for g, o in zip(res.records, ores.records):
        near = abs(o.rho0 - wl.tol) < 0.01 * wl.tol
        if not near:
            assert bool(g["solved"]) == o.solved, (g, o)
        assert abs(g["rho0"] - o.rho0) <= 1e-3 * o.rho0 + 1e-12, (g, o)
        if g["solved"] and o.solved and not near:
            assert abs(g["its"] - o.its) <= 2, (g, o)
            if not abs(g["rho"] - trunc) < 1e-6 * trunc:
                assert bool(g["kept"]) == o.kept, (g, o)
        assert g["converged"] and g["final_res"] <= wl.tol * (1 + 1e-6)
    assert res.m == ores.Q.shape[1]
    # solutions against direct solves
    X = res.X.cpu().numpy()
    for i in range(len(pts)):
        Xd = np.linalg.solve(orc.A(i).toarray(), orc.B) if wl.n <= 4096 else None
        Xi = X[i * n_rhs:(i + 1) * n_rhs].T
        ref = Xd if Xd is not None else ores.X[i]
        err = np.linalg.norm(Xi - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert err.max() <= sol_tol, (i, err.max())
    # the basis: same subspace as the oracle's, orthonormal
    Q = res.Q().cpu().numpy().T
    assert np.abs(Q.T @ Q - np.eye(res.m)).max() <= 1e-12
    cos = principal_cosines(ores.Q, Q)
    assert cos.min() >= 1 - 1e-8
    # reduced matrices: the MFMA Gram against numpy on the GPU's own basis, and the
    # reduced transfer function against the full one at every sample point
    ns = wl.n_src
    for i, p in enumerate(pts):
        Ar, Br, Cr, Er = [t.cpu().numpy() for t in prob.reduced(res, p)]
        A = orc.A(i)
        Ar_ref = Q.T @ (A @ Q)
        assert np.abs(Ar - Ar_ref).max() <= 1e-12 * np.abs(Ar_ref).max()
        assert np.abs(Er - np.eye(res.m)).max() <= 1e-12
        np.testing.assert_allclose(Br, Q.T @ orc.B[:, :ns], rtol=0, atol=1e-15)
        np.testing.assert_allclose(Cr, Q.T @ orc.B[:, ns:], rtol=0, atol=1e-15)
        if wl.n_src == 0 or wl.n_det == 0:
            continue
        psir = orom.reduced_transfer(Ar, Br, Cr)
        psir_o = orom.reduced_transfer(*orom.reduced_matrices(ores.Q, A, orc.B[:, :ns], orc.B[:, ns:])[:3])
        assert np.abs(psir - psir_o).max() <= psi_tol * np.abs(psir_o).max()
        if interpolates:
            psi = orc.psi(i)
            assert np.abs(psir - psi).max() <= psi_tol * np.abs(psi).max(), i


def test_slab2d_32_sequence_parity(drv):
    wl = ph.WORKLOADS["slab2d_32"]
    orc = OracleProblem(wl)
    ores = orc.run()
    prob, pts, res = _gpu_run(drv, wl)
    _check_sequence(wl, orc, ores, res, prob, pts)
    res.close()
    prob.close()


@pytest.mark.parametrize("wl", [ph.small(3, (12, 11, 10), n_src=5, n_det=4, K=3),
                                ph.small(3, (10, 10, 12), n_src=4, n_det=4, K=3, D="lognormal"),
                                ph.small(2, (40, 23), n_src=6, n_det=5, K=3)])
def test_small_sequence_parity(drv, wl):
    orc = OracleProblem(wl)
    ores = orc.run()
    prob, pts, res = _gpu_run(drv, wl)
    _check_sequence(wl, orc, ores, res, prob, pts)
    res.close()
    prob.close()


@pytest.mark.parametrize("radius,compact", [((0.10, 0.14), True), ((0.6, 0.8), False)])
def test_bump_support_paths(drv, radius, compact):
    """The border term V^T (dmu o q) and the per-point Gram V^T diag(dmu) V run on V
    gathered on the rows of bump support when that support is at most max(1024, n/4)
    rows, else on the full rows with zero chunks skipped.  Small bumps (about 2% of the
    grid) take the first path, large ones (over 90%) the second; both match the oracle."""
    from oracle import operator as op
    wl = ph.small(3, (15, 14, 13), n_src=4, n_det=3, K=3).replace(radius=radius)
    cap = min(wl.n, max(1024, wl.n // 4))
    for p in ph.parameter_points(wl):
        mu = op.mu_field(wl.dim, wl.N, p.mu0, p.centers, p.radii, p.amps)
        support = int(np.count_nonzero(mu != p.mu0))
        assert (0 < support <= cap) == compact, (support, cap)
    orc = OracleProblem(wl)
    ores = orc.run()
    prob, pts, res = _gpu_run(drv, wl)
    _check_sequence(wl, orc, ores, res, prob, pts)
    res.close()
    prob.close()


def test_no_recycle_seed(drv):
    """k_u = 0: the first solve is plain CG from zero (the empty-basis edge case)."""
    wl = ph.small(3, (9, 9, 9), n_src=3, n_det=3, K=2, k_u=0)
    orc = OracleProblem(wl, k_u=0)
    ores = orc.run()
    prob, pts, res = _gpu_run(drv, wl, k_u=0)
    assert res.stats["k_u"] == 0
    _check_sequence(wl, orc, ores, res, prob, pts)


def test_truncated_corrections(drv):
    """A large truncation threshold drops many corrections; the right-hand side after a
    dropped one starts from V y (V unchanged) instead of the bordered start.  Decisions,
    solutions and the basis against the oracle run with the same threshold."""
    # rho (the share of a unit correction outside V) is 0.97-1.0 here, as a correction is
    # A-orthogonal to V; trunc = 0.982 drops 5 of the 18 corrections and sits at least 0.28%
    # from every rho of this sequence (oracle), far beyond the FP64 differences of the sides
    wl = ph.small(3, (10, 9, 8), n_src=3, n_det=3, K=3, tol=1e-10, D="lognormal")
    trunc = 0.982
    orc = OracleProblem(wl)
    ores = orc.run(trunc=trunc)
    prob, pts, res = _gpu_run(drv, wl, trunc=trunc)
    recs = res.records
    dropped_then_solved = [
        (a["point"], a["rhs"]) for a, b in zip(recs, recs[1:])
        if a["solved"] and not a["kept"] and b["solved"] and b["point"] == a["point"]]
    assert dropped_then_solved, "the pattern this test is for did not occur"
    assert any(r["solved"] and r["kept"] for r in recs)
    _check_sequence(wl, orc, ores, res, prob, pts, interpolates=False, trunc=trunc)


def test_cap_and_repeated_point(drv):
    """Basis cap reached mid-sequence; a repeated point needs no iteration."""
    import torch
    wl = ph.small(3, (8, 9, 10), n_src=4, n_det=4, K=2, tol=1e-9, cap=16)
    orc = OracleProblem(wl)
    ores = orc.run(cap=16)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, cap=16)
    assert res.m == 16 == ores.Q.shape[1]
    assert res.stats["n_dropped_cap"] > 0
    _check_sequence(wl, orc, ores, res, prob, pts, interpolates=False)
    # repeated point: every RHS of the second copy is skipped
    wl2 = ph.small(2, (14, 14), n_src=3, n_det=3, K=1, tol=1e-10)
    prob2 = drv.problem_from_workload(wl2)
    p2 = drv.points_from_workload(wl2)
    res2 = prob2.solve([p2[0], p2[0]], 1e-10)
    second = [r for r in res2.records if r["point"] == 1]
    assert all(r["its"] == 0 and not r["solved"] and r["rho0"] <= 1e-10 for r in second)


def test_single_rhs_and_determinism(drv):
    import torch
    wl = ph.small(3, (10, 11, 12), n_src=1, n_det=0, K=3)
    orc = OracleProblem(wl)
    ores = orc.run()
    prob, pts, res = _gpu_run(drv, wl)
    _check_sequence(wl, orc, ores, res, prob, pts)
    res_b = prob.solve(pts, wl.tol, wl.trunc)
    assert torch.equal(res.X, res_b.X)
    assert [r["its"] for r in res.records] == [r["its"] for r in res_b.records]


def test_kernel_timing_accounting(drv):
    """Every timing class enabled: results unchanged, event times and byte counts sane."""
    import torch
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (12, 10, 11), n_src=3, n_det=3, K=2)
    prob, pts, res = _gpu_run(drv, wl)
    res_t = prob.solve(pts, wl.tol, wl.trunc, timing=(1 << R.ROM_NK) - 1)
    assert torch.equal(res.X, res_t.X)
    k = res_t.stats["kernels"]
    its = res_t.stats["total_its"]
    # one update per iteration; one operator step per iteration plus, per CG sweep, the one
    # that found the sweep converged; a start and a finish per sweep
    sweeps = sum(1 + r["restarts"] for r in res_t.records if r["solved"])
    assert k["dcg_update"]["launches"] == its
    assert k["dcg_op"]["launches"] == its + sweeps
    assert k["dcg_ends"]["launches"] == 2 * sweeps
    for name in ("dcg_op", "dcg_update", "dcg_ends", "gemvt", "gemvn", "gram", "outer"):
        assert k[name]["launches"] > 0 and k[name]["ms"] > 0 and k[name]["bytes"] > 0, name
    assert res.stats["kernels"]["dcg_op"]["ms"] == 0.0      # no events when timing is off


def test_invalid_inputs_rejected(drv):
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (6, 6, 6), n_src=2, n_det=2, K=1)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    prob.src_idx = np.array([0, wl.n], dtype=np.int64)        # out of range
    with pytest.raises(R.RomError) as e:
        prob.solve(pts, 1e-8)
    assert e.value.status == R.ROM_EINVAL
    prob.src_idx = np.array([0, 1], dtype=np.int64)
    import torch
    opts = R.make_opts(1e-8)
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RomError) as e:
        R.rom_solve_sequence(prob.op, pts, prob.src_idx, prob.src_scale, prob.det_idx,
                             prob.det_scale, prob.U0, prob.k_u, opts, ws)
    assert e.value.status == R.ROM_ECAPACITY
    bad = R.MuParams(0.01, np.zeros((1, 3)), np.array([-1.0]), np.array([0.01]))
    with pytest.raises(R.RomError) as e:
        prob.solve([bad], 1e-8)
    assert e.value.status == R.ROM_EINVAL
