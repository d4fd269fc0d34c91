"""GPU parity where the recycle spaces are wide, where U_j reaches its column cap, and the
sequence's breakdown statuses.

* Recycle spaces of more than 32 columns run the widest variants of the deflated-CG
  kernels (U_j and A U_j streamed per row, nothing preloaded): 40 columns of U_0, and 20
  columns of U_0 plus 16 learned-style recycle vectors, in FP64 and mixed precision, in
  the paper's order and in groups; gated like the narrower cases.
* U_j holds at most ROM_NJ_MAX = 64 columns (the paper lets it grow without bound): a
  sequence that reaches the cap matches the oracle run with the same cap (uj_cap=64),
  decision by decision, and reports the corrections that stayed out of U_j.
* A(p) with a strongly negative absorption bump is indefinite: the sequence stops with
  ROM_ENOTSPD.  An absorption background near the largest double overflows the operator
  product: the sequence stops with ROM_ENONFINITE.  Both are raised from the kernels'
  own checks (the kernels exit normally)."""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem
from test_gpu_mixed import _check_mixed
from test_gpu_parity import _check_sequence
from test_gpu_recycle import _gates

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def drv(gpu):
    from paper_1602_00138_amd import driver
    return driver


WIDE = ph.small(3, (12, 11, 10), n_src=4, n_det=3, K=3, k_u=40)


@pytest.mark.parametrize("group", [1, 4])
def test_wide_recycle_space_fp64(drv, group):
    orc = OracleProblem(WIDE)
    ores = orc.run(group=group)
    prob = drv.problem_from_workload(WIDE)
    pts = drv.points_from_workload(WIDE)
    print(f"\nwide U_j: k_u {WIDE.k_u}, group {group}", flush=True)
    res = prob.solve(pts, WIDE.tol, WIDE.trunc, group=group)
    assert res.stats["k_u"] == ores.k_u == 40
    assert sum(r["solved"] for r in res.records) > 0
    _check_sequence(WIDE, orc, ores, res, prob, pts)
    res.close()
    prob.close()


@pytest.mark.parametrize("group", [1, 4])
def test_wide_recycle_space_mixed(drv, group):
    from paper_1602_00138_amd import rom as R
    orc = OracleProblem(WIDE)
    ores = orc.run(group=group)
    prob = drv.problem_from_workload(WIDE)
    pts = drv.points_from_workload(WIDE)
    print(f"\nwide U_j mixed: k_u {WIDE.k_u}, group {group}", flush=True)
    res = prob.solve(pts, WIDE.tol, WIDE.trunc, group=group, precision=R.ROM_PREC_MIXED)
    assert res.stats["k_u"] == 40
    _check_mixed(WIDE, orc, ores, prob, pts, res)
    res.close()
    prob.close()


@pytest.mark.parametrize("precision,group", [(0, 1), (1, 1), (0, 4), (1, 4)])
def test_recycle_vectors_widen_past_32(drv, precision, group):
    """20 columns of U_0, X_0(:, j) and 16 recycle vectors per point: U_j of 37 or more
    columns at every point after the first."""
    import torch
    wl = ph.small(3, (14, 13, 12), n_src=5, n_det=5, K=3, nb=3, tol=1e-10, D="lognormal",
                  k_u=20)
    orc = OracleProblem(wl)
    ores = orc.run()
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    rnd = torch.as_tensor(np.random.default_rng(3).standard_normal((len(pts), 16, wl.n))
                          .astype(np.float32), device="cuda")
    print(f"\nrecycle vectors, k_u 20, precision {precision}, group {group}", flush=True)
    res = prob.solve(pts, wl.tol, wl.trunc, group=group, precision=precision, recycle=rnd)
    assert res.stats["k_u"] == 20
    _gates(res, orc, pts, prob, wl, ores)
    # U_j keeps orthonormal persistent columns (the recycle vectors are left out of its
    # Gram-Schmidt pass): the next point's recycle Gram factorises, every solve converged
    assert res.status == 0 and all(r["converged"] for r in res.records)
    res.close()
    prob.close()


def test_uj_column_cap(drv):
    """k_u = 60: U_j = [U_0, X_0(:, j)] has 61 columns after the first point and reaches
    the 64-column cap after three more kept corrections; the oracle with uj_cap = 64 takes
    the same decisions."""
    wl = ph.small(3, (12, 12, 11), n_src=3, n_det=3, K=6, nb=3, tol=1e-10, k_u=60)
    orc = OracleProblem(wl)
    ores = orc.run()
    capped = orc.wl and __import__("oracle.sequence", fromlist=["x"]).solve_sequence(
        orc.As, orc.mus, orc.B, orc.U0, wl.tol, wl.trunc, uj_cap=64)
    widest = max(len(w) for w in capped.W_extra)
    assert ores.k_u == 60 and widest == 4
    assert max(len(w) for w in ores.W_extra) > 4, "the sequence did not reach the cap"
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    print(f"\nU_j cap: k_u {wl.k_u}, K {wl.K}", flush=True)
    res = prob.solve(pts, wl.tol, wl.trunc)
    assert res.stats["n_uj_capped"] > 0
    _check_sequence(wl, orc, capped, res, prob, pts)
    res.close()
    prob.close()


def test_indefinite_operator_reports_enotspd(drv):
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (9, 9, 9), n_src=2, n_det=2, K=1)
    prob = drv.problem_from_workload(wl)
    bad = R.MuParams(0.01, np.array([[0.5, 0.5, 0.5]]), np.array([0.35]), np.array([-60.0]))
    with pytest.raises(R.RomError) as e:
        prob.solve([bad], 1e-8)
    assert e.value.status == R.ROM_ENOTSPD
    # the library stays usable after the error
    ok = prob.solve(drv.points_from_workload(wl), 1e-8)
    assert all(r["converged"] for r in ok.records)
    ok.close()
    prob.close()


def test_overflow_reports_enonfinite(drv):
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (9, 9, 9), n_src=1, n_det=0, K=1, k_u=0)
    prob = drv.problem_from_workload(wl, k_u=0)
    prob.src_scale = np.array([2.0])
    huge = R.MuParams(1.7e308, np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    with pytest.raises(R.RomError) as e:
        prob.solve([huge], 1e-8)
    assert e.value.status == R.ROM_ENONFINITE
    prob.close()
