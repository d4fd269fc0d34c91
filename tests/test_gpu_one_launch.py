"""GPU parity of the one-launch CG step (opts.cg_step = 2): the update of step k-1 folded
into operator step k, s, q and w alternating between two buffers by step parity, and every
block summing the previous step's partial rows itself.  The recurrences are those of the
two-launch step (Sec. 4.2.1, deflated CG with the split direction), so the same oracle gates
hold: sequences in FP64 and mixed precision, one node and two nodes per thread, the
variable-coefficient operator, 2-D grids, groups, recycle spaces past 32 columns, graph
replays, and the launch accounting of the timing class."""
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


# odd nx (one node per thread) and even nx (two), constant and log-normal D, 2-D and 3-D
CASES = [ph.WORKLOADS["slab2d_32"],
         ph.small(3, (9, 8, 7), n_src=4, n_det=3, K=3),
         ph.small(3, (12, 11, 10), n_src=5, n_det=4, K=3),
         ph.small(3, (10, 10, 12), n_src=4, n_det=4, K=3, D="lognormal"),
         ph.small(3, (11, 6, 9), n_src=3, n_det=3, K=3, D="lognormal"),
         ph.small(2, (40, 23), n_src=6, n_det=5, K=3)]


@pytest.mark.parametrize("wl", CASES)
def test_one_launch_sequence_parity(drv, wl):
    print(f"\none-launch FP64 {wl.N}", flush=True)
    orc = OracleProblem(wl)
    ores = orc.run()
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, cg_step=2)
    _check_sequence(wl, orc, ores, res, prob, pts)
    res.close()
    prob.close()


@pytest.mark.parametrize("wl,group", [(CASES[2], 1), (CASES[3], 8), (CASES[5], 1)])
def test_one_launch_mixed_parity(drv, wl, group):
    from paper_1602_00138_amd import rom as R
    print(f"\none-launch mixed {wl.N} group {group}", flush=True)
    orc = OracleProblem(wl)
    ores = orc.run(group=group)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, group=group, precision=R.ROM_PREC_MIXED,
                     cg_step=2)
    _check_mixed(wl, orc, ores, prob, pts, res)
    res.close()
    prob.close()


@pytest.mark.parametrize("wl,group", [(CASES[2], 3), (CASES[5], 16)])
def test_one_launch_group_parity(drv, wl, group):
    print(f"\none-launch group {group} {wl.N}", flush=True)
    orc = OracleProblem(wl)
    ores = orc.run(group=group)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, group=group, cg_step=2)
    _check_sequence(wl, orc, ores, res, prob, pts)
    res.close()
    prob.close()


@pytest.mark.parametrize("precision,group", [(0, 1), (1, 4)])
def test_one_launch_wide_recycle_space(drv, precision, group):
    """U_j of 37 or more columns (20 of U_0, X_0(:, j), 16 recycle vectors): the widest
    variant, whose vector sums go through LDS per plane."""
    import torch
    wl = ph.small(3, (14, 13, 12), n_src=5, n_det=5, K=3, nb=3, tol=1e-10, D="lognormal",
                  k_u=20)
    print(f"\none-launch wide precision {precision} group {group}", flush=True)
    orc = OracleProblem(wl)
    ores = orc.run()
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    rnd = torch.as_tensor(np.random.default_rng(3).standard_normal((len(pts), 16, wl.n))
                          .astype(np.float32), device="cuda")
    res = prob.solve(pts, wl.tol, wl.trunc, group=group, precision=precision, recycle=rnd,
                     cg_step=2)
    _gates(res, orc, pts, prob, wl, ores)
    assert res.status == 0 and all(r["converged"] for r in res.records)
    res.close()
    prob.close()


@pytest.mark.parametrize("precision,group", [(0, 1), (1, 1), (0, 4)])
def test_one_launch_agrees_with_two_launch(drv, precision, group):
    """Same recurrences in both forms: the same decisions and basis size, iteration counts
    within 1 (only the summation order of the dot products differs), solutions within the
    solver tolerance of each other."""
    import torch
    wl = ph.small(3, (13, 12, 11), n_src=5, n_det=4, K=3, D="lognormal")
    print(f"\none vs two launches precision {precision} group {group}", flush=True)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    two = prob.solve(pts, wl.tol, wl.trunc, precision=precision, group=group, cg_step=1)
    one = prob.solve(pts, wl.tol, wl.trunc, precision=precision, group=group, cg_step=2)
    assert two.m == one.m
    for a, b in zip(two.records, one.records):
        assert (a["solved"], a["kept"]) == (b["solved"], b["kept"])
        assert abs(a["its"] - b["its"]) <= 1, (a, b)
        assert b["converged"]
    X1, X2 = one.X.cpu().numpy(), two.X.cpu().numpy()
    err = np.linalg.norm(X1 - X2, axis=1) / np.linalg.norm(X2, axis=1)
    assert err.max() <= 1e-8
    two.close()
    one.close()
    prob.close()


@pytest.mark.parametrize("precision,group", [(0, 1), (1, 1), (0, 4), (1, 8)])
def test_one_launch_graph_replay_equals_eager(drv, precision, group):
    """Chunks of 8 one-launch steps (parities 1, 0, ...) replayed from a captured graph
    after the eager step 0 give bitwise the eager results."""
    import torch
    wl = ph.small(3, (13, 12, 11), n_src=5, n_det=4, K=3, D="lognormal")
    print(f"\none-launch graph precision {precision} group {group}", flush=True)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    eager = prob.solve(pts, wl.tol, wl.trunc, precision=precision, group=group, cg_step=2)
    graph = prob.solve(pts, wl.tol, wl.trunc, precision=precision, group=group, graph=1,
                       cg_step=2)
    assert torch.equal(eager.X, graph.X)
    assert [r["its"] for r in eager.records] == [r["its"] for r in graph.records]
    assert eager.m == graph.m
    eager.close()
    graph.close()
    prob.close()


def test_one_launch_timing_accounting(drv):
    """Per CG sweep: step 0, one launch per iteration, and the launch that read the stopping
    test; no launch of the two-launch classes; results unchanged by the events."""
    import torch
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (12, 10, 11), n_src=3, n_det=3, K=2)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, cg_step=2)
    res_t = prob.solve(pts, wl.tol, wl.trunc, timing=(1 << R.ROM_NK) - 1, cg_step=2)
    assert torch.equal(res.X, res_t.X)
    k = res_t.stats["kernels"]
    its = res_t.stats["total_its"]
    sweeps = sum(1 + r["restarts"] for r in res_t.records if r["solved"])
    assert k["dcg_step"]["launches"] == its + 2 * sweeps
    assert k["dcg_op"]["launches"] == 0 and k["dcg_update"]["launches"] == 0
    assert k["dcg_ends"]["launches"] == 2 * sweeps
    assert k["dcg_step"]["ms"] > 0 and k["dcg_step"]["bytes"] > 0
    res.close()
    res_t.close()
    prob.close()


def test_invalid_cg_step_rejected(drv):
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (8, 8, 8), n_src=2, n_det=2, K=1)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    with pytest.raises(R.RomError) as e:
        prob.solve(pts, wl.tol, wl.trunc, cg_step=3)
    assert e.value.status == R.ROM_EINVAL
    prob.close()
