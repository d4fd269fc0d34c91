"""GPU parity of the batched form (right-hand sides in groups of g sharing one outer
projection, solved together, appended in order) against the oracle run with the same
group size.  The plain FP64 group path follows the oracle's decisions, iteration
counts (within 2) and basis (principal angles) under the same tolerances as the
sequential form; the mixed-precision group path meets the mixed-form bounds."""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem
from test_gpu_mixed import _check_mixed
from test_gpu_parity import _check_sequence

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def drv(gpu):
    from paper_1602_00138_amd import driver
    return driver


CASES = [(ph.WORKLOADS["cfg1"], 4),
         (ph.small(3, (12, 11, 10), n_src=5, n_det=4, K=3), 3),
         (ph.small(3, (10, 10, 12), n_src=4, n_det=4, K=3, D="lognormal"), 8),
         (ph.small(2, (40, 23), n_src=6, n_det=5, K=3), 16)]


@pytest.mark.parametrize("wl,group", CASES)
def test_group_sequence_parity(drv, wl, group):
    orc = OracleProblem(wl)
    ores = orc.run(group=group)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, group=group)
    _check_sequence(wl, orc, ores, res, prob, pts)
    res.close()
    prob.close()


@pytest.mark.parametrize("wl,group", CASES[:3])
def test_group_mixed_parity(drv, wl, group):
    from paper_1602_00138_amd import rom as R
    orc = OracleProblem(wl)
    ores = orc.run(group=group)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, group=group, precision=R.ROM_PREC_MIXED)
    _check_mixed(wl, orc, ores, prob, pts, res)
    res.close()
    prob.close()


def test_group_cap_and_skips(drv):
    """Cap reached inside a group; a repeated point skips every member of every group."""
    wl = ph.small(3, (8, 9, 10), n_src=4, n_det=4, K=2, tol=1e-9, cap=16)
    orc = OracleProblem(wl)
    ores = orc.run(cap=16, group=3)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, cap=16, group=3)
    assert res.m == 16 == ores.Q.shape[1]
    _check_sequence(wl, orc, ores, res, prob, pts, interpolates=False)
    wl2 = ph.small(2, (14, 14), n_src=3, n_det=3, K=1, tol=1e-10)
    prob2 = drv.problem_from_workload(wl2)
    p2 = drv.points_from_workload(wl2)
    res2 = prob2.solve([p2[0], p2[0]], 1e-10, group=4)
    second = [r for r in res2.records if r["point"] == 1]
    assert all(r["its"] == 0 and not r["solved"] and r["rho0"] <= 1e-10 for r in second)


def test_group_one_equals_sequential(drv):
    import torch
    wl = ph.small(3, (10, 11, 12), n_src=3, n_det=2, K=2)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    a = prob.solve(pts, wl.tol, wl.trunc)
    b = prob.solve(pts, wl.tol, wl.trunc, group=1)
    assert torch.equal(a.X, b.X)


def test_autotuned_shape_parity(drv):
    """With the CG launch shape autotuned, results still match the oracle (the shape only
    changes summation order), and a second solve in the process reuses the shape."""
    import torch
    wl = ph.small(3, (14, 13, 12), n_src=5, n_det=4, K=2)
    orc = OracleProblem(wl)
    for group in (1, 4):
        ores = orc.run(group=group)
        prob = drv.problem_from_workload(wl)
        pts = drv.points_from_workload(wl)
        res = prob.solve(pts, wl.tol, wl.trunc, group=group, tune=1)
        _check_sequence(wl, orc, ores, res, prob, pts)
        again = prob.solve(pts, wl.tol, wl.trunc, group=group, tune=1)
        assert torch.equal(res.X, again.X)
        res.close()
        again.close()
        prob.close()
