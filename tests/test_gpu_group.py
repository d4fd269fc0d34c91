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


CASES = [(ph.WORKLOADS["slab2d_32"], 4),
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


def test_concurrent_sequences_on_uneven_grids(drv):
    """Independent sequences on grids of different sizes run concurrently (one stream
    and host thread each): every result is bitwise the one the sequence gives alone, and
    matches the oracle.  A failing job reports its own error without stopping the rest."""
    import torch
    from paper_1602_00138_amd import rom as R
    wls = [ph.small(3, (10, 11, 12), n_src=3, n_det=3, K=2),
           ph.small(3, (14, 9, 8), n_src=4, n_det=2, K=3, D="lognormal"),
           ph.small(2, (30, 21), n_src=3, n_det=4, K=2)]
    probs = [drv.problem_from_workload(w) for w in wls]
    pts = [drv.points_from_workload(w) for w in wls]
    for prec, group in ((R.ROM_PREC_FP64, 1), (R.ROM_PREC_MIXED, 4)):
        many = drv.solve_many(probs, pts, 1e-10, keep_X=True, precision=prec, group=group)
        for w, prob, p, res in zip(wls, probs, pts, many):
            alone = prob.solve(p, 1e-10, w.trunc, precision=prec, group=group)
            assert torch.equal(res.X, alone.X)
            assert res.m == alone.m
            assert [r["its"] for r in res.records] == [r["its"] for r in alone.records]
            alone.close()
    orc = OracleProblem(wls[1])
    ores = orc.run(tol=1e-10)
    many = drv.solve_many(probs, pts, 1e-10, keep_X=True)
    _check_sequence(wls[1].replace(tol=1e-10), orc, ores, many[1], probs[1], pts[1])
    bad = list(pts)
    bad[1] = [R.MuParams(0.01, np.zeros((1, 3)), np.array([-1.0]), np.array([0.01]))]
    with pytest.raises(R.RomError) as e:
        drv.solve_many(probs, bad, 1e-10)
    assert e.value.status == R.ROM_EINVAL and "job 1" in str(e.value)


@pytest.mark.parametrize("precision,group", [(0, 1), (1, 1), (0, 4), (1, 8)])
def test_graph_replay_equals_eager(drv, precision, group):
    """CG chunks replayed from a captured HIP graph give bitwise the eager results (the
    graph is replayed many times per solve, with host polls and other eager work between
    the replays)."""
    import torch
    wl = ph.small(3, (13, 12, 11), n_src=5, n_det=4, K=3, D="lognormal")
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    eager = prob.solve(pts, wl.tol, wl.trunc, precision=precision, group=group)
    graph = prob.solve(pts, wl.tol, wl.trunc, precision=precision, group=group, graph=1)
    assert torch.equal(eager.X, graph.X)
    assert [r["its"] for r in eager.records] == [r["its"] for r in graph.records]
    assert eager.m == graph.m
    eager.close()
    graph.close()
    prob.close()
