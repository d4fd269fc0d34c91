"""The streaming form of Algorithm 2 (rom_sequence_begin / point / basis / end): fed the
same points one at a time it takes the same decisions and returns the same solutions,
records and basis as rom_solve_sequence, bit for bit (the same kernels in the same order);
the basis view between points gives the reduced matrices of the basis so far; a point past
the sized count and any call after an error are rejected."""
import numpy as np
import pytest

import phantoms as ph

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,group", [(0, 1), (1, 1), (0, 4)])
def test_stream_equals_whole_sequence(gpu, precision, group):
    import torch
    from paper_1602_00138_amd import driver
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (12, 10, 11), n_src=4, n_det=3, K=3, D="lognormal")
    prob = driver.problem_from_workload(wl)
    pts = driver.points_from_workload(wl)
    whole = prob.solve(pts, wl.tol, wl.trunc, precision=precision, group=group)
    s = prob.stream(len(pts), wl.tol, wl.trunc, precision=precision, group=group)
    Xs = []
    for i, p in enumerate(pts):
        X = torch.empty((wl.n_rhs, wl.n), dtype=torch.float64, device="cuda")
        status, recs = s.point(p, X)
        assert status == R.ROM_OK and len(recs) == wl.n_rhs
        assert all(r["point"] == i for r in recs)
        Xs.append(X)
        # the basis so far, as a view: its size is the last record's m
        V = s.basis_view()
        n, m = R.rom_basis_dims(V)
        assert n == wl.n and m == recs[-1]["m"]
    with pytest.raises(R.RomError) as e:
        s.point(pts[0])
    assert e.value.status == R.ROM_EINVAL
    res = s.end()
    assert torch.equal(torch.cat(Xs), whole.X)
    assert [(r["its"], r["kept"], r["rho0"]) for r in res.records] == \
        [(r["its"], r["kept"], r["rho0"]) for r in whole.records]
    assert res.m == whole.m and torch.equal(res.Q(), whole.Q())
    assert res.stats["total_its"] == whole.stats["total_its"]
    a = [t.cpu().numpy() for t in prob.reduced(res, pts[-1])]
    b = [t.cpu().numpy() for t in prob.reduced(whole, pts[-1])]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    res.close()
    whole.close()
    prob.close()


def test_stream_stops_after_error(gpu):
    from paper_1602_00138_amd import driver
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (9, 9, 9), n_src=2, n_det=2, K=2)
    prob = driver.problem_from_workload(wl)
    pts = driver.points_from_workload(wl)
    s = prob.stream(3, 1e-8)
    s.point(pts[0])
    bad = R.MuParams(0.01, np.array([[0.5, 0.5, 0.5]]), np.array([0.35]), np.array([-60.0]))
    with pytest.raises(R.RomError) as e:
        s.point(bad)
    assert e.value.status == R.ROM_ENOTSPD
    with pytest.raises(R.RomError) as e:
        s.point(pts[1])
    assert e.value.status == R.ROM_EINVAL
    with pytest.raises(R.RomError):
        s.end()
    prob.close()
