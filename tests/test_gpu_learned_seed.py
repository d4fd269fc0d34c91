"""The learned seed end to end on a 32^3 grid: the network is trained on the GPU on
solutions the method itself produced at other parameter points, its guesses then start
the solves of new points, in the paper's order and in groups of 4.  The solutions must pass
the same gates as without a guess (FP64 true residual <= tol under the oracle's operator,
agreement with the oracle's solutions, the reduced transfer function interpolating the
full one -- the correction appended is still x - x0), every accepted guess lowers the
starting residual, and the trained network's guesses need fewer CG iterations in total
than no guess (and lower the starting residual more than the untrained network's)."""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem
from oracle import rom as orom

pytestmark = pytest.mark.gpu

TRAIN = ph.small(3, (32, 32, 32), n_src=8, n_det=8, K=12, tol=1e-10, seed=4242)
WL = ph.small(3, (32, 32, 32), n_src=8, n_det=8, K=3, tol=1e-10, seed=777)


@pytest.fixture(scope="module")
def trained(gpu):
    from paper_1602_00138_amd import driver, seed
    prob = driver.problem_from_workload(WL)
    train_pts = driver.points_from_workload(TRAIN)
    pts = driver.points_from_workload(WL)
    inputs, targets = seed.dataset(prob, train_pts, 1e-10)
    net = seed.SeedNet((32, 32, 32), 8, seed.he_init(5).astype(np.float32))
    g0 = seed.guesses(net, prob, pts)
    losses = seed.train(net, inputs, targets, steps=300, lr=2e-3, seed=1)
    print(f"\ntraining loss {np.mean(losses[:10]):.3e} -> {np.mean(losses[-10:]):.3e}")
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])
    g1 = seed.guesses(net, prob, pts)
    orc = OracleProblem(WL)
    yield prob, pts, g0, g1, orc, orc.run()
    net.close()
    prob.close()


def _gates(res, prob, pts, orc, ores):
    n_rhs = WL.n_rhs
    assert all(r["converged"] and r["final_res"] <= WL.tol * (1 + 1e-6) for r in res.records)
    for r in res.records:
        if r["solved"]:
            assert r["rho_guess"] <= r["rho0"] * (1 + 1e-12)
    X = res.X.cpu().numpy()
    for i, p in enumerate(pts):
        A = orc.A(i)
        Xi = X[i * n_rhs:(i + 1) * n_rhs].T
        rel = np.linalg.norm(orc.B - A @ Xi, axis=0) / np.linalg.norm(orc.B, axis=0)
        assert rel.max() <= WL.tol * (1 + 1e-6)
        err = np.linalg.norm(Xi - ores.X[i], axis=0) / np.linalg.norm(ores.X[i], axis=0)
        assert err.max() <= 1e-7
        Ar, Br, Cr, _ = [t.cpu().numpy() for t in prob.reduced(res, p)]
        psir = orom.reduced_transfer(Ar, Br, Cr)
        psi = orc.psi(i)
        assert np.abs(psir - psi).max() <= 1e-6 * np.abs(psi).max()


def _summary(res):
    solved = [r for r in res.records if r["solved"]]
    gain = [np.log10(r["rho0"] / r["rho_guess"]) for r in solved if r["rho_guess"] > 0]
    return (sum(r["its"] for r in res.records), len(solved),
            float(np.mean(gain)) if gain else 0.0, res.m)


@pytest.mark.parametrize("group", [1, 4])
def test_learned_seed_ab(trained, group):
    prob, pts, g0, g1, orc, ores = trained
    plain = prob.solve(pts, WL.tol, WL.trunc, group=group)
    untrained = prob.solve(pts, WL.tol, WL.trunc, guess=g0, group=group)
    learned = prob.solve(pts, WL.tol, WL.trunc, guess=g1, group=group)
    for res in (untrained, learned):
        _gates(res, prob, pts, orc, ores)
    sp, su, sl = _summary(plain), _summary(untrained), _summary(learned)
    print(f"group {group}: iterations / solved / mean log10 residual drop by the guess / m:\n"
          f"  no guess   {sp}\n  untrained  {su}\n  learned    {sl}")
    assert sl[2] >= su[2]
    assert sl[0] < sp[0], (sl, sp)
    for r in (plain, untrained, learned):
        r.close()
