"""The learned seed end to end on a 32^3 grid: the network is trained on the GPU on
solutions the method itself produced at other parameter points, its guesses then start
the solves of new points.  The solutions must pass the same gates as without a guess
(FP64 true residual <= tol under the oracle's operator, agreement with the oracle's
solutions, the reduced transfer function interpolating the full one — the correction
appended is still x - x0), every accepted guess lowers the starting residual, and the
test reports what the trained network gains over the untrained one and over no guess."""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem
from oracle import rom as orom

pytestmark = pytest.mark.gpu


def test_learned_seed_ab(gpu):
    import torch
    from paper_1602_00138_amd import driver, seed
    train_wl = ph.small(3, (32, 32, 32), n_src=8, n_det=8, K=12, tol=1e-10, seed=4242)
    wl = ph.small(3, (32, 32, 32), n_src=8, n_det=8, K=3, tol=1e-10, seed=777)
    prob = driver.problem_from_workload(wl)
    train_pts = driver.points_from_workload(train_wl)
    pts = driver.points_from_workload(wl)
    inputs, targets = seed.dataset(prob, train_pts, 1e-10)
    net = seed.SeedNet((32, 32, 32), 8, seed.he_init(5).astype(np.float32))
    g0 = seed.guesses(net, prob, pts)
    losses = seed.train(net, inputs, targets, steps=300, lr=2e-3, seed=1)
    print(f"\ntraining loss {np.mean(losses[:10]):.3e} -> {np.mean(losses[-10:]):.3e}")
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])
    g1 = seed.guesses(net, prob, pts)
    plain = prob.solve(pts, wl.tol, wl.trunc)
    untrained = prob.solve(pts, wl.tol, wl.trunc, guess=g0)
    learned = prob.solve(pts, wl.tol, wl.trunc, guess=g1)
    orc = OracleProblem(wl)
    ores = orc.run()
    n_rhs = wl.n_rhs
    for res in (untrained, learned):
        assert all(r["converged"] and r["final_res"] <= wl.tol * (1 + 1e-6) for r in res.records)
        for r in res.records:
            if r["solved"]:
                assert r["rho_guess"] <= r["rho0"] * (1 + 1e-12)
        X = res.X.cpu().numpy()
        Q = res.Q().cpu().numpy().T
        for i, p in enumerate(pts):
            A = orc.A(i)
            Xi = X[i * n_rhs:(i + 1) * n_rhs].T
            rel = np.linalg.norm(orc.B - A @ Xi, axis=0) / np.linalg.norm(orc.B, axis=0)
            assert rel.max() <= wl.tol * (1 + 1e-6)
            err = np.linalg.norm(Xi - ores.X[i], axis=0) / np.linalg.norm(ores.X[i], axis=0)
            assert err.max() <= 1e-7
            Ar, Br, Cr, _ = [t.cpu().numpy() for t in prob.reduced(res, p)]
            psir = orom.reduced_transfer(Ar, Br, Cr)
            psi = orc.psi(i)
            assert np.abs(psir - psi).max() <= 1e-6 * np.abs(psi).max()

    def summary(res):
        solved = [r for r in res.records if r["solved"]]
        gain = [np.log10(r["rho0"] / r["rho_guess"]) for r in solved if r["rho_guess"] > 0]
        return (sum(r["its"] for r in res.records), len(solved),
                float(np.mean(gain)) if gain else 0.0, res.m)

    sp, su, sl = summary(plain), summary(untrained), summary(learned)
    print(f"iterations / solved / mean log10 residual drop by the guess / m:\n"
          f"  no guess   {sp}\n  untrained  {su}\n  learned    {sl}")
    # the trained network's guesses lower the starting residual more than untrained ones
    assert sl[2] >= su[2]
    for r in (plain, untrained, learned):
        r.close()
    net.close()
    prob.close()
