"""The learned seed's second output: 16 recycle vectors per parameter point that join the
recycle spaces U_j (not V).

* The 16-output network against the FP64 reference network on the same BF16-rounded
  parameters and inputs: outputs, and the parameter gradient of a given output gradient
  (rom_seednet_backward) -- the gates of the one-output network (output 2e-2, gradients
  1e-1 relative, the differences being BF16 storage of activations and gradients).
* rom_subspace_loss against the oracle's definition (least-squares projection) and its
  gradient (central differences pin it): loss to 1e-9, gradient to 1e-6 relative (the
  GPU rounds the gradient to FP32); linearly dependent outputs give ROM_ENOTSPD.
* Sequences with recycle vectors pass the gates of the plain form (FP64 true residual under
  the oracle's operator, oracle solutions, interpolation of the transfer function); with the
  oracle's own solutions of some right-hand sides as recycle vectors the solves that see V
  as it was at the point start need few iterations; random recycle vectors change
  iterations, not results.
* End to end: the network trained on the subspace loss on other points lowers the loss,
  and its vectors keep every gate."""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem
from oracle import rom as orom
from oracle import seednet as sn

pytestmark = pytest.mark.gpu


def bf16(a: np.ndarray) -> np.ndarray:
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def test_sixteen_output_network_matches_reference(gpu):
    import torch
    from paper_1602_00138_amd import seed
    rng = np.random.default_rng(17)
    grid, B, k = (16, 16, 16), 2, 16
    p = seed.unflatten(seed.he_init(3, outputs=k), outputs=k)
    for name in p:
        if name.endswith(".b"):
            p[name] = 0.05 * rng.standard_normal(p[name].shape)
        p[name] = bf16(p[name]) if name.endswith(".w") else \
            np.asarray(p[name], dtype=np.float32).astype(np.float64)
    flat = seed.flatten(p)
    x = bf16(rng.standard_normal((B, 3) + grid[::-1]))
    net = seed.SeedNet(grid, B, flat.astype(np.float32), outputs=k)
    xin = torch.as_tensor(x.reshape(B, 3, -1), dtype=torch.float32, device="cuda")
    y = net.forward(xin).cpu().numpy()
    assert y.shape == (B, k, 16 ** 3)
    # output gradient of the loss 1e-3 ||y||^2 / 2 (correlated with the outputs, as the
    # gradient of any fitting loss is; a random one sums random-sign terms per parameter)
    refs = [sn.forward(p, x[b]) for b in range(B)]
    dy = np.stack([bf16(1e-3 * r[0]) for r in refs])
    din = torch.as_tensor(dy.reshape(B, k, -1), dtype=torch.float32, device="cuda")
    ref_g = None
    for b in range(B):
        ref, a = refs[b]
        e = _rel(y[b], ref.reshape(k, -1))
        assert e <= 2e-2, (b, e)
        gb = seed.flatten(sn.backward(p, a, dy[b]))
        ref_g = gb if ref_g is None else ref_g + gb
    g = net.backward(xin, din, grads=True).astype(np.float64)
    gg, rg = seed.unflatten(g, outputs=k), seed.unflatten(ref_g, outputs=k)
    worst = 0.0
    for name, _, _ in seed.layers(k):
        for suf in (".w", ".b"):
            e = _rel(gg[name + suf], rg[name + suf])
            worst = max(worst, e)
            assert e <= 1e-1, (name + suf, e)
    print(f"\nworst gradient rel. error {worst:.2e}")
    # one Adam step moves the parameters and keeps them finite
    before = net.params()
    net.adam(1e-3)
    after = net.params()
    assert np.isfinite(after).all() and np.abs(after - before).max() > 0
    net.close()


def test_subspace_loss_parity(gpu):
    import torch
    from paper_1602_00138_amd import rom as R
    rng = np.random.default_rng(5)
    n, k, s = 5000, 16, 24
    Y = rng.standard_normal((k, n)).astype(np.float32)
    basis = rng.standard_normal((n, 6))
    X = np.hstack([basis @ rng.standard_normal((6, s - 4)), rng.standard_normal((n, 4))])
    X *= rng.uniform(0.1, 10.0, s)
    Yd = torch.as_tensor(Y, device="cuda")
    Xd = torch.as_tensor(np.asfortranarray(X).T.copy(), device="cuda")   # (s, n) rows = columns
    dY = torch.empty_like(Yd)
    scratch = torch.empty(R.rom_subspace_loss_bytes(n, k, s), dtype=torch.uint8, device="cuda")
    loss = R.rom_subspace_loss(Yd, k, Xd, n, n, s, dY, scratch)
    N = Y.astype(np.float64).T
    ref = sn.subspace_loss(N, X)
    assert abs(loss - ref) <= 1e-9 * ref, (loss, ref)
    G = sn.subspace_loss_grad(N, X).T                                   # (k, n)
    assert _rel(dY.cpu().numpy(), G) <= 1e-6
    # loss only (no gradient)
    assert abs(R.rom_subspace_loss(Yd, k, Xd, n, n, s, None, scratch) - loss) <= 1e-15 * loss
    # dependent outputs
    Yb = Y.copy()
    Yb[3] = Yb[1]
    with pytest.raises(R.RomError) as e:
        R.rom_subspace_loss(torch.as_tensor(Yb, device="cuda"), k, Xd, n, n, s, dY, scratch)
    assert e.value.status == R.ROM_ENOTSPD


def _gates(res, orc, pts, prob, wl, ores):
    X = res.X.cpu().numpy()
    n_rhs = wl.n_rhs
    assert all(r["converged"] and r["final_res"] <= wl.tol * (1 + 1e-6) for r in res.records)
    for i, p in enumerate(pts):
        A = orc.A(i)
        Xi = X[i * n_rhs:(i + 1) * n_rhs].T
        rel = np.linalg.norm(orc.B - A @ Xi, axis=0) / np.linalg.norm(orc.B, axis=0)
        assert rel.max() <= wl.tol * (1 + 1e-6)
        err = np.linalg.norm(Xi - ores.X[i], axis=0) / np.linalg.norm(ores.X[i], axis=0)
        assert err.max() <= 1e-7
        Ar, Br, Cr, _ = [t.cpu().numpy() for t in prob.reduced(res, p)]
        psi = orc.psi(i)
        assert np.abs(orom.reduced_transfer(Ar, Br, Cr) - psi).max() <= 1e-6 * np.abs(psi).max()


@pytest.mark.parametrize("group", [1, 4])
def test_sequence_with_recycle_vectors(gpu, group):
    import torch
    from paper_1602_00138_amd import driver
    from paper_1602_00138_amd import rom as R
    wl = ph.small(3, (14, 13, 12), n_src=6, n_det=6, K=3, nb=3, tol=1e-10, D="lognormal")
    orc = OracleProblem(wl)
    ores = orc.run()
    prob = driver.problem_from_workload(wl)
    pts = driver.points_from_workload(wl)
    K, n, n_rhs = len(pts), wl.n, wl.n_rhs
    plain = prob.solve(pts, wl.tol, wl.trunc, group=group)
    _gates(plain, orc, pts, prob, wl, ores)
    # (a) the oracle's solutions of right-hand sides 0, 3, 7, 10 as recycle vectors
    chosen = [0, 3, 7, 10]
    rec = np.stack([ores.X[i][:, chosen].T for i in range(K)]).astype(np.float32)
    exact = prob.solve(pts, wl.tol, wl.trunc, group=group,
                       recycle=torch.as_tensor(rec, device="cuda"))
    _gates(exact, orc, pts, prob, wl, ores)
    its_plain = {(r["point"], r["rhs"]): r["its"] for r in plain.records}
    # the vectors are made A-orthogonal to V as it stands at the point start, which is the
    # V of the first right-hand side (the first group's members, for groups): there the
    # correction x_j - x0 lies in span(U_j) up to the FP32 rounding of x_j, so CG only
    # cleans up the last digits (later solves see V grown by this point's corrections)
    first = set(range(group))
    for r in exact.records:
        if r["rhs"] in chosen and r["rhs"] in first and r["solved"]:
            assert r["its"] <= max(0.6 * its_plain[(r["point"], r["rhs"])], 8), r
    tot = lambda res: sum(r["its"] for r in res.records)
    print(f"\ngroup {group}: iterations plain {tot(plain)}, with exact recycle vectors {tot(exact)}")
    # (b) random recycle vectors (16 per point)
    rnd = torch.as_tensor(np.random.default_rng(1).standard_normal((K, 16, n)).astype(np.float32),
                          device="cuda")
    randr = prob.solve(pts, wl.tol, wl.trunc, group=group, recycle=rnd)
    _gates(randr, orc, pts, prob, wl, ores)
    print(f"group {group}: with random recycle vectors {tot(randr)}")
    for res in (plain, exact, randr):
        res.close()
    # too many vectors
    with pytest.raises(R.RomError):
        prob.solve(pts, wl.tol, wl.trunc, recycle=torch.zeros((K, 17, n), dtype=torch.float32,
                                                              device="cuda"))


def test_trained_recycle_network(gpu):
    import torch
    from paper_1602_00138_amd import driver, seed
    train_wl = ph.small(3, (32, 32, 32), n_src=8, n_det=8, K=12, tol=1e-10, seed=4242)
    wl = ph.small(3, (32, 32, 32), n_src=8, n_det=8, K=3, tol=1e-10, seed=777)
    prob = driver.problem_from_workload(wl)
    train_pts = driver.points_from_workload(train_wl)
    pts = driver.points_from_workload(wl)
    inputs, X = seed.recycle_dataset(prob, train_pts, 1e-10)
    net = seed.SeedNet((32, 32, 32), 4, seed.he_init(8, outputs=16).astype(np.float32),
                       outputs=16)
    losses = seed.train_recycle(net, inputs, X, wl.n_rhs, steps=150, lr=2e-3, seed=2)
    print(f"\nsubspace loss {np.mean(losses[:5]):.3e} -> {np.mean(losses[-5:]):.3e}")
    assert np.mean(losses[-5:]) < 0.7 * np.mean(losses[:5])
    vec = seed.recycle_vectors(net, prob, pts)
    assert vec.shape == (len(pts), 16, wl.n)
    orc = OracleProblem(wl)
    ores = orc.run()
    plain = prob.solve(pts, wl.tol, wl.trunc)
    learned = prob.solve(pts, wl.tol, wl.trunc, recycle=vec)
    _gates(learned, orc, pts, prob, wl, ores)
    tot = lambda res: sum(r["its"] for r in res.records)
    print(f"iterations: plain {tot(plain)}, with learned recycle vectors {tot(learned)}")
    plain.close()
    learned.close()
    net.close()
