"""Pins for the FP64 reference of the learned-seed network: convolution against SciPy's
n-dimensional correlation, every backward against central finite differences, the pooling
and upsampling backward passes against their adjoint identities, and Adam's first step
against its closed form."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import seednet as sn


def test_conv3d_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 4, 6))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    y = sn.conv3d(x, w, b)
    for o in range(2):
        ref = b[o] + sum(ndi.correlate(x[i], w[o, i], mode="constant", cval=0.0) for i in range(3))
        np.testing.assert_allclose(y[o], ref, rtol=1e-13, atol=1e-13)


def _fd(f, x, idx, h=1e-6):
    xp = x.copy()
    xm = x.copy()
    xp[idx] += h
    xm[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


def test_conv3d_backward_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 3, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    dy = rng.standard_normal((3, 4, 3, 5))
    dx, dw, db = sn.conv3d_backward(x, w, dy)
    L = lambda xx, ww, bb: float((dy * sn.conv3d(xx, ww, bb)).sum())
    for idx in [(0, 0, 0, 0), (1, 3, 2, 4), (0, 2, 1, 2)]:
        assert abs(_fd(lambda t: L(t, w, b), x, idx) - dx[idx]) <= 1e-7 * (1 + abs(dx[idx]))
    for idx in [(0, 0, 0, 0, 0), (2, 1, 2, 1, 0), (1, 0, 1, 2, 2)]:
        assert abs(_fd(lambda t: L(x, t, b), w, idx) - dw[idx]) <= 1e-7 * (1 + abs(dw[idx]))
    for o in range(3):
        assert abs(_fd(lambda t: L(x, w, t), b, (o,)) - db[o]) <= 1e-7 * (1 + abs(db[o]))


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 6, 8))
    y = rng.standard_normal((3, 2, 3, 4))
    assert abs((sn.pool(x) * y).sum() - (x * sn.pool_backward(y)).sum()) <= 1e-12
    assert abs((sn.up(y) * x).sum() - (y * sn.up_backward(x)).sum()) <= 1e-12
    c = np.full((1, 4, 4, 4), 2.5)
    np.testing.assert_allclose(sn.pool(c), 2.5)
    np.testing.assert_allclose(sn.pool(sn.up(y)), y)


@pytest.fixture(scope="module")
def net():
    rng = np.random.default_rng(3)
    p = sn.init_params(rng, c_in=3, c_out=1)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((3, 8, 8, 8))
    t = rng.standard_normal((8, 8, 8))
    return p, x, t


def test_network_gradient_finite_differences(net):
    p, x, t = net
    loss, g = sn.loss_and_grad(p, x, t)
    rng = np.random.default_rng(4)
    for k in sn.LAYERS:
        for suffix in (".w", ".b"):
            name = k + suffix
            idx = tuple(int(rng.integers(s)) for s in p[name].shape)

            def f(v):
                q = dict(p)
                q[name] = v
                return sn.loss_and_grad(q, x, t)[0]

            fd = _fd(f, p[name], idx, h=1e-5)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1e-3, abs(fd)), (name, fd, g[name][idx])


def test_gradient_check_catches_missing_skip(net):
    """A planted mistake (the decoder's skip gradient into e0 dropped) fails the same
    finite-difference check that the correct backward passes."""
    p, x, t = net
    y, a = sn.forward(p, x)
    loss, dy = sn.mse(y, t)
    # the correct chain down to level 1, then e0 without its skip term
    dd0 = sn.conv3d_backward(a["d0"], p["head.w"], dy)[0]
    dz0 = dd0 * (a["d0"] > 0)
    dd1 = sn.up_backward(sn.conv3d_backward(a["u0"], p["d0.w"], dz0)[0])
    dz1 = dd1 * (a["d1"] > 0)
    dd2 = sn.up_backward(sn.conv3d_backward(a["u1"], p["d1.w"], dz1)[0])
    dz2 = dd2 * (a["d2"] > 0)
    de3 = sn.up_backward(sn.conv3d_backward(a["u2"], p["d2.w"], dz2)[0])
    de2 = dz2 + sn.pool_backward(sn.conv3d_backward(a["p3"], p["e3.w"], de3 * (a["e3"] > 0))[0])
    de1 = dz1 + sn.pool_backward(sn.conv3d_backward(a["p2"], p["e2.w"], de2 * (a["e2"] > 0))[0])
    de0_bad = sn.pool_backward(sn.conv3d_backward(a["p1"], p["e1.w"], de1 * (a["e1"] > 0))[0])
    g_bad = sn.conv3d_backward(x, p["e0.w"], de0_bad * (a["e0"] > 0))[1]
    g_ok = sn.backward(p, a, dy)["e0.w"]
    name, idx = "e0.w", (3, 1, 1, 1, 1)

    def f(v):
        q = dict(p)
        q[name] = v
        return sn.loss_and_grad(q, x, t)[0]

    fd = _fd(f, p[name], idx, h=1e-5)
    assert abs(fd - g_ok[idx]) <= 1e-6 * max(1e-3, abs(fd))
    assert abs(fd - g_bad[idx]) > 1e-6 * max(1e-3, abs(fd))


def test_adam_first_step_closed_form():
    p = {"a": np.array([1.0, -2.0, 0.5])}
    g = {"a": np.array([0.3, -0.2, 1e-3])}
    st = {}
    sn.adam(p, g, st, lr=0.01)
    # m_hat = g and v_hat = g^2 after one step: p - lr g / (|g| + eps)
    np.testing.assert_allclose(p["a"], np.array([1.0, -2.0, 0.5]) - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8),
                               rtol=1e-12)


def test_subspace_loss_pins():
    """The recycle-vector loss: zero when the solutions lie in span(N), invariant to
    N -> N S, bounded by 1, equal to 1 - ||Q^T x^||^2 per column (Q an orthonormal basis of
    span(N)), and its gradient against central differences (a planted sign error fails)."""
    rng = np.random.default_rng(9)
    n, k, s = 60, 5, 7
    N = rng.standard_normal((n, k))
    X = rng.standard_normal((n, s)) * rng.uniform(0.1, 10.0, s)
    L = sn.subspace_loss(N, X)
    assert 0.0 < L < 1.0
    Q, _ = np.linalg.qr(N)
    Xh = X / np.linalg.norm(X, axis=0)
    np.testing.assert_allclose(L, np.mean(1.0 - ((Q.T @ Xh) ** 2).sum(axis=0)), rtol=1e-12)
    S = rng.standard_normal((k, k)) + 3 * np.eye(k)
    np.testing.assert_allclose(sn.subspace_loss(N @ S, X), L, rtol=1e-10)
    assert sn.subspace_loss(N, N @ rng.standard_normal((k, 3))) <= 1e-26
    G = sn.subspace_loss_grad(N, X)
    h = 1e-6
    for _ in range(12):
        i, j = rng.integers(n), rng.integers(k)
        Np, Nm = N.copy(), N.copy()
        Np[i, j] += h
        Nm[i, j] -= h
        fd = (sn.subspace_loss(Np, X) - sn.subspace_loss(Nm, X)) / (2 * h)
        assert abs(fd - G[i, j]) <= 1e-7 * (1 + abs(fd))
    # moving N within its own span (N -> N + t N S) leaves the loss unchanged: <G, N S> = 0
    assert abs(np.sum(G * (N @ S))) <= 1e-12 * np.linalg.norm(G) * np.linalg.norm(N @ S)
