"""FP64 reference of the learned-seed network (TEST INFRASTRUCTURE ONLY).

The learned seed is not in the paper: a small 3D convolutional network maps, for one
parameter point and one right-hand side, the fields [normalised absorption, log of the
diffusion coefficient, source indicator] to a guess of the normalised solution
x / max|x|, which the solver then uses as an extra starting direction.

Architecture (4 levels, 16 -> 64 channels, 3x3x3 convolutions with zero padding 1):
    e0 = relu(conv(x;  c_in -> 16))                 level 0 (full grid)
    e1 = relu(conv(pool(e0); 16 -> 32))              level 1 (grid / 2)
    e2 = relu(conv(pool(e1); 32 -> 48))              level 2 (grid / 4)
    e3 = relu(conv(pool(e2); 48 -> 64))              level 3 (grid / 8)
    d2 = relu(conv(up(e3); 64 -> 48) + e2)
    d1 = relu(conv(up(d2); 48 -> 32) + e1)
    d0 = relu(conv(up(d1); 32 -> 16) + e0)
    y  = conv(d0; 16 -> c_out)
pool = 2x2x2 average, up = 2x nearest.  Tensors are (channels, z, y, x); weights
(c_out, c_in, 3, 3, 3) with w[o, i, a, b, c] multiplying x[i, z + a - 1, y + b - 1,
x + c - 1].  Everything here is plain NumPy, one layer at a time.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

CHANNELS = (16, 32, 48, 64)
LAYERS = ("e0", "e1", "e2", "e3", "d2", "d1", "d0", "head")


def layer_shapes(c_in: int = 3, c_out: int = 1) -> Dict[str, Tuple[int, int]]:
    c0, c1, c2, c3 = CHANNELS
    return {"e0": (c0, c_in), "e1": (c1, c0), "e2": (c2, c1), "e3": (c3, c2),
            "d2": (c2, c3), "d1": (c1, c2), "d0": (c0, c1), "head": (c_out, c0)}


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[o] = b[o] + sum_i sum_{a,b,c} w[o,i,a,b,c] x[i, z+a-1, y+b-1, x+c-1]."""
    C, Z, Y, X = x.shape
    xp = _pad(x)
    # im2col: cols[i, a, b, c, z, y, x]
    cols = np.empty((C, 3, 3, 3, Z, Y, X))
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                cols[:, a, bb, c] = xp[:, a:a + Z, bb:bb + Y, c:c + X]
    y = np.einsum("oiabc,iabczyx->ozyx", w, cols, optimize=True)
    return y + b[:, None, None, None]


def conv3d_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients (dx, dw, db) of sum(dy * conv3d(x, w, b))."""
    C, Z, Y, X = x.shape
    xp = _pad(x)
    dw = np.empty_like(w)
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                dw[:, :, a, bb, c] = np.einsum("ozyx,izyx->oi", dy,
                                               xp[:, a:a + Z, bb:bb + Y, c:c + X], optimize=True)
    dxp = np.zeros_like(xp)
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                dxp[:, a:a + Z, bb:bb + Y, c:c + X] += np.einsum("oi,ozyx->izyx", w[:, :, a, bb, c],
                                                                 dy, optimize=True)
    return dxp[:, 1:-1, 1:-1, 1:-1], dw, dy.sum(axis=(1, 2, 3))


def pool(x: np.ndarray) -> np.ndarray:
    C, Z, Y, X = x.shape
    return x.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).mean(axis=(2, 4, 6))


def pool_backward(dy: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up(x: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up_backward(dy: np.ndarray) -> np.ndarray:
    C, Z, Y, X = dy.shape
    return dy.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


def init_params(rng: np.random.Generator, c_in: int = 3, c_out: int = 1) -> Dict[str, np.ndarray]:
    """He-normal weights (std sqrt(2 / (27 c_in))) and zero biases."""
    p = {}
    for name, (co, ci) in layer_shapes(c_in, c_out).items():
        p[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci))
        p[name + ".b"] = np.zeros(co)
    return p


def forward(p: Dict[str, np.ndarray], x: np.ndarray):
    """Network output and the activations the backward pass needs."""
    a = {"x": x}
    a["e0"] = relu(conv3d(x, p["e0.w"], p["e0.b"]))
    a["p1"] = pool(a["e0"])
    a["e1"] = relu(conv3d(a["p1"], p["e1.w"], p["e1.b"]))
    a["p2"] = pool(a["e1"])
    a["e2"] = relu(conv3d(a["p2"], p["e2.w"], p["e2.b"]))
    a["p3"] = pool(a["e2"])
    a["e3"] = relu(conv3d(a["p3"], p["e3.w"], p["e3.b"]))
    a["u2"] = up(a["e3"])
    a["d2"] = relu(conv3d(a["u2"], p["d2.w"], p["d2.b"]) + a["e2"])
    a["u1"] = up(a["d2"])
    a["d1"] = relu(conv3d(a["u1"], p["d1.w"], p["d1.b"]) + a["e1"])
    a["u0"] = up(a["d1"])
    a["d0"] = relu(conv3d(a["u0"], p["d0.w"], p["d0.b"]) + a["e0"])
    y = conv3d(a["d0"], p["head.w"], p["head.b"])
    return y, a


def mse(y: np.ndarray, target: np.ndarray) -> Tuple[float, np.ndarray]:
    """Loss mean over voxels of (y[0] - target)^2 and its gradient w.r.t. y."""
    n = target.size
    diff = y[0] - target
    dy = np.zeros_like(y)
    dy[0] = 2.0 * diff / n
    return float((diff * diff).sum() / n), dy


def backward(p: Dict[str, np.ndarray], a, dy: np.ndarray) -> Dict[str, np.ndarray]:
    """Gradients of sum(dy * forward(p, x)) w.r.t. every parameter (chain rule, layer by
    layer in reverse order)."""
    g = {}

    def conv_b(name, xin, dz):
        dx, dw, db = conv3d_backward(xin, p[name + ".w"], dz)
        g[name + ".w"], g[name + ".b"] = dw, db
        return dx

    dd0 = conv_b("head", a["d0"], dy)
    dz = dd0 * (a["d0"] > 0)                 # relu
    de0 = dz.copy()                          # skip into e0
    du0 = conv_b("d0", a["u0"], dz)
    dd1 = up_backward(du0)
    dz = dd1 * (a["d1"] > 0)
    de1 = dz.copy()
    du1 = conv_b("d1", a["u1"], dz)
    dd2 = up_backward(du1)
    dz = dd2 * (a["d2"] > 0)
    de2 = dz.copy()
    du2 = conv_b("d2", a["u2"], dz)
    de3 = up_backward(du2)
    dz = de3 * (a["e3"] > 0)
    dp3 = conv_b("e3", a["p3"], dz)
    de2 += pool_backward(dp3)
    dz = de2 * (a["e2"] > 0)
    dp2 = conv_b("e2", a["p2"], dz)
    de1 += pool_backward(dp2)
    dz = de1 * (a["e1"] > 0)
    dp1 = conv_b("e1", a["p1"], dz)
    de0 += pool_backward(dp1)
    dz = de0 * (a["e0"] > 0)
    conv_b("e0", a["x"], dz)
    return g


def loss_and_grad(p, x, target):
    y, a = forward(p, x)
    loss, dy = mse(y, target)
    return loss, backward(p, a, dy)


def adam(p, g, state, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) in place on p; state holds m, v and the step count."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m." + k, np.zeros_like(p[k]))
        v = state.setdefault("v." + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] * g[k]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)


def subspace_loss(N: np.ndarray, X: np.ndarray) -> float:
    """Share of the unit-norm solutions outside span(N): (1/s) sum_c ||x^_c - P x^_c||^2 with
    x^_c = x_c / ||x_c|| and P the orthogonal projector onto span(N) (N: n x k, X: n x s).
    The projection is a least-squares fit of each column on N."""
    Xh = X / np.linalg.norm(X, axis=0)
    coef = np.linalg.lstsq(N, Xh, rcond=None)[0]
    R = Xh - N @ coef
    return float((R * R).sum() / X.shape[1])


def subspace_loss_grad(N: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Gradient of subspace_loss w.r.t. N: -(2/s) R (N^T X^)^T (N^T N)^{-1}, with R the
    residual block (differentiating the projector N (N^T N)^{-1} N^T)."""
    Xh = X / np.linalg.norm(X, axis=0)
    G = N.T @ N
    C = N.T @ Xh
    R = Xh - N @ np.linalg.solve(G, C)
    return -2.0 / X.shape[1] * R @ np.linalg.solve(G, C).T
