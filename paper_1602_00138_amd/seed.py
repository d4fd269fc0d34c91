"""Learned seed: the network object over caller-owned torch buffers (rom_seednet_*), and
the flat parameter layout shared with the reference implementation."""
from __future__ import annotations

from typing import Dict

import numpy as np
import torch

from . import rom as R

def layers(outputs: int = 1):
    """(name, in, out) per layer; the head has `outputs` channels (1: the guess network, up
    to 16: the recycle-vector network)."""
    return (("e0", 3, 16), ("e1", 16, 32), ("e2", 32, 48), ("e3", 48, 64),
            ("d2", 64, 48), ("d1", 48, 32), ("d0", 32, 16), ("head", 16, outputs))


LAYERS = layers(1)


def flatten(params: Dict[str, np.ndarray]) -> np.ndarray:
    """Per layer: weights (o, i, 3, 3, 3) then biases (o), in network order."""
    out = []
    outputs = np.asarray(params["head.b"]).size
    for name, _, _ in layers(outputs):
        out.append(np.asarray(params[name + ".w"], dtype=np.float64).reshape(-1))
        out.append(np.asarray(params[name + ".b"], dtype=np.float64).reshape(-1))
    return np.concatenate(out)


def unflatten(flat: np.ndarray, outputs: int = 1) -> Dict[str, np.ndarray]:
    p, k = {}, 0
    for name, ci, co in layers(outputs):
        nw = co * ci * 27
        p[name + ".w"] = np.asarray(flat[k:k + nw], dtype=np.float64).reshape(co, ci, 3, 3, 3)
        k += nw
        p[name + ".b"] = np.asarray(flat[k:k + co], dtype=np.float64)
        k += co
    return p


def he_init(seed: int, outputs: int = 1) -> np.ndarray:
    """He-normal weights and zero biases from a seeded generator (flat layout)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in layers(outputs):
        p[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci))
        p[name + ".b"] = np.zeros(co)
    return flatten(p)


class SeedNet:
    def __init__(self, grid, batch: int, params: np.ndarray, device="cuda:0", outputs: int = 1):
        self.grid = tuple(int(g) for g in grid)
        self.batch = int(batch)
        self.outputs = int(outputs)
        nx, ny, nz = self.grid
        self.nparams, pb, wb = R.rom_seednet_bytes(nx, ny, nz, batch, self.outputs)
        self.pmem = torch.empty(pb, dtype=torch.uint8, device=device)
        self.wmem = torch.empty(wb, dtype=torch.uint8, device=device)
        self.net = R.rom_seednet_create(nx, ny, nz, batch, params, self.pmem, self.wmem,
                                        outputs=self.outputs)
        self.n = nx * ny * nz

    def forward(self, inputs: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
        """[b][N] for a one-output network, [b][outputs][N] otherwise."""
        b = inputs.shape[0]
        if out is None:
            shape = (b, self.n) if self.outputs == 1 else (b, self.outputs, self.n)
            out = torch.empty(shape, dtype=torch.float32, device=inputs.device)
        R.rom_seednet_forward(self.net, inputs.contiguous(), out, b)
        return out

    def backward(self, inputs: torch.Tensor, dy: torch.Tensor, grads: bool = False):
        """Propagate the output gradient dy back; returns the parameter gradient if asked."""
        return R.rom_seednet_backward(self.net, inputs.contiguous(), dy.contiguous(),
                                      inputs.shape[0], self.nparams if grads else 0)

    def adam(self, lr: float) -> None:
        R.rom_seednet_adam(self.net, lr)

    def gradients(self, inputs: torch.Tensor, targets: torch.Tensor):
        return R.rom_seednet_gradients(self.net, inputs.contiguous(), targets.contiguous(),
                                       inputs.shape[0], self.nparams)

    def train_step(self, inputs: torch.Tensor, targets: torch.Tensor, lr: float) -> float:
        return R.rom_seednet_train_step(self.net, inputs.contiguous(), targets.contiguous(),
                                        inputs.shape[0], lr)

    def params(self) -> np.ndarray:
        return R.rom_seednet_params(self.net, self.nparams)

    def close(self):
        R.rom_seednet_destroy(self.net)
        self.net = 0


def make_inputs(prob, point: R.MuParams, idx: np.ndarray, out: torch.Tensor = None,
                scratch: torch.Tensor = None) -> torch.Tensor:
    """Network inputs [count][3][N] for the right-hand sides at nodes idx at one point
    (rom_seednet_inputs)."""
    idx = np.asarray(idx, dtype=np.int64)
    dev = prob.device
    if out is None:
        out = torch.empty((idx.size, 3, prob.n), dtype=torch.float32, device=dev)
    if scratch is None:
        scratch = torch.empty(8 * (prob.n + idx.size), dtype=torch.uint8, device=dev)
    R.rom_seednet_inputs(prob.op, point, idx, out, scratch)
    return out


def make_targets(X: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    """Targets x / max|x| (FP32 [count][N]) from FP64 solutions X (count, N)."""
    count, n = X.shape
    if out is None:
        out = torch.empty((count, n), dtype=torch.float32, device=X.device)
    scratch = torch.empty(512 * count, dtype=torch.uint8, device=X.device)
    R.rom_seednet_targets(X, n, n, count, out, scratch)
    return out


def rhs_nodes(prob) -> np.ndarray:
    return np.concatenate([prob.src_idx, prob.det_idx])


def dataset(prob, points, tol: float, keep_solutions: bool = False, **solve_kw):
    """Training pairs from the method's own solutions: run the sequence on `points` and
    return (inputs [K n_rhs][3][N], targets [K n_rhs][N]), and the FP64 solutions
    (K n_rhs, N) as a third item if keep_solutions."""
    res = prob.solve(points, tol, keep_X=True, **solve_kw)
    X = res.X
    res.close()
    idx = rhs_nodes(prob)
    inputs = torch.empty((len(points) * idx.size, 3, prob.n), dtype=torch.float32,
                         device=prob.device)
    for i, p in enumerate(points):
        make_inputs(prob, p, idx, out=inputs[i * idx.size:(i + 1) * idx.size])
    targets = make_targets(X)
    if keep_solutions:
        return inputs, targets, X
    del X
    return inputs, targets


def train(net: SeedNet, inputs: torch.Tensor, targets: torch.Tensor, steps: int, lr: float,
          seed: int = 0, log=None):
    """Adam on shuffled minibatches of net.batch samples; returns the losses."""
    rng = np.random.default_rng(seed)
    n = inputs.shape[0]
    order = rng.permutation(n)
    losses = []
    pos = 0
    for s in range(steps):
        if pos + net.batch > n:
            order = rng.permutation(n)
            pos = 0
        sel = torch.as_tensor(order[pos:pos + net.batch], device=inputs.device)
        pos += net.batch
        losses.append(net.train_step(inputs.index_select(0, sel), targets.index_select(0, sel), lr))
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"seed network step {s}: loss {losses[-1]:.4e}")
    return losses


def guesses(net: SeedNet, prob, points) -> torch.Tensor:
    """Network guesses for every (point, right-hand side), FP32 [K n_rhs][N]."""
    idx = rhs_nodes(prob)
    K = len(points)
    out = torch.empty((K * idx.size, prob.n), dtype=torch.float32, device=prob.device)
    inp = torch.empty((idx.size, 3, prob.n), dtype=torch.float32, device=prob.device)
    scratch = torch.empty(8 * (prob.n + idx.size), dtype=torch.uint8, device=prob.device)
    for i, p in enumerate(points):
        make_inputs(prob, p, idx, out=inp, scratch=scratch)
        for b0 in range(0, idx.size, net.batch):
            b1 = min(idx.size, b0 + net.batch)
            net.forward(inp[b0:b1], out=out[i * idx.size + b0:i * idx.size + b1])
    return out


# ---- recycle-vector network (second output) -------------------------------------------
# A network with 16 outputs maps the point-only fields [(mu - mu0)/0.03, log(D/0.03), 0] to
# 16 vectors per parameter point.  It is trained with the subspace loss (the share of the
# point's unit-norm solutions outside the span of the 16 outputs, rom_subspace_loss), and
# its outputs join the recycle spaces U_j of every right-hand side at that point.

def point_inputs(prob, points, out: torch.Tensor = None) -> torch.Tensor:
    """Network inputs [K][3][N] without a source indicator (rom_seednet_inputs, idx -1)."""
    K = len(points)
    dev = prob.device
    if out is None:
        out = torch.empty((K, 3, prob.n), dtype=torch.float32, device=dev)
    scratch = torch.empty(8 * (prob.n + 1), dtype=torch.uint8, device=dev)
    for i, p in enumerate(points):
        R.rom_seednet_inputs(prob.op, p, np.array([-1], dtype=np.int64), out[i:i + 1], scratch)
    return out


def recycle_dataset(prob, points, tol: float, **solve_kw):
    """(inputs [K][3][N], solutions (K n_rhs, N) FP64) from the method's own solves."""
    res = prob.solve(points, tol, keep_X=True, **solve_kw)
    X = res.X
    res.close()
    return point_inputs(prob, points), X


def train_recycle(net: SeedNet, inputs: torch.Tensor, X: torch.Tensor, n_rhs: int, steps: int,
                  lr: float, seed: int = 0, log=None):
    """Adam on the subspace loss over minibatches of net.batch points; the batch loss is the
    sum of the per-point losses (Adam does not see its scale).  Returns the mean per-point
    loss of every step."""
    rng = np.random.default_rng(seed)
    K, n = inputs.shape[0], inputs.shape[2]
    k = net.outputs
    dev = inputs.device
    Y = torch.empty((net.batch, k, n), dtype=torch.float32, device=dev)
    dY = torch.empty_like(Y)
    scratch = torch.empty(R.rom_subspace_loss_bytes(n, k, n_rhs), dtype=torch.uint8, device=dev)
    order = rng.permutation(K)
    pos = 0
    losses = []
    for s in range(steps):
        b = min(net.batch, K)
        if pos + b > K:
            order = rng.permutation(K)
            pos = 0
        sel = order[pos:pos + b]
        pos += b
        inp = inputs.index_select(0, torch.as_tensor(sel, device=dev))
        net.forward(inp, out=Y[:b])
        tot = 0.0
        for t, i in enumerate(sel):
            Xi = X[i * n_rhs:(i + 1) * n_rhs]          # N x n_rhs, column-major
            tot += R.rom_subspace_loss(Y[t], k, Xi, n, n, n_rhs, dY[t], scratch)
        net.backward(inp, dY[:b])
        net.adam(lr)
        losses.append(tot / b)
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"recycle network step {s}: subspace loss {losses[-1]:.4e}")
    return losses


def recycle_vectors(net: SeedNet, prob, points) -> torch.Tensor:
    """The network's recycle vectors for every point, FP32 (K, outputs, N)."""
    inp = point_inputs(prob, points)
    K = len(points)
    out = torch.empty((K, net.outputs, prob.n), dtype=torch.float32, device=prob.device)
    for b0 in range(0, K, net.batch):
        b1 = min(K, b0 + net.batch)
        net.forward(inp[b0:b1], out=out[b0:b1])
    return out
