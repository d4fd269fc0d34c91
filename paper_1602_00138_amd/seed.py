"""Learned seed: the network object over caller-owned torch buffers (rom_seednet_*), and
the flat parameter layout shared with the reference implementation."""
from __future__ import annotations

from typing import Dict

import numpy as np
import torch

from . import rom as R

LAYERS = (("e0", 3, 16), ("e1", 16, 32), ("e2", 32, 48), ("e3", 48, 64),
          ("d2", 64, 48), ("d1", 48, 32), ("d0", 32, 16), ("head", 16, 1))


def flatten(params: Dict[str, np.ndarray]) -> np.ndarray:
    """Per layer: weights (o, i, 3, 3, 3) then biases (o), in network order."""
    out = []
    for name, _, _ in LAYERS:
        out.append(np.asarray(params[name + ".w"], dtype=np.float64).reshape(-1))
        out.append(np.asarray(params[name + ".b"], dtype=np.float64).reshape(-1))
    return np.concatenate(out)


def unflatten(flat: np.ndarray) -> Dict[str, np.ndarray]:
    p, k = {}, 0
    for name, ci, co in LAYERS:
        nw = co * ci * 27
        p[name + ".w"] = np.asarray(flat[k:k + nw], dtype=np.float64).reshape(co, ci, 3, 3, 3)
        k += nw
        p[name + ".b"] = np.asarray(flat[k:k + co], dtype=np.float64)
        k += co
    return p


def he_init(seed: int) -> np.ndarray:
    """He-normal weights and zero biases from a seeded generator (flat layout)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in LAYERS:
        p[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci))
        p[name + ".b"] = np.zeros(co)
    return flatten(p)


class SeedNet:
    def __init__(self, grid, batch: int, params: np.ndarray, device="cuda:0"):
        self.grid = tuple(int(g) for g in grid)
        self.batch = int(batch)
        nx, ny, nz = self.grid
        self.nparams, pb, wb = R.rom_seednet_bytes(nx, ny, nz, batch)
        self.pmem = torch.empty(pb, dtype=torch.uint8, device=device)
        self.wmem = torch.empty(wb, dtype=torch.uint8, device=device)
        self.net = R.rom_seednet_create(nx, ny, nz, batch, params, self.pmem, self.wmem)
        self.n = nx * ny * nz

    def forward(self, inputs: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
        b = inputs.shape[0]
        if out is None:
            out = torch.empty((b, self.n), dtype=torch.float32, device=inputs.device)
        R.rom_seednet_forward(self.net, inputs.contiguous(), out, b)
        return out

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
