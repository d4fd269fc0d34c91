"""Shared test helpers: run the CPU oracle on a phantoms workload."""
from __future__ import annotations

import numpy as np

import phantoms as ph
from oracle import operator as op
from oracle import rom as orom
from oracle import sequence as oseq


class OracleProblem:
    def __init__(self, wl, mode="independent", K=None, k_u=None):
        self.wl = wl
        self.D = ph.diffusion_field(wl)
        self.As = op.assemble_Astar(wl.dim, wl.N, wl.bc, self.D, wl.robin_A)
        self.pts = ph.parameter_points(wl, K=K, mode=mode)
        self.mus = [op.mu_field(wl.dim, wl.N, p.mu0, p.centers, p.radii, p.amps) for p in self.pts]
        si, di = ph.rhs_nodes(wl)
        ss, ds = ph.rhs_scales(wl)
        self.B = oseq.rhs_matrix(wl.n, si, ss, di, ds)
        self.U0 = ph.smooth_modes(wl, k_u)

    def A(self, i):
        return op.assemble_A(self.As, self.mus[i])

    def run(self, tol=None, trunc=None, cap=0, mus=None, group=1):
        wl = self.wl
        return oseq.solve_sequence(self.As, mus if mus is not None else self.mus, self.B, self.U0,
                                   wl.tol if tol is None else tol,
                                   wl.trunc if trunc is None else trunc, cap=cap, group=group)

    def psi(self, i):
        ns = self.wl.n_src
        if ns == 0 or self.wl.n_det == 0:
            return np.zeros((self.wl.n_det, ns))
        return orom.full_transfer(self.A(i), self.B[:, :ns], self.B[:, ns:])


def principal_cosines(Qa: np.ndarray, Qb: np.ndarray) -> np.ndarray:
    """Cosines of the principal angles between range(Qa) and range(Qb) (orthonormal)."""
    return np.linalg.svd(Qa.T @ Qb, compute_uv=False)
