"""Device-resident problems driven through the C ABI (torch supplies memory and stream).

Nothing here computes: it sizes and allocates the caller-owned buffers the ABI asks
for, calls rom_assemble_operator / rom_solve_sequence / rom_reduced_transfer /
rom_apply_operator, and hands back torch views of what the library wrote.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import rom as R


@dataclass
class SequenceResult:
    status: int
    basis: int
    records: List[dict]
    stats: dict
    workspace: Optional[torch.Tensor]  # owns the basis memory (released by close)
    X: Optional[torch.Tensor]          # (K * n_rhs, N): row i*n_rhs + j is solution (i, j)
    n: int
    m: int

    def Q(self) -> torch.Tensor:
        """Copy of the global basis as an (m, N) tensor (row c = column c of V)."""
        out = torch.empty((self.m, self.n), dtype=torch.float64, device=self.workspace.device)
        R.rom_basis_copy(self.basis, out)
        return out

    def close(self):
        """Destroys the basis handle and drops the workspace it lived in and the solutions
        (a 128^3 sequence in groups holds tens of GB)."""
        if self.basis:
            R.rom_basis_destroy(self.basis)
            self.basis = 0
        self.workspace = None
        self.X = None


class Problem:
    """One assembled operator A_* with its sources, detectors and recycle seed U_0."""

    def __init__(self, dim: int, N: Sequence[int], bc: Sequence[int], robin_A: float, D,
                 src_idx, src_scale, det_idx, det_scale, U0: Optional[np.ndarray],
                 device="cuda:0"):
        self.device = torch.device(device)
        self.dim = dim
        self.N = tuple(int(x) for x in N) + (1,) * (3 - len(N))
        self.n = int(np.prod(self.N))
        self.grid = R.make_grid(dim, self.N, bc, robin_A)
        var = not np.isscalar(D)
        self.op_mem = torch.empty(R.rom_operator_bytes(self.grid, var), dtype=torch.uint8,
                                  device=self.device)
        self.D_field = torch.as_tensor(np.asarray(D, dtype=np.float64), device=self.device) if var else None
        self.op = R.rom_assemble_operator(self.grid, 0.0 if var else float(D), self.D_field,
                                          self.op_mem)
        self.src_idx = np.asarray(src_idx, dtype=np.int64)
        self.src_scale = np.asarray(src_scale, dtype=np.float64)
        self.det_idx = np.asarray(det_idx, dtype=np.int64)
        self.det_scale = np.asarray(det_scale, dtype=np.float64)
        self.k_u = 0 if U0 is None else int(U0.shape[1])
        # column-major N x k_u == row-major k_u x N
        self.U0 = None if U0 is None or self.k_u == 0 else torch.as_tensor(
            np.ascontiguousarray(np.asarray(U0, dtype=np.float64).T), device=self.device)

    def set_U0(self, U: Optional[torch.Tensor]) -> None:
        """Use the rows of U ((k_u, N), e.g. rom_lowest_modes' eigenvectors of A(p_0)) as
        the recycle seed U_0 of later sequences (None: no seed)."""
        if U is None or U.shape[0] == 0:
            self.U0, self.k_u = None, 0
            return
        assert U.dim() == 2 and U.shape[1] == self.n
        self.U0 = U.to(dtype=torch.float64, device=self.device).contiguous()
        self.k_u = int(U.shape[0])

    @property
    def n_rhs(self) -> int:
        return self.src_idx.size + self.det_idx.size

    def solve(self, points: List[R.MuParams], tol: float, trunc: float = 1e-8, cap: int = 0,
              maxit: int = 0, check_every: int = 0, timing: int = 0,
              keep_X: bool = True, precision: int = R.ROM_PREC_FP64,
              inner_tol: float = 0.0, group: int = 0, tune: int = 0,
              graph: int = 0, guess: Optional[torch.Tensor] = None,
              recycle: Optional[torch.Tensor] = None, cg_step: int = 0) -> SequenceResult:
        """recycle: (K, n_recycle, N) FP32 learned recycle vectors per point (they join the
        recycle spaces U_j at their point), or None."""
        if recycle is not None:
            assert recycle.dim() == 3 and recycle.shape[0] == len(points) and \
                recycle.shape[2] == self.n and recycle.dtype == torch.float32
            recycle = recycle.contiguous()
        opts = R.make_opts(tol, trunc, cap, maxit, check_every, timing, precision, inner_tol,
                           group, tune, graph, guess, recycle, cg_step)
        K = len(points)
        nbytes = R.rom_sequence_bytes(self.op, self.src_idx.size, self.det_idx.size, self.k_u, K, opts)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        X = torch.empty((K * self.n_rhs, self.n), dtype=torch.float64, device=self.device) if keep_X else None
        status, basis, records, st = R.rom_solve_sequence(
            self.op, points, self.src_idx, self.src_scale, self.det_idx, self.det_scale, self.U0,
            self.k_u, opts, ws, X)
        n, m = R.rom_basis_dims(basis)
        return SequenceResult(status, basis, records, R.stats_dict(st), ws, X, n, m)

    def stream(self, K: int, tol: float, trunc: float = 1e-8, cap: int = 0, **kw) -> "SequenceStream":
        """A sequence taken one parameter point at a time (rom_sequence_begin): at most K
        points; kw as for solve (precision, group, tune, timing, guess, recycle...)."""
        opts = R.make_opts(tol, trunc, cap, kw.pop("maxit", 0), kw.pop("check_every", 0),
                           kw.pop("timing", 0), kw.pop("precision", R.ROM_PREC_FP64),
                           kw.pop("inner_tol", 0.0), kw.pop("group", 0), kw.pop("tune", 0),
                           kw.pop("graph", 0), kw.pop("guess", None), kw.pop("recycle", None),
                           kw.pop("cg_step", 0))
        assert not kw, kw
        nbytes = R.rom_sequence_bytes(self.op, self.src_idx.size, self.det_idx.size, self.k_u, K, opts)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = R.rom_sequence_begin(self.op, K, self.src_idx, self.src_scale, self.det_idx,
                                 self.det_scale, self.U0, self.k_u, opts, ws)
        return SequenceStream(self, h, ws)

    def reduced(self, res: SequenceResult, p: R.MuParams):
        """(A_r, B_r, C_r, E_r) of eq. (newreduced) as float64 tensors (column-major
        buffers returned as their row-major transposes, i.e. A_r^T = A_r etc.)."""
        m = res.m
        dev = self.device
        Ar = torch.empty((m, m), dtype=torch.float64, device=dev)
        Er = torch.empty((m, m), dtype=torch.float64, device=dev)
        Br = torch.empty((self.src_idx.size, m), dtype=torch.float64, device=dev)
        Cr = torch.empty((self.det_idx.size, m), dtype=torch.float64, device=dev)
        scratch = torch.empty(R.rom_reduced_bytes(res.basis), dtype=torch.uint8, device=dev)
        R.rom_reduced_transfer(res.basis, p, Ar, Br, Cr, Er, scratch)
        # column-major m x m read as row-major is the transpose; B_r (m x n_src col-major)
        # read row-major is (n_src x m) = B_r^T
        return Ar.T.contiguous(), Br.T.contiguous(), Cr.T.contiguous(), Er.T.contiguous()

    def reduced_jacobian(self, res: SequenceResult, p: R.MuParams) -> torch.Tensor:
        """d Psi_r / d p_k for every bump parameter of p (per bump: amplitude, radius,
        centre coordinates) as a float64 tensor (nparams, n_det, n_src)."""
        dev = self.device
        ns, nd = self.src_idx.size, self.det_idx.size
        npar = int(np.asarray(p.radii).size) * (self.dim + 2)
        J = torch.empty((npar, ns, nd), dtype=torch.float64, device=dev)
        scratch = torch.empty(R.rom_reduced_jacobian_bytes(res.basis), dtype=torch.uint8,
                              device=dev)
        R.rom_reduced_jacobian(res.basis, p, J, scratch)
        # each block is n_det x n_src column-major = (n_src, n_det) row-major
        return J.transpose(1, 2).contiguous()

    def reduced_response(self, res: SequenceResult, p: R.MuParams, sigma) -> torch.Tensor:
        """Psi_r(sigma) = C_r^T (i sigma I + A_r(p))^{-1} B_r for each shift sigma = omega/nu,
        as a complex128 tensor (ns, n_det, n_src)."""
        dev = self.device
        sig = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
        ns, nd = self.src_idx.size, self.det_idx.size
        Pr = torch.empty((sig.size, ns, nd), dtype=torch.float64, device=dev)
        Pi = torch.empty_like(Pr)
        scratch = torch.empty(R.rom_reduced_response_bytes(res.basis), dtype=torch.uint8,
                              device=dev)
        R.rom_reduced_response(res.basis, p, sig, Pr, Pi, scratch)
        # each block is n_det x n_src column-major = (n_src, n_det) row-major
        return torch.complex(Pr, Pi).transpose(1, 2).contiguous()

    def shifted_solve(self, p: R.MuParams, B: torch.Tensor, sigma, tol: float = 1e-8,
                      maxit: int = 0, allow_noconv: bool = False):
        """(A(p) + i sigma I) X = B for the columns of B ((nb, N) rows) and every shift:
        returns (X complex128 (ns, nb, N), its (nb,), true relative residuals (ns, nb),
        status)."""
        dev = self.device
        B = B.to(dtype=torch.float64, device=dev).contiguous()
        nb = B.shape[0]
        sig = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
        Xr = torch.empty((sig.size, nb, self.n), dtype=torch.float64, device=dev)
        Xi = torch.empty_like(Xr)
        scratch = torch.empty(R.rom_shifted_solve_bytes(self.op, nb, sig.size),
                              dtype=torch.uint8, device=dev)
        st, its, res = R.rom_shifted_solve(self.op, p, B, nb, sig, tol, maxit or self.n, Xr, Xi,
                                           scratch, allow_noconv=allow_noconv)
        return torch.complex(Xr, Xi), its, res, st

    def lowest_modes(self, p: R.MuParams, k: int, X0: torch.Tensor, tol: float = 1e-8,
                     maxit: int = 200, allow_noconv: bool = False):
        """The k smallest eigenpairs of A(p) from the starting block X0 ((kx, N) rows, kx >= k
        columns): returns (U as (k, N) rows, eigenvalues (k,), sweeps), plus the status with
        allow_noconv (ROM_ENOCONV when the residual test did not pass within maxit)."""
        X0 = X0.to(dtype=torch.float64, device=self.device).contiguous()
        kx = X0.shape[0]
        U = torch.empty((k, self.n), dtype=torch.float64, device=self.device)
        scratch = torch.empty(R.rom_lowest_modes_bytes(self.op, kx), dtype=torch.uint8,
                              device=self.device)
        out = R.rom_lowest_modes(self.op, p, k, X0, kx, tol, maxit, U, scratch,
                                 allow_noconv=allow_noconv)
        return (U,) + tuple(out)

    def apply(self, p: R.MuParams, X: torch.Tensor) -> torch.Tensor:
        """Y = A(p) X for X given as (k, N) rows (each row a vector)."""
        X = X.contiguous()
        Y = torch.empty_like(X)
        scratch = torch.empty(8 * self.n, dtype=torch.uint8, device=self.device)
        R.rom_apply_operator(self.op, p, X, Y, X.shape[0], scratch)
        return Y

    def close(self):
        if self.op:
            R.rom_operator_destroy(self.op)
            self.op = 0


class SequenceStream:
    """Algorithm 2 fed one point at a time (rom_sequence_point); the basis so far is a
    view (rom_sequence_basis) until end() returns the final SequenceResult."""

    def __init__(self, prob: Problem, handle, workspace: torch.Tensor):
        self.prob = prob
        self.h = handle
        self.workspace = workspace
        self.records: List[dict] = []

    def point(self, p: R.MuParams, X: Optional[torch.Tensor] = None):
        """Solve point p; X ((n_rhs, N) float64, or None) receives its solutions."""
        status, recs = R.rom_sequence_point(self.h, p, X)
        self.records.extend(recs)
        return status, recs

    def basis_view(self) -> int:
        return R.rom_sequence_basis(self.h)

    def stats(self) -> dict:
        """Totals so far (stats_dict of rom_sequence_stats)."""
        return R.stats_dict(R.rom_sequence_stats(self.h))

    def end(self) -> SequenceResult:
        basis, st = R.rom_sequence_end(self.h)
        n, m = R.rom_basis_dims(basis)
        stats = R.stats_dict(st)
        status = R.ROM_ENOCONV if stats["n_nonconv"] else R.ROM_OK
        return SequenceResult(status, basis, self.records, stats, self.workspace, None, n, m)


def solve_many(problems: List["Problem"], points: List[List[R.MuParams]], tol: float,
               trunc: float = 1e-8, keep_X: bool = False, streams=None,
               **opt_kw) -> List[SequenceResult]:
    """Independent sequences (e.g. one per grid) solved concurrently, each on its own
    stream (created here unless given) and host thread (rom_solve_sequences)."""
    jobs = []
    if streams is None:
        streams = [torch.cuda.Stream(device=p.device) for p in problems]
    opt_kw = dict(opt_kw)
    for prob, pts, stream in zip(problems, points, streams):
        cap = opt_kw.get("cap", 0)
        opts = R.make_opts(tol, trunc, cap, opt_kw.get("maxit", 0), opt_kw.get("check_every", 0),
                           opt_kw.get("timing", 0), opt_kw.get("precision", R.ROM_PREC_FP64),
                           opt_kw.get("inner_tol", 0.0), opt_kw.get("group", 0),
                           opt_kw.get("tune", 0), opt_kw.get("graph", 0),
                           cg_step=opt_kw.get("cg_step", 0))
        K = len(pts)
        nbytes = R.rom_sequence_bytes(prob.op, prob.src_idx.size, prob.det_idx.size, prob.k_u, K,
                                      opts)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=prob.device)
        X = torch.empty((K * prob.n_rhs, prob.n), dtype=torch.float64,
                        device=prob.device) if keep_X else None
        jobs.append(dict(op=prob.op, params=pts, src_idx=prob.src_idx, src_scale=prob.src_scale,
                         det_idx=prob.det_idx, det_scale=prob.det_scale, U0=prob.U0, k_u=prob.k_u,
                         opts=opts, workspace=ws, X_out=X, stream=stream))
    torch.cuda.synchronize()     # inputs resident before the other streams read them
    outs = R.rom_solve_sequences(jobs)
    res = []
    for jb, (status, basis, records, st) in zip(jobs, outs):
        n, m = R.rom_basis_dims(basis)
        res.append(SequenceResult(status, basis, records, R.stats_dict(st), jb["workspace"],
                                  jb["X_out"], n, m))
    return res


def problem_from_workload(wl, device="cuda:0", k_u: Optional[int] = None) -> Problem:
    """Build a Problem from a phantoms.Workload (seeded synthetic inputs)."""
    import phantoms as ph
    D = ph.diffusion_field(wl)
    s, d = ph.rhs_nodes(wl)
    ss, ds = ph.rhs_scales(wl)
    U0 = ph.smooth_modes(wl, k_u)
    return Problem(wl.dim, wl.N, wl.bc, wl.robin_A, D, s, ss, d, ds, U0, device=device)


def points_from_workload(wl, K: Optional[int] = None, mode: str = "independent") -> List[R.MuParams]:
    import phantoms as ph
    return [R.MuParams(p.mu0, p.centers, p.radii, p.amps)
            for p in ph.parameter_points(wl, K=K, mode=mode)]
