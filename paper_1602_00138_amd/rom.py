"""Thin ctypes binding of the C ABI in include/rom.h (librom.so, gfx950).

Every function here has the name of the C entry point it marshals to and does
nothing but argument conversion: device buffers are torch tensors (their data
pointers are passed), the stream is torch's current stream unless given.  All
arithmetic of the method runs in the library's HIP kernels.  Importing this
module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librom.so")

ROM_OK = 0
ROM_EINVAL = -1
ROM_ENOTSPD = -2
ROM_ENONFINITE = -3
ROM_ENOCONV = -4
ROM_ECAPACITY = -5
ROM_EHIP = -6
ROM_NJ_MAX = 64
ROM_STATIC_MAX_N = 1 << 21
ROM_MAX_BUMPS = 64
ROM_PREC_FP64 = 0
ROM_PREC_MIXED = 1

(ROM_K_DCG_OP, ROM_K_DCG_UPDATE, ROM_K_DCG_ENDS, ROM_K_GEMVT, ROM_K_GEMVN, ROM_K_GRAM, ROM_K_OUTER,
 ROM_K_OTHER, ROM_K_DCG_STEP) = range(9)
ROM_NK = 9
KERNEL_CLASSES = ["dcg_op", "dcg_update", "dcg_ends", "gemvt", "gemvn", "gram", "outer", "other",
                  "dcg_step"]

EXPORTED = ["rom_operator_bytes", "rom_assemble_operator", "rom_apply_operator",
            "rom_apply_operator_static", "rom_sequence_bytes", "rom_sequence_begin",
            "rom_sequence_point", "rom_sequence_basis", "rom_sequence_stats", "rom_sequence_end",
            "rom_solve_sequence", "rom_solve_sequences", "rom_reduced_bytes", "rom_reduced_transfer",
            "rom_reduced_jacobian_bytes", "rom_reduced_jacobian", "rom_lowest_modes_bytes",
            "rom_lowest_modes", "rom_shifted_solve_bytes", "rom_shifted_solve",
            "rom_reduced_response_bytes", "rom_reduced_response", "rom_basis_dims",
            "rom_basis_copy", "rom_operator_destroy", "rom_basis_destroy", "rom_last_error",
            "rom_seednet_bytes", "rom_seednet_create", "rom_seednet_forward",
            "rom_seednet_gradients", "rom_seednet_train_step", "rom_seednet_backward",
            "rom_seednet_adam", "rom_seednet_params", "rom_subspace_loss_bytes",
            "rom_subspace_loss",
            "rom_seednet_destroy", "rom_seednet_inputs", "rom_seednet_targets"]


class rom_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("bc", C.c_int * 6), ("robin_A", C.c_double)]


class rom_mu(C.Structure):
    _fields_ = [("nb", C.c_int), ("centers", C.POINTER(C.c_double)),
                ("radii", C.POINTER(C.c_double)), ("amps", C.POINTER(C.c_double)),
                ("mu0", C.c_double)]


class rom_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("trunc", C.c_double), ("inner_tol", C.c_double),
                ("cap", C.c_int), ("maxit", C.c_int), ("check_every", C.c_int), ("timing", C.c_int),
                ("precision", C.c_int), ("group", C.c_int), ("tune", C.c_int), ("graph", C.c_int),
                ("guess", C.c_void_p), ("recycle", C.c_void_p), ("n_recycle", C.c_int),
                ("cg_step", C.c_int)]


class rom_record(C.Structure):
    _fields_ = [("point", C.c_int), ("rhs", C.c_int), ("rho0", C.c_double), ("its", C.c_int),
                ("solved", C.c_int), ("kept", C.c_int), ("rho", C.c_double),
                ("final_res", C.c_double), ("m", C.c_int), ("restarts", C.c_int),
                ("converged", C.c_int), ("fp64_sweeps", C.c_int), ("rho_guess", C.c_double)]


class rom_stats(C.Structure):
    _fields_ = [("m", C.c_int), ("k_u", C.c_int), ("n_solved", C.c_int), ("n_kept", C.c_int),
                ("n_dropped_trunc", C.c_int), ("n_dropped_cap", C.c_int),
                ("n_nonconv", C.c_int), ("total_its", C.c_longlong), ("seconds", C.c_double),
                ("kernel_ms", C.c_double * ROM_NK), ("kernel_bytes", C.c_double * ROM_NK),
                ("kernel_flops", C.c_double * ROM_NK), ("kernel_launches", C.c_longlong * ROM_NK),
                ("n_uj_capped", C.c_int)]


class rom_sequence_job(C.Structure):
    _fields_ = [("op", C.c_void_p), ("params", C.POINTER(rom_mu)), ("K", C.c_int),
                ("src_idx", C.POINTER(C.c_int64)), ("src_scale", C.POINTER(C.c_double)),
                ("n_src", C.c_int), ("det_idx", C.POINTER(C.c_int64)),
                ("det_scale", C.POINTER(C.c_double)), ("n_det", C.c_int), ("U0", C.c_void_p),
                ("k_u", C.c_int), ("opts", C.POINTER(rom_opts)), ("workspace", C.c_void_p),
                ("ws_bytes", C.c_size_t), ("basis", C.POINTER(C.c_void_p)), ("X_out", C.c_void_p),
                ("records", C.POINTER(rom_record)), ("stats", C.POINTER(rom_stats)),
                ("stream", C.c_void_p), ("status", C.c_int), ("message", C.c_char * 192)]


class RomError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rom status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_1602_00138_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    P = C.POINTER
    sig = {
        "rom_operator_bytes": (C.c_int, [P(rom_grid), C.c_int, P(sz)]),
        "rom_assemble_operator": (C.c_int, [P(rom_grid), C.c_double, vp, vp, sz, P(vp), vp]),
        "rom_apply_operator": (C.c_int, [vp, P(rom_mu), vp, vp, C.c_int, vp, sz, vp]),
        "rom_apply_operator_static": (C.c_int, [vp, P(rom_mu), vp, vp, C.c_int, vp]),
        "rom_sequence_bytes": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, P(rom_opts), P(sz)]),
        "rom_solve_sequence": (C.c_int, [vp, P(rom_mu), C.c_int, P(C.c_int64), P(C.c_double), C.c_int,
                                         P(C.c_int64), P(C.c_double), C.c_int, vp, C.c_int,
                                         P(rom_opts), vp, sz, P(vp), vp, P(rom_record),
                                         P(rom_stats), vp]),
        "rom_solve_sequences": (C.c_int, [P(rom_sequence_job), C.c_int]),
        "rom_sequence_begin": (C.c_int, [vp, C.c_int, P(C.c_int64), P(C.c_double), C.c_int,
                                         P(C.c_int64), P(C.c_double), C.c_int, vp, C.c_int,
                                         P(rom_opts), vp, sz, P(vp), vp]),
        "rom_sequence_point": (C.c_int, [vp, P(rom_mu), vp, P(rom_record)]),
        "rom_sequence_basis": (C.c_int, [vp, P(vp)]),
        "rom_sequence_stats": (C.c_int, [vp, P(rom_stats)]),
        "rom_sequence_end": (C.c_int, [vp, P(vp), P(rom_stats)]),
        "rom_reduced_bytes": (C.c_int, [vp, P(sz)]),
        "rom_reduced_transfer": (C.c_int, [vp, P(rom_mu), vp, vp, vp, vp, vp, sz, vp]),
        "rom_reduced_jacobian_bytes": (C.c_int, [vp, P(sz)]),
        "rom_reduced_jacobian": (C.c_int, [vp, P(rom_mu), vp, vp, sz, vp]),
        "rom_lowest_modes_bytes": (C.c_int, [vp, C.c_int, P(sz)]),
        "rom_shifted_solve_bytes": (C.c_int, [vp, C.c_int, C.c_int, P(sz)]),
        "rom_shifted_solve": (C.c_int, [vp, P(rom_mu), vp, C.c_int, P(C.c_double), C.c_int,
                                        C.c_double, C.c_int, vp, vp, P(C.c_int),
                                        P(C.c_double), vp, sz, vp]),
        "rom_reduced_response_bytes": (C.c_int, [vp, P(sz)]),
        "rom_reduced_response": (C.c_int, [vp, P(rom_mu), P(C.c_double), C.c_int, vp, vp, vp,
                                           sz, vp]),
        "rom_lowest_modes": (C.c_int, [vp, P(rom_mu), C.c_int, vp, C.c_int, C.c_double, C.c_int,
                                       vp, P(C.c_double), P(C.c_int), vp, sz, vp]),
        "rom_basis_dims": (C.c_int, [vp, P(C.c_int64), P(C.c_int)]),
        "rom_basis_copy": (C.c_int, [vp, vp, vp]),
        "rom_operator_destroy": (None, [vp]),
        "rom_basis_destroy": (None, [vp]),
        "rom_last_error": (C.c_char_p, []),
        "rom_seednet_bytes": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P(C.c_int64),
                                        P(sz), P(sz)]),
        "rom_seednet_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P(C.c_float),
                                         vp, sz, vp, sz, P(vp), vp]),
        "rom_seednet_backward": (C.c_int, [vp, vp, vp, C.c_int, P(C.c_float), vp]),
        "rom_seednet_adam": (C.c_int, [vp, C.c_float, vp]),
        "rom_subspace_loss_bytes": (C.c_int, [C.c_int64, C.c_int, C.c_int, P(sz)]),
        "rom_subspace_loss": (C.c_int, [vp, C.c_int, vp, C.c_int64, C.c_int64, C.c_int,
                                        P(C.c_double), vp, vp, sz, vp]),
        "rom_seednet_forward": (C.c_int, [vp, vp, vp, C.c_int, vp]),
        "rom_seednet_gradients": (C.c_int, [vp, vp, vp, C.c_int, P(C.c_float), P(C.c_double), vp]),
        "rom_seednet_train_step": (C.c_int, [vp, vp, vp, C.c_int, C.c_float, P(C.c_double), vp]),
        "rom_seednet_params": (C.c_int, [vp, P(C.c_float), vp]),
        "rom_seednet_destroy": (None, [vp]),
        "rom_seednet_inputs": (C.c_int, [vp, P(rom_mu), P(C.c_int64), C.c_int, vp, vp, sz, vp]),
        "rom_seednet_targets": (C.c_int, [vp, C.c_int64, C.c_int64, C.c_int, vp, vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _check(status: int, allow=()):
    if status != ROM_OK and status not in allow:
        raise RomError(status, rom_last_error())
    return status


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def rom_last_error() -> str:
    s = _lib.rom_last_error()
    return s.decode() if s else ""


def make_grid(dim: int, N: Sequence[int], bc: Sequence[int], robin_A: float) -> rom_grid:
    g = rom_grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = int(N[a]) if a < len(N) else 1
    for f in range(6):
        g.bc[f] = int(bc[f])
    g.robin_A = float(robin_A)
    return g


def make_opts(tol: float, trunc: float = 1e-8, cap: int = 0, maxit: int = 0,
              check_every: int = 0, timing: int = 0, precision: int = ROM_PREC_FP64,
              inner_tol: float = 0.0, group: int = 0, tune: int = 0, graph: int = 0,
              guess=None, recycle=None, cg_step: int = 0) -> rom_opts:
    """guess: device FP32 tensor (K * n_rhs, N) of initial guesses, or None; recycle: device
    FP32 tensor (K, n_recycle, N) of learned recycle vectors per point, or None (both kept
    alive by the caller during the solve)."""
    nrec = int(recycle.shape[1]) if recycle is not None else 0
    return rom_opts(float(tol), float(trunc), float(inner_tol), int(cap), int(maxit),
                    int(check_every), int(timing), int(precision), int(group), int(tune),
                    int(graph), _ptr(guess), _ptr(recycle), nrec, int(cg_step))


@dataclass
class MuParams:
    """Host-side absorption parameters of one point (kept alive during a call)."""
    mu0: float
    centers: np.ndarray
    radii: np.ndarray
    amps: np.ndarray

    def c_struct(self) -> rom_mu:
        self._c = np.ascontiguousarray(self.centers, dtype=np.float64).reshape(-1)
        self._r = np.ascontiguousarray(self.radii, dtype=np.float64)
        self._a = np.ascontiguousarray(self.amps, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        return rom_mu(int(self._r.size), self._c.ctypes.data_as(dp), self._r.ctypes.data_as(dp),
                      self._a.ctypes.data_as(dp), float(self.mu0))


def rom_operator_bytes(grid: rom_grid, variable_D: bool) -> int:
    out = C.c_size_t(0)
    _check(_lib.rom_operator_bytes(C.byref(grid), int(bool(variable_D)), C.byref(out)))
    return int(out.value)


def rom_assemble_operator(grid: rom_grid, D_const: float, D_field, op_mem, stream=None) -> int:
    h = C.c_void_p()
    _check(_lib.rom_assemble_operator(C.byref(grid), float(D_const), _ptr(D_field), _ptr(op_mem),
                                      op_mem.numel() * op_mem.element_size(), C.byref(h),
                                      _stream(stream)))
    return h.value


def rom_apply_operator(op: int, p: MuParams, X, Y, k: int, scratch, stream=None) -> None:
    mu = p.c_struct()
    _check(_lib.rom_apply_operator(op, C.byref(mu), _ptr(X), _ptr(Y), int(k), _ptr(scratch),
                                   scratch.numel() * scratch.element_size(), _stream(stream)))


def rom_apply_operator_static(op: int, p: MuParams, X, Y, k: int, stream=None) -> None:
    mu = p.c_struct()
    _check(_lib.rom_apply_operator_static(op, C.byref(mu), _ptr(X), _ptr(Y), int(k),
                                          _stream(stream)))


def rom_sequence_bytes(op: int, n_src: int, n_det: int, k_u: int, K: int, opts: rom_opts) -> int:
    out = C.c_size_t(0)
    _check(_lib.rom_sequence_bytes(op, n_src, n_det, k_u, K, C.byref(opts), C.byref(out)))
    return int(out.value)


def rom_solve_sequence(op: int, params: List[MuParams], src_idx, src_scale, det_idx, det_scale,
                       U0, k_u: int, opts: rom_opts, workspace, X_out=None, stream=None):
    """Returns (status, basis handle, records list, stats); raises on errors other
    than ROM_ENOCONV."""
    K = len(params)
    arr = (rom_mu * K)(*[p.c_struct() for p in params])
    si = np.ascontiguousarray(src_idx, dtype=np.int64)
    ss = np.ascontiguousarray(src_scale, dtype=np.float64)
    di = np.ascontiguousarray(det_idx, dtype=np.int64)
    ds = np.ascontiguousarray(det_scale, dtype=np.float64)
    n_rhs = si.size + di.size
    recs = (rom_record * (K * n_rhs))()
    st = rom_stats()
    basis = C.c_void_p()
    P = C.POINTER
    status = _lib.rom_solve_sequence(
        op, arr, K, si.ctypes.data_as(P(C.c_int64)), ss.ctypes.data_as(P(C.c_double)), si.size,
        di.ctypes.data_as(P(C.c_int64)), ds.ctypes.data_as(P(C.c_double)), di.size,
        _ptr(U0), int(k_u), C.byref(opts), _ptr(workspace),
        workspace.numel() * workspace.element_size(), C.byref(basis), _ptr(X_out), recs,
        C.byref(st), _stream(stream))
    records = [{f: getattr(r, f) for f, _ in rom_record._fields_} for r in recs]
    if status != ROM_OK and status != ROM_ENOCONV:
        err = RomError(status, rom_last_error())
        # the right-hand sides completed before the error (zeroed records after them)
        err.records = [r for r in records if r["converged"] or r["solved"] or r["rho0"] > 0]
        raise err
    return status, basis.value, records, st



class SequenceHandle:
    """Host-side state of a streaming sequence (keeps the arrays the library reads)."""

    def __init__(self, handle: int, n_rhs: int, keep):
        self.handle = handle
        self.n_rhs = n_rhs
        self._keep = keep


def rom_sequence_begin(op: int, K: int, src_idx, src_scale, det_idx, det_scale, U0, k_u: int,
                       opts: rom_opts, workspace, stream=None) -> SequenceHandle:
    si = np.ascontiguousarray(src_idx, dtype=np.int64)
    ss = np.ascontiguousarray(src_scale, dtype=np.float64)
    di = np.ascontiguousarray(det_idx, dtype=np.int64)
    ds = np.ascontiguousarray(det_scale, dtype=np.float64)
    h = C.c_void_p()
    P = C.POINTER
    _check(_lib.rom_sequence_begin(
        op, int(K), si.ctypes.data_as(P(C.c_int64)), ss.ctypes.data_as(P(C.c_double)), si.size,
        di.ctypes.data_as(P(C.c_int64)), ds.ctypes.data_as(P(C.c_double)), di.size, _ptr(U0),
        int(k_u), C.byref(opts), _ptr(workspace), workspace.numel() * workspace.element_size(),
        C.byref(h), _stream(stream)))
    return SequenceHandle(h.value, si.size + di.size, (U0, opts, workspace))


def rom_sequence_point(seq: SequenceHandle, p: MuParams, X_out=None):
    """Returns (status, records of the point); raises on errors other than ROM_ENOCONV."""
    mu = p.c_struct()
    recs = (rom_record * seq.n_rhs)()
    status = _check(_lib.rom_sequence_point(seq.handle, C.byref(mu), _ptr(X_out), recs),
                    allow=(ROM_ENOCONV,))
    return status, [{f: getattr(r, f) for f, _ in rom_record._fields_} for r in recs]


def rom_sequence_basis(seq: SequenceHandle) -> int:
    V = C.c_void_p()
    _check(_lib.rom_sequence_basis(seq.handle, C.byref(V)))
    return V.value


def rom_sequence_stats(seq: SequenceHandle) -> rom_stats:
    st = rom_stats()
    _check(_lib.rom_sequence_stats(seq.handle, C.byref(st)))
    return st


def rom_sequence_end(seq: SequenceHandle):
    """Returns (basis handle, stats)."""
    basis = C.c_void_p()
    st = rom_stats()
    h, seq.handle = seq.handle, None
    _check(_lib.rom_sequence_end(h, C.byref(basis), C.byref(st)))
    return basis.value, st


def rom_solve_sequences(jobs: List[dict]):
    """Run several sequences concurrently (one host thread and one stream each).  Each job
    is a dict of rom_solve_sequence arguments: op, params, src_idx, src_scale, det_idx,
    det_scale, U0, k_u, opts, workspace, X_out (or None), stream (or None).  Returns a
    list of (status, basis handle, records, stats); raises on errors other than
    ROM_ENOCONV (the error of the first failing job)."""
    n = len(jobs)
    arr = (rom_sequence_job * n)()
    keep = []
    out = []
    P = C.POINTER
    for q, jb in enumerate(jobs):
        params = jb["params"]
        K = len(params)
        mus = (rom_mu * K)(*[p.c_struct() for p in params])
        si = np.ascontiguousarray(jb["src_idx"], dtype=np.int64)
        ss = np.ascontiguousarray(jb["src_scale"], dtype=np.float64)
        di = np.ascontiguousarray(jb["det_idx"], dtype=np.int64)
        ds = np.ascontiguousarray(jb["det_scale"], dtype=np.float64)
        recs = (rom_record * (K * (si.size + di.size)))()
        st = rom_stats()
        basis = C.c_void_p()
        opts = jb["opts"]
        ws = jb["workspace"]
        keep.append((mus, si, ss, di, ds, recs, st, basis, opts, params))
        j = arr[q]
        j.op = jb["op"]
        j.params = C.cast(mus, P(rom_mu))
        j.K = K
        j.src_idx = si.ctypes.data_as(P(C.c_int64))
        j.src_scale = ss.ctypes.data_as(P(C.c_double))
        j.n_src = si.size
        j.det_idx = di.ctypes.data_as(P(C.c_int64))
        j.det_scale = ds.ctypes.data_as(P(C.c_double))
        j.n_det = di.size
        j.U0 = _ptr(jb.get("U0"))
        j.k_u = int(jb.get("k_u", 0))
        j.opts = C.pointer(opts)
        j.workspace = _ptr(ws)
        j.ws_bytes = ws.numel() * ws.element_size()
        j.basis = C.pointer(basis)
        j.X_out = _ptr(jb.get("X_out"))
        j.records = C.cast(recs, P(rom_record))
        j.stats = C.pointer(st)
        j.stream = _stream(jb.get("stream"))
    status = _lib.rom_solve_sequences(arr, n)
    for q in range(n):
        mus, si, ss, di, ds, recs, st, basis, opts, params = keep[q]
        records = [{f: getattr(r, f) for f, _ in rom_record._fields_} for r in recs]
        out.append((arr[q].status, basis.value, records, st))
    if status != ROM_OK and status != ROM_ENOCONV:
        raise RomError(status, rom_last_error())
    return out

def rom_reduced_bytes(basis: int) -> int:
    out = C.c_size_t(0)
    _check(_lib.rom_reduced_bytes(basis, C.byref(out)))
    return int(out.value)


def rom_reduced_transfer(basis: int, p: MuParams, Ar, Br, Cr, Er, scratch, stream=None) -> None:
    mu = p.c_struct()
    _check(_lib.rom_reduced_transfer(basis, C.byref(mu), _ptr(Ar), _ptr(Br), _ptr(Cr), _ptr(Er),
                                     _ptr(scratch), scratch.numel() * scratch.element_size(),
                                     _stream(stream)))


def rom_reduced_jacobian_bytes(basis: int) -> int:
    out = C.c_size_t(0)
    _check(_lib.rom_reduced_jacobian_bytes(basis, C.byref(out)))
    return int(out.value)


def rom_reduced_jacobian(basis: int, p: MuParams, J, scratch, stream=None) -> None:
    mu = p.c_struct()
    _check(_lib.rom_reduced_jacobian(basis, C.byref(mu), _ptr(J), _ptr(scratch),
                                     scratch.numel() * scratch.element_size(), _stream(stream)))


def rom_lowest_modes_bytes(op: int, kx: int) -> int:
    out = C.c_size_t(0)
    _check(_lib.rom_lowest_modes_bytes(op, int(kx), C.byref(out)))
    return int(out.value)


def rom_lowest_modes(op: int, p: MuParams, k: int, X0, kx: int, tol: float, maxit: int, U,
                     scratch, stream=None, allow_noconv: bool = False):
    """Returns (lambda (k,), sweeps), or (lambda, sweeps, status) with allow_noconv; U is
    filled on the device."""
    mu = p.c_struct()
    lam = (C.c_double * k)()
    sweeps = C.c_int(0)
    st = _check(_lib.rom_lowest_modes(op, C.byref(mu), int(k), _ptr(X0), int(kx), float(tol),
                                      int(maxit), _ptr(U), lam, C.byref(sweeps), _ptr(scratch),
                                      scratch.numel() * scratch.element_size(), _stream(stream)),
                allow=(ROM_ENOCONV,) if allow_noconv else ())
    out = (np.array(lam[:], dtype=np.float64), int(sweeps.value))
    return out + (st,) if allow_noconv else out


def rom_shifted_solve_bytes(op: int, nb: int, ns: int) -> int:
    out = C.c_size_t(0)
    _check(_lib.rom_shifted_solve_bytes(op, int(nb), int(ns), C.byref(out)))
    return int(out.value)


def rom_shifted_solve(op: int, p: MuParams, B, nb: int, sigma, tol: float, maxit: int, Xr, Xi,
                      scratch, stream=None, allow_noconv: bool = False):
    """Returns (status, its (nb,), resid (ns, nb)); Xr, Xi are filled on the device."""
    mu = p.c_struct()
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    ns = sig.size
    sarr = (C.c_double * ns)(*sig.tolist())
    its = (C.c_int * nb)()
    res = (C.c_double * (nb * ns))()
    st = _check(_lib.rom_shifted_solve(op, C.byref(mu), _ptr(B), int(nb), sarr, int(ns),
                                       float(tol), int(maxit), _ptr(Xr), _ptr(Xi), its, res,
                                       _ptr(scratch), scratch.numel() * scratch.element_size(),
                                       _stream(stream)),
                allow=(ROM_ENOCONV,) if allow_noconv else ())
    return st, np.array(its[:], dtype=np.int64), np.array(res[:]).reshape(ns, nb)


def rom_reduced_response_bytes(basis: int) -> int:
    out = C.c_size_t(0)
    _check(_lib.rom_reduced_response_bytes(basis, C.byref(out)))
    return int(out.value)


def rom_reduced_response(basis: int, p: MuParams, sigma, Psi_re, Psi_im, scratch,
                         stream=None) -> None:
    mu = p.c_struct()
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    sarr = (C.c_double * max(sig.size, 1))(*sig.tolist())
    _check(_lib.rom_reduced_response(basis, C.byref(mu), sarr, int(sig.size), _ptr(Psi_re),
                                     _ptr(Psi_im), _ptr(scratch),
                                     scratch.numel() * scratch.element_size(), _stream(stream)))


def rom_basis_dims(basis: int):
    n = C.c_int64(0)
    m = C.c_int(0)
    _check(_lib.rom_basis_dims(basis, C.byref(n), C.byref(m)))
    return int(n.value), int(m.value)


def rom_basis_copy(basis: int, dst, stream=None) -> None:
    _check(_lib.rom_basis_copy(basis, _ptr(dst), _stream(stream)))


def rom_operator_destroy(op: int) -> None:
    _lib.rom_operator_destroy(op)


def rom_basis_destroy(basis: int) -> None:
    _lib.rom_basis_destroy(basis)


def stats_dict(st: rom_stats) -> dict:
    d = {f: getattr(st, f) for f in ("m", "k_u", "n_solved", "n_kept", "n_dropped_trunc",
                                     "n_dropped_cap", "n_nonconv", "total_its", "seconds",
                                     "n_uj_capped")}
    d["kernels"] = {KERNEL_CLASSES[k]: {"ms": st.kernel_ms[k], "bytes": st.kernel_bytes[k],
                                        "flops": st.kernel_flops[k],
                                        "launches": int(st.kernel_launches[k])}
                    for k in range(ROM_NK)}
    return d


# ---- learned seed network ---------------------------------------------------------------

def rom_seednet_bytes(nx: int, ny: int, nz: int, batch: int, outputs: int = 1):
    npar, pb, wb = C.c_int64(), C.c_size_t(), C.c_size_t()
    _check(_lib.rom_seednet_bytes(nx, ny, nz, batch, outputs, C.byref(npar), C.byref(pb),
                                  C.byref(wb)))
    return npar.value, pb.value, wb.value


def rom_seednet_create(nx: int, ny: int, nz: int, batch: int, params: np.ndarray, param_mem,
                       work_mem, stream=None, outputs: int = 1) -> int:
    params = np.ascontiguousarray(params, dtype=np.float32)
    net = C.c_void_p()
    _check(_lib.rom_seednet_create(nx, ny, nz, batch, outputs,
                                   params.ctypes.data_as(C.POINTER(C.c_float)),
                                   _ptr(param_mem), param_mem.numel() * param_mem.element_size(),
                                   _ptr(work_mem), work_mem.numel() * work_mem.element_size(),
                                   C.byref(net), _stream(stream)))
    return net.value


def rom_seednet_forward(net: int, inputs, outputs, batch: int, stream=None):
    _check(_lib.rom_seednet_forward(net, _ptr(inputs), _ptr(outputs), batch, _stream(stream)))


def rom_seednet_gradients(net: int, inputs, targets, batch: int, nparams: int, stream=None):
    g = np.empty(nparams, dtype=np.float32)
    loss = C.c_double()
    _check(_lib.rom_seednet_gradients(net, _ptr(inputs), _ptr(targets), batch,
                                      g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                      _stream(stream)))
    return loss.value, g


def rom_seednet_train_step(net: int, inputs, targets, batch: int, lr: float, stream=None) -> float:
    loss = C.c_double()
    _check(_lib.rom_seednet_train_step(net, _ptr(inputs), _ptr(targets), batch, float(lr),
                                       C.byref(loss), _stream(stream)))
    return loss.value


def rom_seednet_backward(net: int, inputs, dy, batch: int, nparams: int = 0, stream=None):
    """Parameter gradient of a loss whose output gradient is dy (returned if nparams > 0)."""
    g = np.empty(nparams, dtype=np.float32) if nparams > 0 else None
    _check(_lib.rom_seednet_backward(net, _ptr(inputs), _ptr(dy), batch,
                                     g.ctypes.data_as(C.POINTER(C.c_float)) if g is not None
                                     else None, _stream(stream)))
    return g


def rom_seednet_adam(net: int, lr: float, stream=None) -> None:
    _check(_lib.rom_seednet_adam(net, float(lr), _stream(stream)))


def rom_subspace_loss_bytes(N: int, k: int, s: int) -> int:
    out = C.c_size_t(0)
    _check(_lib.rom_subspace_loss_bytes(int(N), int(k), int(s), C.byref(out)))
    return int(out.value)


def rom_subspace_loss(Y, k: int, X, N: int, ldx: int, s: int, dY, scratch, stream=None) -> float:
    loss = C.c_double(0.0)
    _check(_lib.rom_subspace_loss(_ptr(Y), int(k), _ptr(X), int(N), int(ldx), int(s),
                                  C.byref(loss), _ptr(dY) if dY is not None else None,
                                  _ptr(scratch), scratch.numel() * scratch.element_size(),
                                  _stream(stream)))
    return loss.value


def rom_seednet_params(net: int, nparams: int, stream=None) -> np.ndarray:
    p = np.empty(nparams, dtype=np.float32)
    _check(_lib.rom_seednet_params(net, p.ctypes.data_as(C.POINTER(C.c_float)), _stream(stream)))
    return p


def rom_seednet_destroy(net: int):
    if net:
        _lib.rom_seednet_destroy(net)


def rom_seednet_inputs(op: int, p: MuParams, idx, out, scratch, stream=None):
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    mu = p.c_struct()
    _check(_lib.rom_seednet_inputs(op, C.byref(mu), idx.ctypes.data_as(C.POINTER(C.c_int64)),
                                   idx.size, _ptr(out), _ptr(scratch),
                                   scratch.numel() * scratch.element_size(), _stream(stream)))


def rom_seednet_targets(X, n: int, ldx: int, count: int, out, scratch, stream=None):
    _check(_lib.rom_seednet_targets(_ptr(X), n, ldx, count, _ptr(out), _ptr(scratch),
                                    scratch.numel() * scratch.element_size(), _stream(stream)))
