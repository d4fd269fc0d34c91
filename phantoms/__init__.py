"""Seeded synthetic DOT workloads (phantoms) shared by the CPU oracle and the GPU path.

This module only *describes* inputs: grid shapes, boundary kinds, diffusion fields,
absorption-bump parameters per parameter point, source/detector node indices and
a set of analytic smooth modes used as the offline recycle seed U_0.  It contains
none of the method's arithmetic (no operator assembly, no solves, no projections).

Paper context (arXiv:1602.00138):
  * Sec. 2.1, eq. (ModelPDE1-4): slab domain, Robin condition on the top/bottom
    faces, zero Dirichlet on the lateral faces, point sources and detectors on
    the Robin faces (sources and detectors not co-located, Sec. 3.1).
  * Sec. 3.1: after eliminating the Robin boundary unknowns the effective
    sources/receivers are scaled columns of the identity located at the first
    interior layer next to the face.
  * Sec. 4.2.2: U_0 holds (estimates of) the eigenvectors of the first system
    matrix for its 10 smallest eigenvalues, computed offline (Sec. 4.4).
  * Sec. 5: 32 sources + 32 detectors, absorption given by compactly supported
    radial basis functions.

The five workloads below are synthetic stand-ins for the paper's experiments (its
ground-truth images, noisy data and optimiser iterates are not available).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Face order used everywhere: -x, +x, -y, +y, -z, +z.  0 = Dirichlet, 1 = Robin.
DIRICHLET = 0
ROBIN = 1


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    N: Tuple[int, int, int]          # interior nodes per axis (N[2] == 1 in 2D)
    D: object                        # float, or "lognormal"
    mu0: float
    nb: int                          # absorption bumps per parameter point
    radius: Tuple[float, float]
    amp: Tuple[float, float]
    n_src: int
    n_det: int
    K: int                           # parameter points (including p_0)
    tol: float
    trunc: float = 1e-8
    cap: int = 0                     # 0 = no cap
    robin_A: float = 1.0
    seed: int = 1000
    d_seed: int = 2000
    k_u: int = 10

    @property
    def n(self) -> int:
        return int(self.N[0] * self.N[1] * self.N[2])

    @property
    def n_rhs(self) -> int:
        return self.n_src + self.n_det

    @property
    def bc(self) -> Tuple[int, ...]:
        return face_kinds(self.dim)

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def face_kinds(dim: int) -> Tuple[int, ...]:
    """Robin on the source/detector faces (2D: y=0,1; 3D: z=0,1), Dirichlet laterally."""
    if dim == 2:
        return (DIRICHLET, DIRICHLET, ROBIN, ROBIN, DIRICHLET, DIRICHLET)
    return (DIRICHLET, DIRICHLET, DIRICHLET, DIRICHLET, ROBIN, ROBIN)


WORKLOADS = {
    # 2D 32^2, plain FP64, checked against dense Cholesky.
    "slab2d_32": Workload("slab2d_32", 2, (32, 32, 1), 0.03, 0.01, 3, (0.05, 0.15),
                          (0.005, 0.02), 8, 8, 4, 1e-10, seed=1001, d_seed=2001),
    # 3D 64^3, plain FP64, 32+32 RHS, 16 points (timing tolerance 1e-8).
    "cube64": Workload("cube64", 3, (64, 64, 64), 0.03, 0.01, 8, (0.04, 0.12), (0.005, 0.03),
                       32, 32, 16, 1e-8, seed=1002, d_seed=2002),
    # Three uneven 3D grids (48^3, 64^3, 96^3), 8 points each, 32+32 RHS.
    "uneven48": Workload("uneven48", 3, (48, 48, 48), 0.03, 0.01, 3, (0.05, 0.15),
                         (0.005, 0.02), 32, 32, 8, 1e-8, seed=1003, d_seed=2003),
    "uneven64": Workload("uneven64", 3, (64, 64, 64), 0.03, 0.01, 3, (0.05, 0.15),
                         (0.005, 0.02), 32, 32, 8, 1e-8, seed=1103, d_seed=2103),
    "uneven96": Workload("uneven96", 3, (96, 96, 96), 0.03, 0.01, 3, (0.05, 0.15),
                         (0.005, 0.02), 32, 32, 8, 1e-8, seed=1203, d_seed=2203),
    # 3D 128^3 with log-normal D, capped basis.
    "cube128_lognormal": Workload("cube128_lognormal", 3, (128, 128, 128), "lognormal", 0.01,
                                  16, (0.04, 0.12), (0.005, 0.03), 48, 48, 32, 1e-8, cap=256,
                                  seed=1004, d_seed=2004),
    # 3D 96^3 with log-normal D, 64+64 RHS.
    "cube96_lognormal": Workload("cube96_lognormal", 3, (96, 96, 96), "lognormal", 0.01, 12,
                                 (0.04, 0.12), (0.005, 0.03), 64, 64, 16, 1e-8, seed=1005,
                                 d_seed=2005),
}


def small(dim: int = 3, N: Sequence[int] = (12, 12, 12), n_src: int = 4, n_det: int = 4,
          K: int = 3, nb: int = 3, D="const", tol: float = 1e-10, seed: int = 7,
          k_u: int = 10, cap: int = 0) -> Workload:
    """A small workload of the same structure, for tests."""
    N3 = tuple(N) + (1,) * (3 - len(N))
    if dim == 2:
        N3 = (N3[0], N3[1], 1)
    return Workload(f"small{dim}d", dim, N3, 0.03 if D == "const" else "lognormal", 0.01, nb,
                    (0.08, 0.2), (0.005, 0.03), n_src, n_det, K, tol, cap=cap, seed=seed,
                    d_seed=seed + 1000, k_u=k_u)


# --------------------------------------------------------------------------------------
# geometry


def spacing(wl: Workload) -> Tuple[float, float, float]:
    """Node spacing per axis on the unit square/cube: h = 1/(N+1) (nodes at (i+1)h)."""
    return tuple(1.0 / (wl.N[a] + 1) if a < wl.dim else 1.0 for a in range(3))


def node_coords(wl: Workload) -> np.ndarray:
    """(n, dim) coordinates of the unknowns in x-fastest lexicographic order."""
    axes = [(np.arange(wl.N[a]) + 1.0) / (wl.N[a] + 1) for a in range(wl.dim)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")      # slowest axis first
    cols = [m.reshape(-1) for m in mesh[::-1]]           # back to x, y, (z)
    return np.stack(cols, axis=1)


def diffusion_field(wl: Workload):
    """Scalar D, or the per-node log-normal field D = 0.03 exp(0.3 z), z ~ N(0,1)."""
    if wl.D == "lognormal":
        z = np.random.default_rng(wl.d_seed).standard_normal(wl.n)
        return 0.03 * np.exp(0.3 * z)
    return float(wl.D)


# --------------------------------------------------------------------------------------
# parameter points: compact RBF bumps


@dataclasses.dataclass
class Bumps:
    mu0: float
    centers: np.ndarray   # (nb, dim)
    radii: np.ndarray     # (nb,)
    amps: np.ndarray      # (nb,)


def parameter_points(wl: Workload, K: Optional[int] = None, mode: str = "independent") -> List[Bumps]:
    """Draw the absorption bumps of every parameter point.

    independent: each point draws centers U(0.2,0.8)^d, radii, amplitudes in that
    order from one PCG64 stream seeded with ``wl.seed``.
    drift: p_0 as above, then each point moves the previous one by up to 10% of
    each parameter's range (mimicking successive optimiser iterates).
    """
    K = wl.K if K is None else K
    rng = np.random.default_rng(wl.seed)
    d = wl.dim
    pts: List[Bumps] = []
    for k in range(K):
        if mode == "independent" or k == 0:
            c = rng.uniform(0.2, 0.8, (wl.nb, d))
            r = rng.uniform(wl.radius[0], wl.radius[1], wl.nb)
            a = rng.uniform(wl.amp[0], wl.amp[1], wl.nb)
        elif mode == "drift":
            prev = pts[-1]
            c = np.clip(prev.centers + 0.06 * rng.uniform(-1, 1, (wl.nb, d)), 0.2, 0.8)
            r = np.clip(prev.radii + 0.1 * (wl.radius[1] - wl.radius[0]) * rng.uniform(-1, 1, wl.nb),
                        wl.radius[0], wl.radius[1])
            a = np.clip(prev.amps + 0.1 * (wl.amp[1] - wl.amp[0]) * rng.uniform(-1, 1, wl.nb),
                        wl.amp[0], wl.amp[1])
        else:
            raise ValueError(mode)
        pts.append(Bumps(wl.mu0, c, r, a))
    return pts


# --------------------------------------------------------------------------------------
# sources and detectors (effective unit columns at the first interior layer)


def rhs_nodes(wl: Workload) -> Tuple[np.ndarray, np.ndarray]:
    """Node indices of the effective sources and detectors.

    2D: sources evenly spaced on the top interior row (y = 1 side), detectors on the
    bottom row (y = 0 side).  3D: an 8 x (n/8) lattice on the z = 0 layer (sources)
    and on the z = 1 layer (detectors), first lattice index fastest.
    """
    N = wl.N

    def spread(count, length):
        return ((np.arange(count) + 0.5) * length / count).astype(np.int64)

    if wl.dim == 2:
        if min(wl.n_src, wl.n_det) == 0:
            raise ValueError("2D workloads need sources and detectors")
        src = spread(wl.n_src, N[0]) + N[0] * (N[1] - 1)
        det = spread(wl.n_det, N[0])
        return src.astype(np.int64), det.astype(np.int64)

    def lattice(count, layer):
        if count == 0:
            return np.zeros(0, dtype=np.int64)
        na = 8 if count >= 8 and count % 8 == 0 else count
        nbb = count // na
        ia = spread(na, N[0])
        ib = spread(nbb, N[1])
        idx = [ia[a] + N[0] * (ib[b] + N[1] * layer) for b in range(nbb) for a in range(na)]
        return np.asarray(idx, dtype=np.int64)

    return lattice(wl.n_src, 0), lattice(wl.n_det, N[2] - 1)


def rhs_scales(wl: Workload) -> Tuple[np.ndarray, np.ndarray]:
    """Unit scales (relative residuals and the recycled basis do not depend on them)."""
    return np.ones(wl.n_src), np.ones(wl.n_det)


# --------------------------------------------------------------------------------------
# offline recycle seed U_0: analytic smooth modes


def smooth_modes(wl: Workload, k_u: Optional[int] = None) -> np.ndarray:
    """k_u analytic smooth modes of the background slab problem, columns unit 2-norm.

    Along a Dirichlet-Dirichlet axis the modes are sin(k pi x); along an axis with a
    Robin face the interval is extended by the extrapolation length 2*A*D at that
    face and the mode is the sine of the extended interval.  The k_u products with
    the smallest continuous eigenvalue sum(k_a pi / L_a)^2 are returned (ties in
    x-fastest index order).  They are estimates of the low eigenvectors used to
    seed the recycle spaces; the method orthonormalises them itself.
    """
    k_u = wl.k_u if k_u is None else k_u
    if k_u == 0:
        return np.zeros((wl.n, 0))
    Dref = 0.03 if wl.D == "lognormal" else float(wl.D)
    bc = wl.bc
    kmax = 6
    axes = []
    for a in range(wl.dim):
        lo = 2 * wl.robin_A * Dref if bc[2 * a] == ROBIN else 0.0
        hi = 2 * wl.robin_A * Dref if bc[2 * a + 1] == ROBIN else 0.0
        L = 1.0 + lo + hi
        x = (np.arange(wl.N[a]) + 1.0) / (wl.N[a] + 1)
        modes = [np.sin(k * np.pi * (x + lo) / L) for k in range(1, kmax + 1)]
        lams = [(k * np.pi / L) ** 2 for k in range(1, kmax + 1)]
        axes.append((modes, lams))
    combos = []
    import itertools
    for ks in itertools.product(range(kmax), repeat=wl.dim):
        lam = sum(axes[a][1][ks[a]] for a in range(wl.dim))
        combos.append((lam, ks[::-1], ks))
    combos.sort(key=lambda t: (round(t[0], 12), t[1]))
    cols = []
    for lam, _, ks in combos[:k_u]:
        v = axes[0][0][ks[0]]
        for a in range(1, wl.dim):
            v = np.multiply.outer(axes[a][0][ks[a]], v)   # slower axis outside
        v = v.reshape(-1)
        cols.append(v / np.sqrt(np.dot(v, v)))
    return np.ascontiguousarray(np.stack(cols, axis=1))


def describe(wl: Workload) -> dict:
    return {"workload": wl.name, "grid": "x".join(str(x) for x in wl.N[:wl.dim]), "n": wl.n,
            "n_src": wl.n_src, "n_det": wl.n_det, "points": wl.K, "tol": wl.tol,
            "trunc": wl.trunc, "cap": wl.cap, "D": wl.D if isinstance(wl.D, str) else float(wl.D),
            "bumps": wl.nb}
