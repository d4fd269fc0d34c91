"""GPU parity of the reduced Jacobian (rom_reduced_jacobian, eq. (newjac) projected on V)
against the oracle's reduced formula evaluated on the GPU's own basis, at the sample
points and off them, for every bump parameter; and, at the sample points, against the
full-order Jacobian (the interpolation theorem).

Tolerances: the GPU computes -Z^T diag(d mu/d p) U with lifted U = V A_r^{-1} B_r,
Z = V A_r^{-1} C_r, the oracle C_r^T A_r^{-1} (V^T diag(d mu/d p) V) A_r^{-1} B_r: the
same FP64 quantity in a different order; A_r is well conditioned here (kappa < 1e4), so
1e-9 relative to the largest entry of each column.  Against the full Jacobian at the
sample points: 1e-6 (the solutions lie in range(V) to the solver tolerance 1e-10)."""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem
from oracle import operator as op
from oracle import rom as orom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def drv(gpu):
    from paper_1602_00138_amd import driver
    return driver


@pytest.mark.parametrize("wl", [ph.small(2, (17, 13), n_src=4, n_det=3, K=2, nb=2),
                                ph.small(3, (11, 10, 9), n_src=3, n_det=4, K=2, nb=3,
                                         D="lognormal")])
def test_reduced_jacobian_parity(drv, wl):
    from paper_1602_00138_amd import rom as R
    orc = OracleProblem(wl)
    prob = drv.problem_from_workload(wl)
    pts = drv.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc)
    V = res.Q().cpu().numpy().T
    ns = wl.n_src
    Bt, Ct = orc.B[:, :ns], orc.B[:, ns:]
    # the sample points, then a point off them (moved centres, other radii)
    rng = np.random.default_rng(5)
    off = orc.pts[0]
    extra = R.MuParams(off.mu0, np.clip(off.centers + 0.05 * rng.uniform(-1, 1, off.centers.shape),
                                        0.2, 0.8),
                       off.radii * 1.1, off.amps * 0.9)
    cases = [(p, orc.pts[i], i) for i, p in enumerate(pts)] + [(extra, extra, None)]
    for p, op_p, i in cases:
        J = prob.reduced_jacobian(res, p).cpu().numpy()
        mu = op.mu_field(wl.dim, wl.N, op_p.mu0, op_p.centers, op_p.radii, op_p.amps)
        A = op.assemble_A(orc.As, mu)
        Ar, Br, Cr, _ = orom.reduced_matrices(V, A, Bt, Ct)
        G = op.mu_gradient(wl.dim, wl.N, op_p.centers, op_p.radii, op_p.amps)
        assert J.shape == (G.shape[0], wl.n_det, ns)
        for k in range(G.shape[0]):
            ref = orom.reduced_jacobian_column(V, Ar, Br, Cr, G[k])
            scale = np.abs(ref).max()
            assert np.abs(J[k] - ref).max() <= 1e-9 * scale, (i, k)
            if i is not None:
                full = orom.full_jacobian_column(A, Bt, Ct, G[k])
                assert np.abs(J[k] - full).max() <= 1e-6 * np.abs(full).max(), (i, k)
    res.close()
    prob.close()
