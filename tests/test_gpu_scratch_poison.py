"""Entry points that take caller-owned scratch must not read scratch they did not write:
each is called once with scratch holding zeros and once with every byte 0xFF (NaN as a
double, -1 as an integer), and the results must agree bit for bit.  A kernel that reads a
never-written part of its scratch (for instance the zeros above the diagonal of a
triangular factor) turns the second call's result into NaN or garbage."""
import numpy as np
import pytest

import phantoms as ph

pytestmark = pytest.mark.gpu


def _scratch(nbytes, fill):
    import torch
    t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    t.fill_(fill)
    return t


@pytest.fixture(scope="module")
def seq(gpu):
    from paper_1602_00138_amd import driver
    wl = ph.small(3, (16, 15, 14), n_src=5, n_det=6, K=3, nb=3, D="lognormal")
    prob = driver.problem_from_workload(wl)
    pts = driver.points_from_workload(wl)
    res = prob.solve(pts, wl.tol, wl.trunc, keep_X=False)
    yield wl, prob, pts, res
    res.close()


def test_reduced_jacobian_and_response_ignore_scratch_contents(seq):
    import torch
    from paper_1602_00138_amd import rom as R
    wl, prob, pts, res = seq
    p = pts[-1]
    ns, nd = wl.n_src, wl.n_det
    npar = int(np.asarray(p.radii).size) * (wl.dim + 2)
    out = []
    for fill in (0, 255):
        J = torch.empty((npar, ns, nd), dtype=torch.float64, device="cuda")
        R.rom_reduced_jacobian(res.basis, p, J, _scratch(R.rom_reduced_jacobian_bytes(res.basis), fill))
        sig = np.array([0.0, 0.5, 4.0])
        Pr = torch.empty((3, ns, nd), dtype=torch.float64, device="cuda")
        Pi = torch.empty_like(Pr)
        R.rom_reduced_response(res.basis, p, sig, Pr, Pi,
                               _scratch(R.rom_reduced_response_bytes(res.basis), fill))
        m = res.m
        Ar = torch.empty((m, m), dtype=torch.float64, device="cuda")
        Er = torch.empty_like(Ar)
        Br = torch.empty((ns, m), dtype=torch.float64, device="cuda")
        Cr = torch.empty((nd, m), dtype=torch.float64, device="cuda")
        R.rom_reduced_transfer(res.basis, p, Ar, Br, Cr, Er,
                               _scratch(R.rom_reduced_bytes(res.basis), fill))
        out.append([t.cpu().numpy() for t in (J, Pr, Pi, Ar, Br, Cr, Er)])
    for a, b in zip(*out):
        assert np.isfinite(a).all() and np.array_equal(a, b)


def test_solvers_ignore_scratch_contents(seq):
    import torch
    from paper_1602_00138_amd import rom as R
    wl, prob, pts, res = seq
    p = pts[0]
    out = []
    X0 = torch.from_numpy(np.ascontiguousarray(ph.smooth_modes(wl, 12).T)).cuda()
    B = torch.from_numpy(np.random.default_rng(3).standard_normal((2, wl.n))).cuda()
    for fill in (0, 255):
        U = torch.empty((8, wl.n), dtype=torch.float64, device="cuda")
        lam, sw = R.rom_lowest_modes(prob.op, p, 8, X0, 12, 1e-9, 300, U,
                                     _scratch(R.rom_lowest_modes_bytes(prob.op, 12), fill))
        Xr = torch.empty((3, 2, wl.n), dtype=torch.float64, device="cuda")
        Xi = torch.empty_like(Xr)
        st, its, resid = R.rom_shifted_solve(prob.op, p, B, 2, [0.0, 1.0, 9.0], 1e-10, wl.n, Xr, Xi,
                                             _scratch(R.rom_shifted_solve_bytes(prob.op, 2, 3), fill))
        Y = torch.from_numpy(np.random.default_rng(4).standard_normal((6, wl.n)).astype(np.float32)).cuda()
        dY = torch.empty_like(Y)
        loss = R.rom_subspace_loss(Y, 6, B, wl.n, wl.n, 2, dY,
                                   _scratch(R.rom_subspace_loss_bytes(wl.n, 6, 2), fill))
        out.append([U.cpu().numpy(), lam, np.array([sw]), Xr.cpu().numpy(), Xi.cpu().numpy(),
                    its, resid, np.array([loss]), dY.cpu().numpy()])
    for a, b in zip(*out):
        assert np.isfinite(a).all() and np.array_equal(a, b)
