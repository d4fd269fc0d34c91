"""Full-size parity on the 64^3 workload (262,144 unknowns, 32 sources + 32 detectors,
16 independent points, tol 1e-8) in the launch configuration the benchmark times, for
the plain FP64 form and the mixed form.  The oracle cannot run the whole sequence at
this size, so it checks sampled outputs one by one:
  * every record reports convergence; sampled solutions have FP64 true relative
    residual <= tol under the oracle's CSR operator;
  * sampled solutions equal oracle reference solves (plain CG to 1e-13) within
    ||x - x_ref|| <= (tol ||b|| + ||r_ref||) / lambda_lb, where
    lambda_lb = sum over Dirichlet axes of 4 (D/h^2) sin^2(pi h / 2) + mu0 bounds
    lambda_min(A(p)) from below (A_* is a Kronecker sum of 1-D operators, the Robin
    axis one is positive semidefinite, and diag(mu) >= mu0 I);
  * the basis is orthonormal and contains every sampled reference solution to that
    bound plus 3 trunc (a dropped correction leaves at most trunc ||g|| outside);
  * reduced transfer-function columns at the sample points equal C~^T x_ref to 1e-6
    relative (interpolation, Sec. 3.4);
  * sampled entries of A_r(p) = V^T A(p) V equal the oracle's to 1e-12 relative.
"""
import numpy as np
import pytest

import phantoms as ph
from oracle import operator as op
from oracle import rom as orom

pytestmark = pytest.mark.gpu

WL = ph.WORKLOADS["cfg2"]
SAMPLES = [(0, 0), (5, 17), (11, 40), (15, 63)]    # (point, right-hand side)


def lambda_lower_bound(wl, mu0):
    lb = mu0
    for a in range(wl.dim):
        if wl.bc[2 * a] == 0 and wl.bc[2 * a + 1] == 0:
            h = 1.0 / (wl.N[a] + 1)
            lb += 4.0 * (wl.D / h ** 2) * np.sin(np.pi * h / 2) ** 2
    return lb


@pytest.fixture(scope="module")
def reference():
    D = ph.diffusion_field(WL)
    As = op.assemble_Astar(WL.dim, WL.N, WL.bc, D, WL.robin_A)
    pts = ph.parameter_points(WL)
    si, di = ph.rhs_nodes(WL)
    idx = np.concatenate([si, di])
    ref = {}
    for i, j in SAMPLES:
        p = pts[i]
        A = op.assemble_A(As, op.mu_field(WL.dim, WL.N, p.mu0, p.centers, p.radii, p.amps))
        b = np.zeros(WL.n)
        b[idx[j]] = 1.0
        x = orom.full_solve(A, b, 1e-13)
        ref[(i, j)] = (A, b, x, np.linalg.norm(b - A @ x))
    return ref, idx, si, di, pts


@pytest.mark.parametrize("precision,group", [("fp64", 1), ("mixed", 1), ("fp64", 8), ("mixed", 8)])
def test_fullsize_sampled_parity(gpu, reference, precision, group):
    """Groups of 8 at this size append many corrections that are nearly aligned with
    the columns appended just before them (small rho, large projections on V); the
    sampled A_r entries check that the bordered Gram matrix V^T A_* V stays exact."""
    import torch
    from paper_1602_00138_amd import driver
    from paper_1602_00138_amd import rom as R
    ref, idx, si, di, pts_host = reference
    assert isinstance(WL.D, float) and WL.bc[:4] == (0, 0, 0, 0)
    prob = driver.problem_from_workload(WL)
    pts = driver.points_from_workload(WL)
    prec = R.ROM_PREC_MIXED if precision == "mixed" else R.ROM_PREC_FP64
    print(f"\n{WL.name} {precision} group {group}: solving {len(pts)} points x {prob.n_rhs} RHS",
          flush=True)
    res = prob.solve(pts, WL.tol, WL.trunc, precision=prec, group=group)
    n_rhs = prob.n_rhs
    assert all(r["converged"] and r["final_res"] <= WL.tol * (1 + 1e-6) for r in res.records)
    Qd = res.Q()                                   # m x N on the device (rows = columns of V)
    m = res.m
    orth = (Qd @ Qd.T - torch.eye(m, dtype=torch.float64, device=Qd.device)).abs().max().item()
    assert orth <= 1e-12, orth
    worst = {"sol": 0.0, "res": 0.0, "basis": 0.0, "psi": 0.0, "Ar": 0.0}
    ns = WL.n_src
    for (i, j), (A, b, x_ref, r_ref) in ref.items():
        x = res.X[i * n_rhs + j].cpu().numpy()
        rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert rel <= WL.tol * (1 + 1e-6), (i, j, rel)
        lam = lambda_lower_bound(WL, pts_host[i].mu0)
        bound = (WL.tol * np.linalg.norm(b) + r_ref) / lam / np.linalg.norm(x_ref)
        err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
        assert err <= bound, (i, j, err, bound)
        xr = torch.as_tensor(x_ref, device=Qd.device)
        dist = (torch.linalg.norm(xr - Qd.T @ (Qd @ xr)) / torch.linalg.norm(xr)).item()
        assert dist <= bound + 3 * WL.trunc, (i, j, dist)
        Ar, Br, Cr, _ = [t.cpu().numpy() for t in prob.reduced(res, pts[i])]
        if j < ns:
            psir = orom.reduced_transfer(Ar, Br, Cr)[:, j]
            psi = x_ref[di]
            e = np.abs(psir - psi).max() / np.abs(psi).max()
            assert e <= 1e-6, (i, j, e)
            worst["psi"] = max(worst["psi"], e)
        rng = np.random.default_rng(100 * i + j)
        cols = rng.choice(m, size=min(8, m), replace=False)
        rows = rng.choice(m, size=min(8, m), replace=False)
        Vc = Qd[torch.as_tensor(cols, device=Qd.device)].cpu().numpy().T
        Vr = Qd[torch.as_tensor(rows, device=Qd.device)].cpu().numpy().T
        Ar_ref = Vr.T @ (A @ Vc)
        ea = np.abs(Ar[np.ix_(rows, cols)] - Ar_ref).max() / np.abs(np.diag(Ar)).max()
        assert ea <= 1e-12, (i, j, ea)
        worst.update(sol=max(worst["sol"], err), res=max(worst["res"], rel),
                     basis=max(worst["basis"], dist), Ar=max(worst["Ar"], ea))
    st = res.stats
    print(f"{WL.name} {precision} group {group}: m {m}, solved {st['n_solved']}, its {st['total_its']}, "
          f"sweeps {sum(r['restarts'] for r in res.records)}, FP64 fallback sweeps "
          f"{sum(r['fp64_sweeps'] for r in res.records)}; sampled max rel. error vs oracle: "
          f"solution {worst['sol']:.2e}, true residual {worst['res']:.2e}, reference outside "
          f"range(V) {worst['basis']:.2e}, Psi_r {worst['psi']:.2e}, A_r {worst['Ar']:.2e}")
    res.close()
    prob.close()
