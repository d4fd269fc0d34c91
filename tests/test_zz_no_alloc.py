"""GPU check of the allocation-free operator product rom_apply_operator_static against
rom_apply_operator (the same kernels, caller scratch): equal to the last bit, on two calls
in a row with the second on a smaller problem, and against the oracle's CSR product to
rounding (1e-14 relative).  Sizes beyond ROM_STATIC_MAX_N are rejected before any work."""
import numpy as np
import pytest

import phantoms as ph
from helpers import OracleProblem

pytestmark = pytest.mark.gpu


def _pair(drv, R, torch, wl, k, seed):
    orc = OracleProblem(wl)
    prob = drv.problem_from_workload(wl)
    pt = drv.points_from_workload(wl)[1]
    X = torch.as_tensor(np.random.default_rng(seed).standard_normal((k, wl.n)), device="cuda")
    Y_ref = prob.apply(pt, X)
    Y = torch.full_like(X, float("nan"))
    R.rom_apply_operator_static(prob.op, pt, X, Y, k)
    torch.cuda.synchronize()
    Y, Y_ref = Y.cpu().numpy(), Y_ref.cpu().numpy()
    cpu = (orc.A(1) @ X.cpu().numpy().T).T
    prob.close()
    return Y, Y_ref, cpu


def test_static_apply_matches_scratch_apply(gpu):
    import torch
    from paper_1602_00138_amd import driver as drv
    from paper_1602_00138_amd import rom as R
    # first call: a D field and an even nx (two-node product, several columns per thread);
    # second call: a smaller grid with constant D and odd nx (one node per thread)
    for wl, k, seed in ((ph.small(3, (22, 20, 18), D="lognormal"), 5, 1),
                        (ph.small(3, (9, 8, 7)), 3, 2)):
        print(f"static apply: grid {wl.N}, k={k}", flush=True)
        Y, Y_ref, cpu = _pair(drv, R, torch, wl, k, seed)
        assert np.array_equal(Y, Y_ref), (wl.N, k)
        assert np.abs(Y - cpu).max() <= 1e-14 * np.abs(cpu).max(), (wl.N, k)


def test_static_apply_rejects_large_grid(gpu):
    import torch
    from paper_1602_00138_amd import rom as R
    n = (130, 130, 130)
    assert n[0] * n[1] * n[2] > R.ROM_STATIC_MAX_N
    g = R.make_grid(3, n, (0, 0, 0, 0, 1, 1), 1.0)
    mem = torch.empty(R.rom_operator_bytes(g, False), dtype=torch.uint8, device="cuda")
    op = R.rom_assemble_operator(g, 0.03, None, mem)
    X = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    pt = R.MuParams(0.01, np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    with pytest.raises(R.RomError) as e:
        R.rom_apply_operator_static(op, pt, X, X, 1)
    assert e.value.status == R.ROM_ECAPACITY
    R.rom_operator_destroy(op)
