"""Benchmark: full-order solves/sec of the recycled-CG sequence (Algorithm 2, CG form)
on one MI355X, plus the stencil SpMM HBM bandwidth, the roofline position of the
dominant kernel, and the CPU oracle timed on a bounded sample of the same workload.

A step = one pass of the whole path on the workload: assemble A_* (Sec. 3), run
rom_solve_sequence over every parameter point and right-hand side (Sec. 4.3), and
form the reduced matrices of eq. (newreduced) at the last point.  Inputs (grid,
parameters, U_0) are resident before the timed region; one JSON line goes to stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_outer_projection_cube64.md")


def traffic_ratio():
    """Measured HBM bytes / algorithmic bytes of the outer-projection kernels (the fused
    k_gemvn4x3 and the plain k_gemvn4<false>; rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated
    on a plain copy), from the committed profile; None if it was taken on other kernels."""
    try:
        for line in open(TRAFFIC_PROFILE):
            if line.startswith("traffic_ratio_outer_fused:"):
                return float(line.split(":", 1)[1])
    except OSError:
        pass
    return None
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(wl, points, n_sample_rhs: int):
    """The FP64 oracle, untuned, on a bounded sample: assembly plus point 0 for the first
    n_sample_rhs right-hand sides (orthonormalise U_0, outer projections, deflated CG,
    appends)."""
    import threadpoolctl

    import phantoms as ph
    from oracle import operator as op
    from oracle import sequence as oseq
    t0 = time.perf_counter()
    D = ph.diffusion_field(wl)
    As = op.assemble_Astar(wl.dim, wl.N, wl.bc, D, wl.robin_A)
    p = points[0]
    mu = op.mu_field(wl.dim, wl.N, p.mu0, p.centers, p.radii, p.amps)
    si, di = ph.rhs_nodes(wl)
    ss, ds = ph.rhs_scales(wl)
    B = oseq.rhs_matrix(wl.n, si, ss, di, ds)[:, :n_sample_rhs]
    U0 = ph.smooth_modes(wl)
    res = oseq.solve_sequence(As, [mu], B, U0, wl.tol, wl.trunc, keep_X=False)
    dt = time.perf_counter() - t0
    info = threadpoolctl.threadpool_info()
    cores = max([d.get("num_threads", 1) for d in info] + [1])
    its = sum(r.its for r in res.records)
    return {"value": n_sample_rhs / dt, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{wl.name}: assembly + point 0, right-hand sides 1-{n_sample_rhs} "
                      f"({its} CG iterations) in {dt:.1f} s; scipy.sparse products single-threaded, "
                      f"dense NumPy/BLAS on {cores} threads"}


def spmm_bandwidth(prob, point, k: int, reps: int = 10):
    """HBM GB/s of the stencil SpMM Y = A(p) X over k columns (rom_apply_operator).

    Calls alternate between two (X, Y) pairs (2 x 270 MB at 64^3, k = 64), so no call finds
    its operands in the 256 MB Infinity Cache left there by the call before.  The timed calls
    are queued behind a spinning kernel, so host-side launch cost leaves no gaps between
    them; each timed call is the whole entry point (mu(p) on the nodes, then the product)."""
    import torch
    from paper_1602_00138_amd import rom as R
    n = prob.n
    Xs = [torch.randn((k, n), dtype=torch.float64, device="cuda") for _ in range(2)]
    Ys = [torch.empty_like(Xs[0]) for _ in range(2)]
    scratch = torch.empty(8 * n, dtype=torch.uint8, device="cuda")
    for j in range(2):
        R.rom_apply_operator(prob.op, point, Xs[j], Ys[j], k, scratch)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    def timed(call):
        torch.cuda._sleep(20_000_000)
        e0.record(st)
        for r in range(reps):
            call(r)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = timed(lambda r: R.rom_apply_operator(prob.op, point, Xs[r % 2], Ys[r % 2], k, scratch))
    # for comparison: the same calls on one operand pair (resident in the Infinity Cache
    # after the first), and a plain device copy of the same footprint on alternating pairs
    ms_res = timed(lambda r: R.rom_apply_operator(prob.op, point, Xs[0], Ys[0], k, scratch))
    ms_copy = timed(lambda r: Ys[r % 2].copy_(Xs[r % 2]))
    var = prob.D_field is not None
    by = n * (16.0 * k + 8.0 + (24.0 if var else 0.0))
    return {"k": k, "bytes": by, "ms": ms, "GBps": by / ms / 1e6,
            "frac_of_peak": by / ms / 1e6 / HBM_PEAK_GBS,
            "resident_ms": ms_res, "resident_GBps": by / ms_res / 1e6,
            "copy_ms": ms_copy, "copy_GBps": 16.0 * n * k / ms_copy / 1e6,
            "note": "Y = A(p) X, X and Y N x k FP64; bytes = N(16k + 8) (+24N with a D field); "
                    "each timed call also evaluates mu(p) on the nodes (counted as time, not "
                    "bytes); calls alternate between two operand pairs larger than the "
                    "Infinity Cache together; resident_*: repeated calls on one pair; copy_*: "
                    "a plain device copy of X to Y (16 N k bytes read+written) on alternating "
                    "pairs"}


def measure_forms(prob, pts, wl, steps: int):
    """The other forms of the method on the same problem: mixed precision, groups of 8,
    and both (solves/s over `steps` timed solve_sequence calls after one warm-up)."""
    import torch
    from paper_1602_00138_amd import rom as R
    forms = {"mixed": dict(precision=R.ROM_PREC_MIXED),
             "fp64_group8": dict(group=8),
             "mixed_group8": dict(precision=R.ROM_PREC_MIXED, group=8)}
    out = {}
    K, n_rhs = len(pts), prob.n_rhs
    for name, kw in forms.items():
        kw = dict(kw, tune=1)
        prob.solve(pts, wl.tol, wl.trunc, cap=wl.cap, keep_X=False, **kw).close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = None
        for _ in range(steps):
            if last is not None:
                last.close()
            last = prob.solve(pts, wl.tol, wl.trunc, cap=wl.cap, keep_X=False, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = last.stats
        out[name] = {"value": K * n_rhs * steps / dt, "ms_per_step": 1e3 * dt / steps,
                     "basis_m": st["m"], "inner_its": st["total_its"], "solved": st["n_solved"],
                     "nonconverged": st["n_nonconv"]}
        last.close()
        log(f"form {name}: {out[name]['value']:.1f} solves/s, m={st['m']}, its={st['total_its']}")
    return out


def measure_jacobian(prob, pts, wl, plain_value: float, res, reps: int = 5):
    """The reduced Jacobian (eq. (newjac) on the basis) at the last point: rom_reduced_jacobian
    on the basis `res` of one sequence is timed; the full-order Jacobian by the adjoint
    approach would need n_src + n_det solves at that point."""
    import torch
    J = prob.reduced_jacobian(res, pts[-1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        J = prob.reduced_jacobian(res, pts[-1])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    out = {"ms": ms, "params": int(J.shape[0]), "shape": [int(J.shape[1]), int(J.shape[2])],
           "basis_m": res.m, "full_order_estimate_ms": 1e3 * prob.n_rhs / plain_value,
           "note": "per call: A_r(p), its inverse Cholesky factor, the lifted states and "
                   "co-states V A_r^{-1} [B_r, C_r], one weighted product per parameter; "
                   "the full-order estimate is n_src + n_det solves at the plain rate"}
    log(f"reduced Jacobian: {ms:.2f} ms for {out['params']} parameters "
        f"({out['shape'][0]}x{out['shape'][1]} each, m={out['basis_m']})")
    return out


def measure_frequency(prob, pts, wl, res, sigma=(0.3, 1.0, 3.0, 10.0), nb: int = 8,
                      reps: int = 3):
    """Nonzero frequency at the last point: the full-order shifted systems of eq. (solves)
    for nb right-hand sides (sources) and the given sigma = omega/nu by rom_shifted_solve
    (to relative residual wl.tol), and the reduced response of the basis `res` at the same
    shifts by rom_reduced_response.  Right-hand sides are resident before timing."""
    import torch
    p = pts[-1]
    B = torch.zeros((nb, prob.n), dtype=torch.float64)
    idx = prob.src_idx[:nb]
    B[np.arange(idx.size), torch.from_numpy(np.asarray(idx, dtype=np.int64))] = \
        torch.from_numpy(np.asarray(prob.src_scale[:nb], dtype=np.float64))
    B = B.to(prob.device)
    prob.shifted_solve(p, B, sigma, tol=wl.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        X, its, resid, _ = prob.shifted_solve(p, B, sigma, tol=wl.tol)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    Psi = prob.reduced_response(res, p, sigma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        Psi = prob.reduced_response(res, p, sigma)
    torch.cuda.synchronize()
    ms_r = 1e3 * (time.perf_counter() - t0) / reps
    out = {"shifts": list(sigma), "rhs": int(idx.size),
           "shifted_solve_ms": ms, "shifted_solves_per_s": idx.size * len(sigma) / (ms / 1e3),
           "cg_its_max": int(its.max()), "max_true_resid": float(resid.max()),
           "reduced_response_ms": ms_r, "basis_m": res.m,
           "note": "multi-shift CG: one real CG on A(p) per right-hand side serves every "
                   "shift; reduced response via the SPD system (A_r + sigma^2 A_r^-1) y_r = B_r"}
    log(f"frequency: {idx.size} RHS x {len(sigma)} shifts in {ms:.1f} ms "
        f"({out['shifted_solves_per_s']:.0f} shifted solves/s, {out['cg_its_max']} its), "
        f"reduced response {ms_r:.2f} ms (m={res.m})")
    return out


def measure_modes(prob, pts, wl, reps: int = 3, guards: int = 6):
    """The U_0 block (the k_u lowest eigenpairs of A(p_0), Algorithm 2's offline input) by
    rom_lowest_modes from the analytic smooth modes, to eigen-residual 1e-8 of the
    Gershgorin bound, with `guards` extra block columns; the starting block is resident."""
    import torch
    import phantoms as ph
    k, kx = wl.k_u, wl.k_u + guards
    X0 = torch.from_numpy(np.ascontiguousarray(ph.smooth_modes(wl, kx).T)).to(prob.device)
    prob.lowest_modes(pts[0], k, X0, tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        U, lam, sweeps = prob.lowest_modes(pts[0], k, X0, tol=1e-8)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    out = {"ms": ms, "k": k, "block": kx, "sweeps": sweeps, "filter_degree": 24,
           "lambda_min": float(lam[0]), "lambda_k": float(lam[-1]),
           "note": "Chebyshev-filtered subspace iteration; each filter step is one fused "
                   "stencil product + three-term recurrence over the block"}
    log(f"lowest modes: {ms:.2f} ms for k={k} (block {kx}), {sweeps} sweeps, "
        f"lambda {lam[0]:.4g}..{lam[-1]:.4g}")
    return out


def measure_learned_seed(prob, pts, wl, steps: int, train_steps: int, train_points: int,
                         plain_value: float, log_every=100):
    """The learned-seed form: the network is trained on the method's own solutions at
    other parameter points (untimed, reported), then every timed step runs the network
    for every (point, RHS) and the mixed-precision sequence started from its guesses."""
    import torch
    import phantoms as ph
    from paper_1602_00138_amd import driver, seed
    from paper_1602_00138_amd import rom as R
    twl = wl.replace(seed=wl.seed + 5000, K=train_points)
    tpts = driver.points_from_workload(twl)
    t0 = time.perf_counter()
    inputs, targets, Xtrain = seed.dataset(prob, tpts, wl.tol, keep_solutions=True)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = seed.SeedNet(wl.N[:3], 8, seed.he_init(5).astype(np.float32))
    t0 = time.perf_counter()
    losses = seed.train(net, inputs, targets, steps=train_steps, lr=2e-3, seed=1,
                        log=lambda m: log(m) if False else None)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del inputs, targets
    log(f"seed network: {len(tpts) * prob.n_rhs} training solutions in {t_data:.1f} s, "
        f"{train_steps} steps in {t_train:.1f} s, loss {np.mean(losses[:10]):.3e} -> "
        f"{np.mean(losses[-10:]):.3e}")
    # the second output: 16 recycle vectors per point, trained on the subspace loss
    rec_steps = max(100, train_steps // 2)
    rnet = seed.SeedNet(wl.N[:3], 4, seed.he_init(8, outputs=16).astype(np.float32), outputs=16)
    t0 = time.perf_counter()
    rlosses = seed.train_recycle(rnet, seed.point_inputs(prob, tpts), Xtrain, prob.n_rhs,
                                 steps=rec_steps, lr=2e-3, seed=2)
    torch.cuda.synchronize()
    t_rtrain = time.perf_counter() - t0
    del Xtrain
    log(f"recycle network: {rec_steps} steps in {t_rtrain:.1f} s, subspace loss "
        f"{np.mean(rlosses[:5]):.3e} -> {np.mean(rlosses[-5:]):.3e}")
    kw = dict(precision=R.ROM_PREC_MIXED, tune=1)
    g = seed.guesses(net, prob, pts)
    prob.solve(pts, wl.tol, wl.trunc, cap=wl.cap, keep_X=False, guess=g, **kw).close()
    torch.cuda.synchronize()
    t_inf = 0.0
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        if last is not None:
            last.close()
        ti = time.perf_counter()
        g = seed.guesses(net, prob, pts)
        torch.cuda.synchronize()
        t_inf += time.perf_counter() - ti
        last = prob.solve(pts, wl.tol, wl.trunc, cap=wl.cap, keep_X=False, guess=g, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    K, n_rhs = len(pts), prob.n_rhs
    st = last.stats
    drops = [np.log10(r["rho0"] / r["rho_guess"]) for r in last.records
             if r["solved"] and r["rho_guess"] > 0]
    out = {"value": K * n_rhs * steps / dt, "ms_per_step": 1e3 * dt / steps,
           "inference_ms_per_step": 1e3 * t_inf / steps, "vs_plain_fp64": K * n_rhs * steps / dt / plain_value,
           "basis_m": st["m"], "inner_its": st["total_its"], "solved": st["n_solved"],
           "mean_log10_residual_drop": float(np.mean(drops)) if drops else 0.0,
           "training": {"points": len(tpts), "solutions": len(tpts) * n_rhs, "steps": train_steps,
                        "batch": 8, "data_s": t_data, "train_s": t_train,
                        "loss_first": float(np.mean(losses[:10])),
                        "loss_last": float(np.mean(losses[-10:]))},
           "precision": "mixed", "group": 1}
    last.close()
    log(f"learned seed (mixed): {out['value']:.1f} solves/s, its {st['total_its']}, "
        f"inference {out['inference_ms_per_step']:.0f} ms/step, residual drop 10^{out['mean_log10_residual_drop']:.2f}")
    # both outputs: guesses and recycle vectors, inference inside every timed step
    g = seed.guesses(net, prob, pts)
    rv = seed.recycle_vectors(rnet, prob, pts)
    prob.solve(pts, wl.tol, wl.trunc, cap=wl.cap, keep_X=False, guess=g, recycle=rv, **kw).close()
    torch.cuda.synchronize()
    t_inf = 0.0
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        if last is not None:
            last.close()
        ti = time.perf_counter()
        g = seed.guesses(net, prob, pts)
        rv = seed.recycle_vectors(rnet, prob, pts)
        torch.cuda.synchronize()
        t_inf += time.perf_counter() - ti
        last = prob.solve(pts, wl.tol, wl.trunc, cap=wl.cap, keep_X=False, guess=g, recycle=rv, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st2 = last.stats
    out["with_recycle_vectors"] = {
        "value": K * n_rhs * steps / dt, "ms_per_step": 1e3 * dt / steps,
        "inference_ms_per_step": 1e3 * t_inf / steps,
        "vs_plain_fp64": K * n_rhs * steps / dt / plain_value, "basis_m": st2["m"],
        "inner_its": st2["total_its"], "solved": st2["n_solved"],
        "training": {"steps": rec_steps, "batch": 4, "train_s": t_rtrain,
                     "loss_first": float(np.mean(rlosses[:5])),
                     "loss_last": float(np.mean(rlosses[-5:]))}}
    last.close()
    net.close()
    rnet.close()
    log(f"learned seed + recycle vectors (mixed): {out['with_recycle_vectors']['value']:.1f} "
        f"solves/s, its {st2['total_its']}, inference "
        f"{out['with_recycle_vectors']['inference_ms_per_step']:.0f} ms/step")
    return out


def measure_concurrent(names, steps: int, **kw):
    """Independent sequences on uneven grids: solves/s run one after another vs all at
    once (rom_solve_sequences, one stream and host thread each)."""
    import torch
    import phantoms as ph
    from paper_1602_00138_amd import driver
    wls = [ph.WORKLOADS[n] for n in names]
    probs = [driver.problem_from_workload(w) for w in wls]
    pts = [driver.points_from_workload(w) for w in wls]
    tol = wls[0].tol
    total = sum(len(p) * pr.n_rhs for p, pr in zip(pts, probs))
    for r in driver.solve_many(probs, pts, tol, **kw):
        r.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for prob, p in zip(probs, pts):
            prob.solve(p, tol, keep_X=False, **kw).close()
    torch.cuda.synchronize()
    serial = total * steps / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    for _ in range(steps):
        for r in driver.solve_many(probs, pts, tol, **kw):
            r.close()
    torch.cuda.synchronize()
    conc = total * steps / (time.perf_counter() - t0)
    log(f"{'+'.join(names)}: serial {serial:.1f} solves/s, concurrent {conc:.1f} solves/s")
    return {"workloads": {w.name: "x".join(map(str, w.N[:w.dim])) for w in wls},
            "solves": total, "serial": serial, "concurrent": conc}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube64")
    ap.add_argument("--points", type=int, default=0, help="parameter points (0: the workload's)")
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--mode", default="independent", choices=["independent", "drift"])
    ap.add_argument("--cpu-sample", type=int, default=24, help="oracle sample RHS (0: skip)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64: plain FP64 recycled CG; mixed: FP32 inner sweeps in FP64 refinement")
    ap.add_argument("--group", type=int, default=1,
                    help="right-hand sides per batch (1: the paper's order, up to 16)")
    ap.add_argument("--tune", type=int, default=1, help="autotune the CG launch shape (0/1)")
    ap.add_argument("--graph", type=int, default=0, help="replay CG steps from captured HIP graphs")
    ap.add_argument("--forms", type=int, default=1,
                    help="also time the mixed / grouped forms on the same problem (0/1)")
    ap.add_argument("--jacobian", type=int, default=1,
                    help="time the reduced Jacobian at the last point (0/1)")
    ap.add_argument("--frequency", type=int, default=1,
                    help="time the nonzero-frequency solves and reduced response (0/1)")
    ap.add_argument("--modes", type=int, default=1,
                    help="time the lowest-eigenpair block U_0 at the first point (0/1)")
    ap.add_argument("--suite", type=int, default=0,
                    help="also time the uneven-grid workload (48^3, 64^3, 96^3 sequences)")
    ap.add_argument("--seed-steps", type=int, default=0,
                    help="train the seed network this many steps and time the learned-seed form")
    ap.add_argument("--seed-points", type=int, default=16, help="training points for the seed network")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run 3 plain device copies of 1 GiB (the reference for the "
                         "HBM traffic counters) and exit")
    ap.add_argument("--kernel", default="outer",
                    help="kernel class for the roofline (outer: the per-RHS start x0 = V c, "
                         "k_gemvn4x3 fused with the previous append's Gram-Schmidt pass or "
                         "k_gemvn4<false>; auto: the class with the most event time)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU "
                                   "sharding is a design note, not implemented)"}))
        sys.exit(2)

    import torch

    if args.copy_calibration:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)
        return

    import phantoms as ph
    from paper_1602_00138_amd import driver
    from paper_1602_00138_amd import rom as R

    assert torch.cuda.is_available(), "bench needs a GPU"
    wl = ph.WORKLOADS[args.workload]
    if args.points:
        wl = wl.replace(K=args.points)
    if args.tol:
        wl = wl.replace(tol=args.tol)
    prob = driver.problem_from_workload(wl)
    pts = driver.points_from_workload(wl, mode=args.mode)
    K, n_rhs = len(pts), prob.n_rhs
    dev = torch.device("cuda:0")

    # caller-owned buffers, allocated once outside the timed region
    prec = R.ROM_PREC_MIXED if args.precision == "mixed" else R.ROM_PREC_FP64
    opts_all = R.make_opts(wl.tol, wl.trunc, wl.cap, timing=(1 << R.ROM_NK) - 1, precision=prec,
                           group=args.group, tune=args.tune, graph=args.graph)
    nbytes = R.rom_sequence_bytes(prob.op, prob.src_idx.size, prob.det_idx.size, prob.k_u, K, opts_all)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    X = torch.empty((K * n_rhs, prob.n), dtype=torch.float64, device=dev)
    log(f"workload {wl.name}: grid {wl.N[:wl.dim]}, n={prob.n}, {n_rhs} RHS x {K} points, "
        f"tol {wl.tol}, workspace {nbytes / 2**30:.2f} GiB")

    def step(opts):
        R.rom_assemble_operator(prob.grid, 0.0 if prob.D_field is not None else float(wl.D),
                                prob.D_field, prob.op_mem)
        status, basis, recs, st = R.rom_solve_sequence(
            prob.op, pts, prob.src_idx, prob.src_scale, prob.det_idx, prob.det_scale, prob.U0,
            prob.k_u, opts, ws, X)
        n, m = R.rom_basis_dims(basis)
        Ar = torch.empty((m, m), dtype=torch.float64, device=dev)
        Br = torch.empty((prob.src_idx.size, m), dtype=torch.float64, device=dev)
        Cr = torch.empty((prob.det_idx.size, m), dtype=torch.float64, device=dev)
        Er = torch.empty((m, m), dtype=torch.float64, device=dev)
        scr = torch.empty(R.rom_reduced_bytes(basis), dtype=torch.uint8, device=dev)
        R.rom_reduced_transfer(basis, pts[-1], Ar, Br, Cr, Er, scr)
        R.rom_basis_destroy(basis)
        return status, recs, R.stats_dict(st)

    # warmup (all kernel classes timed, to find the dominant one)
    stats_w = None
    for w in range(max(args.warmup, 1)):
        t = time.perf_counter()
        status, recs, stats_w = step(opts_all)
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.perf_counter() - t:.2f} s, m={stats_w['m']}, "
            f"solved {stats_w['n_solved']}/{K * n_rhs}, its {stats_w['total_its']}")
    kern = stats_w["kernels"]
    for name, d in kern.items():
        if d["launches"] and d["ms"] > 0:
            log(f"  {name:11s} launches {d['launches']:7d}  {d['ms']:9.2f} ms  "
                f"{d['bytes'] / max(d['ms'], 1e-9) / 1e6:8.0f} GB/s (algorithmic)")
    dom = args.kernel
    if dom == "auto":
        dom = max((k for k in kern if k != "other"), key=lambda k: kern[k]["ms"])
    cls = R.KERNEL_CLASSES.index(dom)
    opts = R.make_opts(wl.tol, wl.trunc, wl.cap, timing=1 << cls, precision=prec, group=args.group,
                       tune=args.tune, graph=args.graph)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg = {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "launches": 0}
    bad = 0
    last = None
    for s in range(args.steps):
        status, recs, st = step(opts)
        d = st["kernels"][dom]
        for k in agg:
            agg[k] += d[k]
        bad += sum(1 for r in recs if not r["converged"])
        last = st
        log(f"step {s}: {st['seconds']:.3f} s in solve_sequence")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = K * n_rhs * args.steps
    value = solves / dt

    avg_ms = agg["ms"] / max(agg["launches"], 1)
    bound = "mfma" if dom == "gram" else "hbm"
    if bound == "hbm":
        achieved = agg["bytes"] / max(agg["ms"], 1e-12) / 1e6
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    else:
        achieved = agg["flops"] / max(agg["ms"], 1e-12) / 1e9
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None}
    roof.update({"kernel": dom, "launches": agg["launches"], "avg_launch_us": 1e3 * avg_ms,
                 "bytes_per_launch": agg["bytes"] / max(agg["launches"], 1)})
    # the counters were taken on cube64 (plain FP64, sequential order); elsewhere: null
    tr = traffic_ratio() if (dom == "outer" and args.precision == "fp64" and args.group == 1
                             and wl.name == "cube64") else None
    if tr is not None:
        roof["traffic"] = tr * roof["bytes_per_launch"]
        roof["traffic_source"] = "profiles/traffic_outer_projection_cube64.md (ratio %.3f)" % tr

    spmm = spmm_bandwidth(prob, pts[-1], 64)
    log(f"SpMM k=64: {spmm['GBps']:.0f} GB/s ({100 * spmm['frac_of_peak']:.1f}% of 8 TB/s); "
        f"operands resident {spmm['resident_GBps']:.0f} GB/s; plain copy {spmm['copy_GBps']:.0f} GB/s")

    jac = freq = None
    if args.jacobian or args.frequency:
        basis = prob.solve(pts, wl.tol, wl.trunc, cap=wl.cap, keep_X=False)
        jac = measure_jacobian(prob, pts, wl, value, basis) if args.jacobian else None
        freq = measure_frequency(prob, pts, wl, basis) if args.frequency else None
        basis.close()
    modes = measure_modes(prob, pts, wl) if args.modes else None
    forms = measure_forms(prob, pts, wl, args.steps) if args.forms else None
    if forms:
        for f in forms.values():
            f["vs_plain_fp64"] = f["value"] / value
    learned = None
    if args.seed_steps > 0:
        learned = measure_learned_seed(prob, pts, wl, args.steps, args.seed_steps,
                                       args.seed_points, value)
    suite = None
    if args.suite:
        from paper_1602_00138_amd import rom as R2
        suite = measure_concurrent(["uneven48", "uneven64", "uneven96"], 1, precision=R2.ROM_PREC_MIXED,
                                   group=8, tune=1)

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(wl, ph.parameter_points(wl, mode=args.mode), args.cpu_sample)
        log(f"cpu oracle: {cpu['value']:.3f} solves/s ({cpu['sample']})")

    out = {
        "metric": "full-order solves/sec at 1e-8 rel. residual; SpMM HBM GB/s vs peak",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == R.ROM_PREC_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {'x'.join(map(str, wl.N[:wl.dim]))} grid, "
                               f"{wl.n_src}+{wl.n_det} RHS, {K} points ({args.mode}), tol {wl.tol}, "
                               + ("plain FP64 recycled CG" if prec == R.ROM_PREC_FP64 else
                                  "FP32 inner recycled CG in FP64 refinement")
                               + (f", groups of {args.group} RHS" if args.group > 1 else ""),
                   "group": args.group, "precision": args.precision,
                   "n": prob.n, "points": K, "rhs": n_rhs, "tol": wl.tol,
                   "basis_m": last["m"], "inner_its": last["total_its"],
                   "solved": last["n_solved"], "nonconverged": bad},
        "roofline": roof,
        "spmm": spmm,
        "forms": forms,
        "reduced_jacobian": jac,
        "lowest_modes": modes,
        "frequency": freq,
        "learned_seed": learned,
        "uneven_grids": suite,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
