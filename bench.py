"""Benchmark of the ghost-gluon DSE hot path on one MI355X.

A step is one Newton iteration of the N = 64 workload (64 Chebyshev
coefficients per dressing function, 256+64 radial x 64 angular quadrature,
decoupling G(0) = 15): the FP64 LU solve of J Delta = F for the matrix held
from the previous step, the update c - Delta, and the Newton matrix and
residual assembly at the new point (dressing, fused point kernels, B.T
contraction on MFMA, assembly), which the next step solves with.
value = Newton-matrix entries (n^2 = 128^2) per second of step time.

Beside it: seconds per Newton solve at N = 64, the 256-problem family solved
batched against the plain path per problem, the implicit-function gradient
against finite differences of re-solves, and the mixed-precision Newton matrix
against FP64 at N = 128 (each on the same GPU, at equal convergence).

Prints one JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
GLUON_SCALAR_FLOPS = 100        # per gluon point, besides the Chebyshev work
GHOST_SCALAR_FLOPS = 60


def gluon_point_flops(cfg: dict) -> float:
    """Algorithmic flops of one launch of the gluon point kernel (Jacobian mode):
    per point (row, radial node, angle) the recurrence 2 max(N), the two series
    and the two k-side targets 4 (N_Z + N_G), and the scalar work of z, s(z),
    the kernels, two exponentials and one logarithm; rows = N_Z + 1."""
    nz, ng = cfg["n_z"], cfg["n_g"]
    pts = (cfg["n_rad"] + cfg["n_ir"]) * cfg["n_ang"] * (nz + 1)
    return pts * (2 * max(nz, ng) + 4 * (nz + ng) + GLUON_SCALAR_FLOPS)


def ghost_point_flops(cfg: dict) -> float:
    nz, ng = cfg["n_z"], cfg["n_g"]
    pts = (cfg["n_rad"] + cfg["n_ir"]) * cfg["n_ang"] * (ng + 1)
    return pts * (6 * nz + GHOST_SCALAR_FLOPS)


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs summarised under profiles/, or None when the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "point_kernel_gluon_n64_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_1206_1779_amd", "csrc", "dse_kernels.hip")
    try:
        vals = {}
        for line in open(path):
            k, _, v = line.strip().partition(": ")
            vals[k] = v
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if vals.get("kernel_source_sha256") != sha or vals.get("traffic_kernel") != kernel:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


# compiler flags of the oracle library the CPU timings use (set in main)
ORACLE_BUILD = "gcc -O2 -fopenmp (portable build)"


def select_oracle_build() -> None:
    """Times the oracle as built for this host (-O3 -march=native, FMA
    contraction off: the same arithmetic as the portable -O2 build the tests
    use); keeps the portable build when that compile fails."""
    global ORACLE_BUILD
    import subprocess
    import oracle
    try:
        ORACLE_BUILD = oracle.use_native_build()
    except (RuntimeError, OSError, subprocess.CalledProcessError) as e:
        print("oracle: host-tuned build unavailable (%s), timing the portable one" % e, file=sys.stderr)


def cpu_baseline(cfg: dict, c, cpu_seconds: float = 20.0, max_steps: int = 50) -> dict:
    """The oracle (plain FP64 C, OpenMP over rows, all host threads) doing the
    same step on the host: LU solve of the held Newton matrix, update, Newton
    matrix and residual at the new point; repeated until about `cpu_seconds` of
    CPU time (wall time x threads) have been spent, at most max_steps times."""
    import numpy as np
    import oracle
    p = oracle.params(**cfg)
    c = np.asarray(c, dtype=np.float64)
    n = p.n_z + p.n_g
    threads = oracle.get_threads()
    J, F = oracle.jacobian(p, c, with_F=True)  # the matrix the first step solves with
    steps = 0
    t0 = time.perf_counter()
    while True:
        c = c - oracle.lu_solve(J, F)
        J, F = oracle.jacobian(p, c, with_F=True)
        steps += 1
        dt = time.perf_counter() - t0
        if dt * threads >= cpu_seconds or steps >= max_steps:
            break
    return {"value": n * n * steps / dt, "unit": "Jacobian entries/s", "cores": threads,
            "kind": "oracle", "build": ORACLE_BUILD, "seconds": dt, "steps": steps,
            "sample": "%d Newton iterations (LU solve, update, J and F at the new point) of the N=64 "
                      "workload from the start guess, %d host threads" % (steps, threads)}


def root_errors(c_gpu, gold: dict) -> dict:
    """Error of converged coefficients against the oracle's root stored in
    tests/golden/oracle_roots.json: largest absolute difference, largest
    elementwise relative difference over |c_j| >= 1e-6 ||c||_inf, and the
    componentwise condition bound and one-ulp floor stored with the root."""
    import numpy as np
    c = np.asarray(c_gpu, dtype=np.float64)
    cr = np.asarray(gold["c"], dtype=np.float64)
    big = np.abs(cr) >= 1e-6 * np.abs(cr).max()
    return {"max_abs": float(np.abs(c - cr).max()),
            "max_elementwise_rel": float((np.abs(c - cr)[big] / np.abs(cr)[big]).max()),
            "bound": gold["bound"], "floor": gold["floor"]}


def load_oracle_roots() -> dict:
    with open(os.path.join(ROOT, "tests", "golden", "oracle_roots.json")) as f:
        return json.load(f)


def bench_root_parity(dse, workloads, torch) -> dict:
    """Converged FP64 coefficients at N = 16 and N = 64 (two full steps after
    convergence, as the stored oracle roots) against the oracle's."""
    gold = load_oracle_roots()
    out = {}
    for name in ("cfg1", "cfg2"):
        s = dse.Solver(**workloads.config(name))
        r = s.newton(extra_iters=2)
        out[name] = dict(root_errors(r.c.cpu().numpy(), gold[name]), iters=r.iters)
    return out


def bench_batched(dse, workloads, torch) -> dict:
    """The 256-problem family (G(0) log-uniform in [5, 50], N_Z, N_G in
    {32, 48, 64}, 256+64 x 64) solved by one batched Newton iteration against
    the plain path run once per problem (one context per (N_Z, N_G), G(0) set
    per problem), both from the asymptotic start to scaled residual < 1e-10."""
    fam = workloads.family(256)
    b = dse.Batch(fam)
    c0 = b.start_guess()
    tune = b.autotune(c0)
    b.newton(c0.clone())  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, res = b.newton(c0.clone())
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    solvers = {}
    for f in fam:
        key = (f["n_z"], f["n_g"])
        if key not in solvers:
            solvers[key] = dse.Solver(**f)
            solvers[key].newton()  # warm-up
    t_plain, iters_plain, dmax = 0.0, [], 0.0
    for i, f in enumerate(fam):
        s = solvers[(f["n_z"], f["n_g"])]
        s.set_physics(g0_inv=f["g0_inv"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.newton()
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        iters_plain.append(r.iters)
        d = float((r.c - res[i].c).abs().max() / r.c.abs().max())
        dmax = max(dmax, d)
    entries = sum((f["n_z"] + f["n_g"]) ** 2 for f in fam)
    return {"problems": len(fam), "batched_s": t_batch, "plain_s": t_plain, "speedup": t_plain / t_batch,
            "all_converged": all(r.status == 0 for r in res),
            "iters_batched_max": max(r.iters for r in res), "iters_plain_max": max(iters_plain),
            "max_rel_coeff_diff_vs_plain": dmax, "jacobian_entries_per_round": entries,
            "assembly_round_ms": tune["best_ms"],
            "assembly_entries_per_s": entries / (tune["best_ms"] * 1e-3),
            "launch": {k: tune[k] for k in ("slices", "persistent_blocks", "order", "tiles_per_item", "fused")},
            "launch_candidates": tune["candidates"]}


def bench_adjoint(dse, workloads, torch) -> dict:
    """Gradient of L = sum_m ln Z(p_m)^2 (64 log-spaced p in [1e-4, 1e4]) with
    respect to alpha(mu^2) and G(0) at N = 64: the implicit-function VJP (one
    Newton matrix at the root, one transposed LU solve, one parameter VJP)
    against central differences of full re-solves (four Newton solves, h = 1e-6),
    both after the same converged solve."""
    cfg = workloads.config("cfg5")
    s = dse.Solver(**cfg)
    pts = torch.as_tensor(workloads.adjoint_loss_points(), dtype=torch.float64, device="cuda:0")
    r = s.newton()
    c = r.c

    def ift():
        # dL/dc = sum_m 2 ln Z(p_m) d ln Z(p_m)/dc (dse_running_coupling, dse_dressing_vjp),
        # then J^T lambda = dL/dc and dL/dtheta = -lambda^T dF/dtheta
        _, lnz, _ = s.running_coupling(c, pts)
        gc = s.dressing_vjp(pts, 2.0 * lnz, None)
        J = s.jacobian(c, with_F=False)
        lam = s.lu_solve(J, gc, trans=True)
        _, ut = s.vjp(c, lam, with_c=False)
        return -ut

    def loss(alpha, g0_inv):
        s.set_physics(alpha_mu=alpha, g0_inv=g0_inv)
        rr = s.newton(c0=c)
        _, lnz, _ = s.running_coupling(rr.c, pts)
        return float((lnz ** 2).sum())

    ift()
    loss(cfg["alpha_mu"], cfg["g0_inv"])  # first use of the loss's own kernels outside the timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = ift()
    torch.cuda.synchronize()
    t_ift = time.perf_counter() - t0
    a0, gi0 = cfg["alpha_mu"], cfg["g0_inv"]
    G0, h = 1.0 / gi0, 1e-6
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fd_a = (loss(a0 + h, gi0) - loss(a0 - h, gi0)) / (2 * h)
    fd_g = (loss(a0, 1.0 / (G0 + h)) - loss(a0, 1.0 / (G0 - h))) / (2 * h)
    torch.cuda.synchronize()
    t_fd = time.perf_counter() - t0
    s.set_physics(alpha_mu=a0, g0_inv=gi0)
    g = g.cpu().tolist()
    dG0 = -g[1] / G0 ** 2
    return {"ift_s": t_ift, "fd_s": t_fd, "speedup": t_fd / t_ift,
            "dL_dalpha": {"ift": g[0], "fd": fd_a, "rel_diff": abs(g[0] - fd_a) / abs(fd_a)},
            "dL_dG0": {"ift": dG0, "fd": fd_g, "rel_diff": abs(dG0 - fd_g) / abs(fd_g)}}


def bench_fd(dse, workloads, torch) -> dict:
    """N = 64: the Newton matrix by the paper's own method, central differences
    of the residual (2n full residual evaluations, dse_jacobian_fd), against
    the analytic matrix of the same context, both on this GPU; the ratio
    separates the gain of the analytic derivatives from that of the hardware."""
    import numpy as np
    cfg = workloads.config("cfg2")
    s = dse.Solver(**cfg)
    c = s.start_guess()
    s.jacobian_fd(c)  # warm-up
    s.jacobian(c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Jfd = s.jacobian_fd(c)
    torch.cuda.synchronize()
    t_fd = time.perf_counter() - t0
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        J, _ = s.jacobian(c)
    torch.cuda.synchronize()
    t_an = (time.perf_counter() - t0) / reps
    J, Jfd = J.cpu().numpy(), Jfd.cpu().numpy()
    return {"fd_ms": t_fd * 1e3, "analytic_ms": t_an * 1e3, "speedup": t_fd / t_an,
            "residual_evaluations": 2 * s.n,
            "normwise_rel_diff": float(np.linalg.norm(J - Jfd) / np.linalg.norm(J))}


def bench_coupling(dse, workloads, torch) -> dict:
    """N = 64: the running coupling alpha(u) = alpha(mu^2) G^2 Z at 2^17
    log-spaced momenta from 1e-6 eps2 to 4 lambda2 on the converged solution
    (G(0) = 15), and its value below eps2, where the IR power laws cancel in
    G^2 Z and alpha is flat."""
    cfg = workloads.config("cfg2")
    s = dse.Solver(**cfg)
    c = s.newton().c
    m = 1 << 17
    u = torch.logspace(math.log10(cfg["eps2"]) - 6, math.log10(4 * cfg["lambda2"]), m,
                       dtype=torch.float64, device=c.device)
    s.running_coupling(c, u)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    al, _, _ = s.running_coupling(c, u)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return {"points": m, "ms": t * 1e3, "points_per_s": m / t, "alpha_ir": float(al[0]),
            "g0_inv": cfg["g0_inv"]}


def bench_lu(dse, workloads, torch, reps: int = 50) -> dict:
    """The device LU alone (dse_lu_solve: row maxima, factorisation with
    partial pivoting, solve) at the Newton orders n = 128 (N = 64) and 256
    (N = 128) on seeded Gaussian matrices with a shifted diagonal; wall time
    per call including its synchronisation, and the solution's residual."""
    import numpy as np
    out = {}
    for n in (128, 256):
        s = dse.Solver(**workloads.config("cfg1", n_z=n // 2, n_g=n - n // 2))
        rng = np.random.default_rng(n)
        A = rng.standard_normal((n, n)) + np.diag(rng.uniform(-3, 3, n))
        b = rng.standard_normal(n)
        Ad = torch.tensor(A, device="cuda:0")
        bd = torch.tensor(b, device="cuda:0")
        for _ in range(3):
            x = s.lu_solve(Ad, bd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            x = s.lu_solve(Ad, bd)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        xn = x.cpu().numpy()
        out["n%d" % n] = {"ms_per_call": dt * 1e3,
                          "rel_residual": float(np.linalg.norm(A @ xn - b) / (np.linalg.norm(A) * np.linalg.norm(xn)))}
    return out


def bench_schwinger(dse, workloads, torch, with_cpu: bool = True) -> dict:
    """The Schwinger function of the gluon propagator (Sec. 2.2; the paper's
    second workload, Table 2): the scaling solution at the paper's parameters
    (Lambda^2 = 5e4, Z(Lambda^2) = 0.256, alpha(mu^2) = 1), Delta(t) at 1024
    times t = 0.02 k GeV^-1 by the 2^17-node mapped Gauss-Legendre rule
    generated on the device (node generation included, as in Table 2); the
    node generation alone; the first zero of Delta, mu^2 (G^2 Z = 1) and
    alpha(M_Z^2).  The oracle is timed beside it on a smaller rule."""
    import numpy as np
    cfg = workloads.config("paper")
    s = dse.Solver(**cfg)
    c = s.newton(extra_iters=2).c
    W = workloads.SCHWINGER
    t = torch.as_tensor(workloads.schwinger_times(), dtype=torch.float64, device=c.device)
    n = W["n_nodes"]
    lib = dse.load()
    ws = torch.empty(lib.dse_schwinger_workspace_bytes(n, t.numel()) + 256, dtype=torch.uint8, device=c.device)
    s.schwinger(c, t, n=n, p_max=W["p_max"], ws=ws)  # warm-up
    dse.gauss_legendre(n, device=c.device)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record()
    d = s.schwinger(c, t, n=n, p_max=W["p_max"], ws=ws)
    ev[1].record()
    ev[2].record()
    dse.gauss_legendre(n, device=c.device)
    ev[3].record()
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    tt = workloads.schwinger_times()
    k = int(np.where(np.diff(np.sign(d)) != 0)[0][0])
    t0 = tt[k] - d[k] * (tt[k + 1] - tt[k]) / (d[k + 1] - d[k])
    alpha_mz, _, _ = s.running_coupling(c, torch.tensor([91.2 ** 2], dtype=torch.float64, device=c.device))
    out = {"workload": workloads.WORKLOAD_NAMES["paper"], "nodes": n, "times": int(t.numel()),
           "p_max": W["p_max"], "total_ms": ev[0].elapsed_time(ev[1]),
           "node_generation_ms": ev[2].elapsed_time(ev[3]), "first_zero_t": t0,
           "mu2": s.renorm_scale(c), "alpha_mz2": float(alpha_mz.item()),
           "paper_table2_s": {"GTX 560 Ti": 4.1, "Tesla C2070": 3.9, "Xeon X5650 sequential": 226.9}}
    if with_cpu:
        import oracle
        p = oracle.params(**cfg)
        nc = 1 << 14
        tc0 = time.perf_counter()
        oracle.gauss_legendre(nc)
        t_gl = time.perf_counter() - tc0
        tc0 = time.perf_counter()
        oracle.schwinger(p, c.cpu().numpy(), tt, n=nc, p_max=W["p_max"])
        t_all = time.perf_counter() - tc0
        # the rule is O(n^2) (n recurrence steps per node), the sum O(n m)
        out["cpu_oracle"] = {"nodes": nc, "times": len(tt), "threads": oracle.get_threads(), "build": ORACLE_BUILD,
                             "gl_s": t_gl, "total_s": t_all,
                             "total_s_extrapolated_to_nodes": t_gl * (n / nc) ** 2
                             + max(t_all - t_gl, 0.0) * (n / nc)}
    return out


def bench_discretisation(dse, workloads, torch) -> dict:
    """Accuracy against cost of the two discretisations (the shared log-GL
    radial grid with GL in theta, and the paper's split at x with tanh-sinh
    angles, Sec. 2-3) on the scaling solution at the paper's parameters,
    N = 24: per grid the device time of one Newton-matrix assembly, the Newton
    solve, the largest error of ln Z and ln G at 64 log-spaced momenta in
    [eps2, lambda2] and of N_c alpha(0) (IR fixed point 8.91512) against a
    split + tanh-sinh reference with 256 nodes per radial interval and 257
    angles."""
    base = workloads.config("paper")
    u = torch.logspace(-6, math.log10(5e4), 64, dtype=torch.float64, device="cuda:0")
    u0 = torch.tensor([base["eps2"] * 1e-6], dtype=torch.float64, device="cuda:0")

    def run(n_rad, n_ir, n_ang, quad):
        s = dse.Solver(**dict(base, n_rad=n_rad, n_ir=n_ir, n_ang=n_ang, quad=quad))
        s.newton()                 # loads the kernels
        r = s.newton(extra_iters=2)  # timed: from the start guess, two steps past convergence
        c = r.c
        s.jacobian(c)
        s.set_timing(True)
        for _ in range(10):
            s.jacobian(c)
        st, _ = s.read_timings()
        s.set_timing(False)
        _, lz, lg = s.running_coupling(c, u)
        a0, _, _ = s.running_coupling(c, u0)
        return {"n_rad": n_rad, "n_ir": n_ir, "n_ang": n_ang, "quad": quad, "assembly_ms": sum(st),
                "newton_ms": r.t_total_ms, "iters": r.iters, "status": r.status}, lz, lg, float(a0.item())

    ref, lz0, lg0, _ = run(256, 256, 257, 3)
    rows = []
    for args in ((96, 24, 24, 0), (192, 48, 32, 0), (384, 96, 64, 0), (768, 192, 128, 0), (1536, 384, 256, 0),
                 (32, 32, 33, 3), (64, 64, 65, 3), (128, 128, 129, 3)):
        row, lz, lg, a0 = run(*args)
        row["max_err_lnZ"] = float((lz - lz0).abs().max())
        row["max_err_lnG"] = float((lg - lg0).abs().max())
        row["alpha0_nc_rel_err"] = abs(base["n_c"] * a0 / 8.91512 - 1.0)
        rows.append(row)
    return {"workload": workloads.WORKLOAD_NAMES["paper"], "reference": ref, "grids": rows}


def bench_mixed(dse, workloads, torch) -> dict:
    """N = 128 per function, 1024+256 radial x 128 angular: the Newton matrix
    with FP32 derivative sums and FP32 MFMA contraction against FP64 (device
    time per assembly, J error against the FP64 matrix), and the Newton solve in
    both precisions (F and the LU in FP64 throughout): iterations, time, and the
    largest per-coefficient difference of the two roots."""
    cfg = workloads.config("cfg3")
    out = {"workload": workloads.WORKLOAD_NAMES["cfg3"]}
    solvers = {"fp64": dse.Solver(**cfg), "mixed": dse.Solver(**dict(cfg, precision=1))}
    c0 = solvers["fp64"].start_guess()
    Js = {}
    for k, s in solvers.items():
        J, _ = s.jacobian(c0)
        Js[k] = J
        s.set_timing(True)
        for _ in range(10):
            s.jacobian(c0)
        st, _ = s.read_timings()
        s.set_timing(False)
        out["assembly_ms_" + k] = sum(st)
        out["stage_ms_" + k] = st
    d = Js["mixed"] - Js["fp64"]
    out["J_normwise_rel_err"] = float(d.norm() / Js["fp64"].norm())
    out["J_worst_row_rel_err"] = float((d.abs().amax(dim=1) / Js["fp64"].abs().amax(dim=1)).max())
    roots = {}
    for k, s in solvers.items():
        s.newton(extra_iters=8)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.newton(extra_iters=8)
        torch.cuda.synchronize()
        out["newton_s_" + k] = time.perf_counter() - t0
        out["newton_iters_" + k] = r.iters
        out["newton_status_" + k] = r.status
        out["newton_fp32_matrices_" + k] = r.n_jacobians_mixed
        roots[k] = r.c
    dc = (roots["mixed"] - roots["fp64"]).abs()
    out["root_max_abs_diff"] = float(dc.max())
    out["root_max_rel_diff"] = float(dc.max() / roots["fp64"].abs().max())
    gold = load_oracle_roots()["cfg3"]
    for k in roots:
        out["root_vs_oracle_" + k] = root_errors(roots[k].cpu().numpy(), gold)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--solves", type=int, default=5, help="Newton solves timed for s/solve")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched, adjoint, mixed and finite-difference comparisons")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device five times (reference for HBM counters)")
    ap.add_argument("--leg", choices=["schwinger", "lu", "batched"], default=None,
                    help="run one secondary leg alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X and has no "
              "multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    import workloads
    from paper_1206_1779_amd import dse

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if not args.no_cpu and not args.copy_calibration:
        select_oracle_build()
    if args.copy_calibration:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb, "launches": 5}), flush=True)
        return 0
    if args.leg:
        legs = {"schwinger": lambda: bench_schwinger(dse, workloads, torch, with_cpu=False),
                "lu": lambda: bench_lu(dse, workloads, torch),
                "batched": lambda: bench_batched(dse, workloads, torch)}
        print(json.dumps({args.leg: legs[args.leg]()}), flush=True)
        return 0
    name = "cfg2"
    cfg = workloads.config(name)
    # the solver's own stream (not the legacy default stream), as a serving
    # loop would use; every tensor operation below is ordered on it
    stream = torch.cuda.Stream(device="cuda:0")
    torch.cuda.set_stream(stream)
    s = dse.Solver(device="cuda:0", stream=stream, **cfg)
    n = s.n
    # the steps run at the solution (the work per step does not depend on c)
    root = s.newton(tol=1e-10).c
    bufs = (root.clone(), torch.empty_like(root))
    F_out, S_out = torch.empty_like(root), torch.empty_like(root)

    def step(k):
        # one Newton iteration in the library: LU solve of the matrix held from
        # the previous step, update, J and F at the new point; the coefficient
        # buffers alternate, so from the second step on every step assembles once
        src, dst = bufs[k % 2], bufs[(k + 1) % 2]
        s.newton_step(src, 1.0, out=(dst, F_out, S_out))

    def timed_steps(graphs: bool) -> float:
        s.set_graphs(graphs)
        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            step(k)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # the step replayed from the library's recorded graphs, then the timed
    # region: K steps with the library's default launches (kernel by kernel,
    # the faster form here: a graph launch adds a gap of about 8 us before
    # its first kernel)
    dt_graph = timed_steps(True)
    dt = timed_steps(False)
    ms_step = dt / args.steps * 1e3
    value = n * n / (dt / args.steps)
    # the same K steps launched one by one, with HIP events around every stage
    # of the assembly on the context's stream (per-kernel durations)
    s.set_graphs(False)
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    dt_eager = time.perf_counter() - t0
    stages, cnt = s.read_timings()
    s.set_timing(False)
    s.set_graphs(False)
    c = s.start_guess()

    # Jacobian assembly alone (device time of its five stages)
    t_asm = sum(stages) * 1e-3
    # dominant kernel: the gluon point kernel, Jacobian mode
    t_gl = stages[1] * 1e-3
    a_gl = gluon_point_flops(cfg)
    achieved = a_gl / t_gl / 1e12
    roof = {"bound": "alu", "kernel": "point_kernel<gluon, 64, jacobian>",
            "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_VALU_PEAK_TFLOPS,
            "traffic": measured_traffic("void dse::point_kernel<0, 64, 1, false, false>"),
            "flops_per_launch": a_gl, "avg_launch_ms": t_gl * 1e3, "launches": cnt,
            "timed": "HIP events around each launch over the second pass of the same steps",
            "ghost_kernel_ms": stages[2], "ghost_kernel_tflops": ghost_point_flops(cfg) / (stages[2] * 1e-3) / 1e12}

    # s / Newton solve from the start guess to scaled residual < 1e-10
    times, iters, split = [float("nan")], [0], (float("nan"), float("nan"))
    if args.solves > 0:
        times, iters = [], []
    for _ in range(args.solves):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = s.newton(tol=1e-10)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        iters.append(r.iters)
        split = (r.t_assembly_ms, r.t_lu_ms)

    out = {
        "metric": "Jacobian entries/s + s/Newton-solve at N=64; batched & adjoint vs plain",
        "value": value, "unit": "Jacobian entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workloads.WORKLOAD_NAMES[name], "n_z": cfg["n_z"], "n_g": cfg["n_g"],
                   "n_rad": cfg["n_rad"], "n_ir": cfg["n_ir"], "n_ang": cfg["n_ang"],
                   "g0": 1.0 / cfg["g0_inv"],
                   "step": "LU solve of the held Newton matrix, update, J+F assembly at the new point",
                   "launch": "kernel by kernel on the solver's stream"},
        "ms_per_step_graph_replay": dt_graph / args.steps * 1e3,
        "ms_per_step_with_stage_events": dt_eager / args.steps * 1e3,
        "assembly_entries_per_s": n * n / t_asm,
        "assembly_ms": t_asm * 1e3,
        "stage_ms": dict(zip(["dressing", "gluon_points", "ghost_points", "contract", "assemble"], stages)),
        "newton_solve_s": statistics.median(times), "newton_iters": iters[0],
        "newton_solve_split_ms": {"assembly": split[0], "lu": split[1]},
        "roofline": roof,
    }
    if not args.no_extras:
        out["batched"] = bench_batched(dse, workloads, torch)
        out["adjoint"] = bench_adjoint(dse, workloads, torch)
        out["mixed"] = bench_mixed(dse, workloads, torch)
        out["fd_jacobian"] = bench_fd(dse, workloads, torch)
        out["coupling"] = bench_coupling(dse, workloads, torch)
        out["root_parity"] = bench_root_parity(dse, workloads, torch)
        out["schwinger"] = bench_schwinger(dse, workloads, torch, with_cpu=not args.no_cpu)
        out["lu"] = bench_lu(dse, workloads, torch)
        out["discretisation"] = bench_discretisation(dse, workloads, torch)
    if not args.no_cpu:
        cb = cpu_baseline(cfg, c.cpu().numpy())
        cb["gpu_speedup"] = value / cb["value"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
