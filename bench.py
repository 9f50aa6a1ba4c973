"""Benchmark of the randomized DOT hot path on one MI355X.

Workload (128^3 configuration): 3D diffusion on 128^3 cells (2,097,152
unknowns), Robin top/bottom and Dirichlet lateral faces, 256 sources on the
top face and 256 detectors on the bottom face, l_s = l_d = 20 simultaneous
sources and detectors made of 10 optimized directions (Alg. 1 on a sampled
Jacobian) plus 10 random directions in their orthogonal complement, PaLS
absorption with 64 RBFs (320 parameters).  One step is one pass of the whole
hot path:
  PaLS absorption and A(theta) -> B W and C V -> the 40 forward + adjoint
  solves to per-column relative residual 1e-8 (binary32 CG with a multigrid
  V-cycle preconditioner, in binary64 refinement) -> sampled misfit ->
  3-part split-bfloat16 sampled Jacobian (400 x 320)
  -> adjoint gradient -> Alg. 1 + lift + complement (next optimized design)
  -> thin SVD of the sampled Jacobian and the truncated-SVD Gauss-Newton
  step.
The metric is right-hand sides solved per second over whole steps.  Legs
beside it: the same 40 solves with Jacobi preconditioning only, the same
solves in binary64 CG at equal 1e-8, and the 1600 x 5000 Jacobian of the
128^3, 1000-RBF configuration (TFLOP/s).

Prints one JSON line; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import concurrent.futures
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic bytes per cell per column of each CG pass (vector streams only)
PASS_BYTES = {
    "pcg1_fp32": 12,   # read r, p_old; write p      (binary32)
    "pcg2_fp32": 20,   # read p, d, r; write d, r    (binary32)
    "pcg1_fp64": 24,
    "pcg2_fp64": 40,
    "resid": 28,       # binary64 b - A x: read b, x; write r; binary32 residual write
}


# HBM bytes per launch of the binary32 CG passes on this workload, from the
# FETCH_SIZE (x 1.99983, calibrated on a 320 MiB copy) and WRITE_SIZE counter
# runs summarized in profiles/sweep_pcg_fp32_128cube_40rhs_hbm_traffic.md; valid
# while the sweep kernel's source (solve.hip up to the end of sweep_kernel: the
# kernel and every helper it uses) hashes to the value recorded with them.
TRAFFIC = {
    "source": "paper_1706_05586_amd/csrc/solve.hip",
    "through": "void sweep_kernel(SweepArgs<T> a) {",
    "sha256": "3f1e0964647ad0c20bc183f0fceadbef64843974ca9b41d1626b7da4d44e7f0d",
    "config": "C3",
    "pcg2_fp32_bytes_per_launch": 1821000000.0,
    "pcg1_fp32_bytes_per_launch": 1411600000.0,
}


def measured_traffic(config_name):
    """Counter-measured bytes per launch, or None once the kernel has changed."""
    import hashlib
    with open(os.path.join(ROOT, TRAFFIC["source"])) as f:
        text = f.read()
    at = text.find(TRAFFIC["through"])
    if at < 0 or config_name != TRAFFIC["config"]:
        return None
    prefix = text[:text.index("\n}\n", at) + 3]
    if hashlib.sha256(prefix.encode()).hexdigest() != TRAFFIC["sha256"]:
        return None
    return TRAFFIC


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--no-jacobian-leg", action="store_true")
    ap.add_argument("--no-jacobi-leg", action="store_true")
    ap.add_argument("--no-inversion-leg", action="store_true")
    ap.add_argument("--no-frequency-leg", action="store_true")
    ap.add_argument("--no-diffusion-leg", action="store_true")
    ap.add_argument("--cpu-repeats", type=int, default=3)
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only run the CPU baseline of --config and print it as JSON")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB between two device buffers 5 times (reference "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": n * 4, "calibrate_copy_bytes_written": n * 4,
                      "launches": 5}), flush=True)


def setup_fields(dl, L, torch, dev, cfg, wl, op, pals, W, V, precision, rtol=1e-8):
    ls, ld = W.shape[1], V.shape[1]
    rhs = dl.empty_colmajor(op.N, ls + ld, dev)
    op.form_rhs(wl.src_cells, W, out=rhs[:, :ls])
    op.form_rhs(wl.det_cells, V, out=rhs[:, ls:])
    res = op.solve(rhs, rtol=rtol, precision=precision)
    return res.x[:, :ls], res.x[:, ls:]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path is built and measured on a single "
              "MI355X (the multi-GPU sharding is described in DESIGN.md, not run); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    if args.cpu_baseline_only:
        import synthetic
        print(json.dumps(cpu_baseline(synthetic.make_workload(synthetic.get_config(args.config)),
                                      args.cpu_repeats)), flush=True)
        return

    # the CPU baseline (oracle on the host, one core) runs in a child process
    # beside the GPU legs; started before this process touches the GPU
    cpu_proc = None
    if not args.no_cpu_baseline:
        import subprocess
        cpu_proc = subprocess.Popen(
            [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--config",
             args.config, "--cpu-repeats", str(args.cpu_repeats)],
            stdout=subprocess.PIPE, text=True)

    import torch

    import synthetic
    import paper_1706_05586_amd as dl
    from paper_1706_05586_amd import _lib as L

    dev = torch.device("cuda:0")
    cfg = synthetic.get_config(args.config)
    wl = synthetic.make_workload(cfg)
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    N = grid.N
    ls, ld = cfg.l_s, cfg.l_d
    k = ls + ld
    log(f"[bench] workload {cfg.name}: N={N} k={k} m0={cfg.m0} n_p={cfg.n_p}")

    # ---------------------------------------------------------------- setup
    th_ref = torch.tensor(wl.theta_ref, device=dev)
    th_true = torch.tensor(wl.theta_true, device=dev)
    _, D = dl.pals_field(grid, pals, th_ref, cfg.mus_prime)
    op = dl.Operator(grid, D)
    # synthetic data: all sources at theta_true, 0.1% relative noise (binary64
    # solves, so the binary32 pass kernels run only in the timed workload)
    op.pals_mua(pals, th_true)
    B = op.form_rhs(wl.src_cells, torch.eye(cfg.n_s, dtype=torch.float64, device=dev))
    full = op.solve(B, rtol=1e-10, precision=L.DOT_FP64)
    M_true = full.x.cpu().numpy()[wl.det_cells, :]
    data = torch.tensor(M_true * (1.0 + cfg.noise * wl.xi), device=dev)
    del B, full
    # optimized design: Alg. 1 on the sampled Jacobian of random samples, then
    # q optimized + (l - q) complementary random directions
    W0 = torch.tensor(wl.w_signs / np.sqrt(ls), device=dev)
    V0 = torch.tensor(wl.v_signs / np.sqrt(ld), device=dev)
    op.pals_mua(pals, th_ref)
    U0, Z0 = setup_fields(dl, L, torch, dev, cfg, wl, op, pals, W0, V0, L.DOT_FP64, 1e-10)
    Js0 = op.jacobian(U0, Z0, L.DOT_JAC_FP64)
    ys = torch.tensor(wl.y_signs, dtype=torch.float64, device=dev)
    zs = torch.tensor(wl.z_signs, dtype=torch.float64, device=dev)
    if cfg.q_s > 0:
        W, V, _ = dl.optimized_design(Js0, W0, V0, cfg.q_s, cfg.q_d, ys, zs)
    else:
        W, V = W0, V0
    DW = dl.gemm(data, W)
    del U0, Z0, Js0
    log(f"[bench] setup done: data from {cfg.n_s} solves, W/V = {cfg.q_s} optimized + "
        f"{ls - cfg.q_s} complementary random")

    rhs = dl.empty_colmajor(N, k, dev)
    x = dl.empty_colmajor(N, k, dev)
    work = torch.empty(op.solve_workspace_bytes(k, L.DOT_MIXED) + 256, dtype=torch.uint8,
                       device=dev)
    work = work[(-work.data_ptr()) % 256:]
    state = {}

    side = torch.cuda.Stream(device=dev)
    pool = concurrent.futures.ThreadPoolExecutor(max_workers=1)

    def design_on_side(Js, main):
        with torch.cuda.stream(side):
            Wn, Vn, info = dl.optimized_design(Js, W, V, cfg.q_s, cfg.q_d, ys, zs)
        # consumed on the main stream after it waits for this one
        Wn.record_stream(main)
        Vn.record_stream(main)
        return Wn, Vn, info

    def step(theta, precision=L.DOT_MIXED, full_path=True, precond=L.DOT_PRECOND_AUTO):
        if full_path:
            op.pals_mua(pals, theta)
            op.form_rhs(wl.src_cells, W, out=rhs[:, :ls])
            op.form_rhs(wl.det_cells, V, out=rhs[:, ls:])
        # multigrid-preconditioned CG: the column flags are polled every other
        # iteration and the binary32 residual is replaced after each drop by
        # 100 (10 iterations, 3 binary64 updates at this size; a drop by 1e4
        # saves an update on some right-hand sides and costs two iterations
        # on these)
        res = op.solve(rhs, rtol=1e-8, precision=precision, inner_rtol=0.01, check_every=2,
                       out=x, work=work, precond=precond)
        if not res.converged:
            raise RuntimeError(f"solve did not converge: {res.relres.max():.3e}")
        state["res"] = res
        marks = [time.perf_counter()]
        if full_path:
            U, Z = x[:, :ls], x[:, ls:]
            Rs, f = op.sampled_misfit(wl.det_cells, U, V, DW)
            Js = op.jacobian(U, Z, L.DOT_JAC_SPLIT_BF16X3)
            g = op.grad_misfit(U, Z, Rs)
            # the next design (Alg. 1) and the Gauss-Newton model both read
            # J_s only: the design runs on a second stream from a worker
            # thread (both sides are latency-bound and wait on the host
            # between launches), the thin SVD here
            main = torch.cuda.current_stream()
            if cfg.q_s > 0:
                side.wait_stream(main)
                fut = pool.submit(design_on_side, Js, main)
            marks.append(time.perf_counter())
            # Gauss-Newton model: thin SVD of J_s (of J_s^T when J_s is tall)
            # and the truncated-SVD step for min ||J_s d + vec(R_s)||, kept to
            # the singular values above 1e-4 s_max
            if Js.shape[1] <= Js.shape[0]:
                sv, Rv, Lv = dl.svd_thin(Js.t(), rcut=1e-10)
            else:
                sv, Lv, Rv = dl.svd_thin(Js, rcut=1e-10)
            t = int((sv > 1e-4 * sv[0]).sum().item())
            d = dl.tsvd_step(Lv, sv, Rv, Rs.t().reshape(-1), t)
            state.update(f=f, Js=Js, g=g, sv=sv, gn_step=d, gn_rank=t)
            marks.append(time.perf_counter())
            if cfg.q_s > 0:
                Wn, Vn, info = fut.result()
                main.wait_stream(side)
                state.update(W_next=Wn, V_next=Vn, hooi_iters=info["hooi_iters"])
            marks.append(time.perf_counter())
        state.setdefault("marks", []).append(marks)

    for _ in range(args.warmup):
        step(th_ref)
    torch.cuda.synchronize()
    # inside the timed steps only the roofline kernel (CG pass 2) and the
    # contraction carry timing events: an event pair holds back the next
    # kernel's start by a few microseconds, so every other kind is timed on
    # a separate solve below
    op.profile_enable(True)
    op.profile_kinds(L.DOT_PROF_PCG2_FP32, L.DOT_PROF_JACOBIAN)
    t0 = time.perf_counter()
    state["marks"] = []
    starts = []
    for _ in range(args.steps):
        starts.append(time.perf_counter())
        step(th_ref)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # host time of each step's phases: the solve (it returns once every
    # column has converged), misfit, Jacobian and gradient (launches only),
    # thin SVD and Gauss-Newton step, the wait for the design
    step_phases = [[round((b - a) * 1e3, 2) for a, b in zip([s0] + m[:-1], m)]
                   for s0, m in zip(starts, state["marks"])]
    log(f"[bench] step phases (solve; misfit, Jacobian, gradient; thin SVD and "
        f"Gauss-Newton step; design wait) ms: {step_phases}")
    ms2, n2, cols2 = op.profile_read(L.DOT_PROF_PCG2_FP32)
    msj, nj, _ = op.profile_read(L.DOT_PROF_JACOBIAN)
    op.profile_enable(False)
    # error of the step's split-bf16 J_s against binary64 on the same fields
    J64 = op.jacobian(x[:, :ls], x[:, ls:], L.DOT_JAC_FP64)
    jac_err = float(torch.linalg.norm(state["Js"] - J64) / torch.linalg.norm(J64))
    res = state["res"]
    value = k * args.steps / elapsed
    solve_ms = None
    log(f"[bench] step: {elapsed / args.steps * 1e3:.1f} ms, {value:.2f} RHS/s, "
        f"iters={res.iters_max}, updates={res.outer}, relres_max={res.relres.max():.2e}")

    bytes2 = cols2 * N * PASS_BYTES["pcg2_fp32"]
    achieved2 = bytes2 / (ms2 * 1e-3) / 1e9 if ms2 > 0 else 0.0

    # solve-only timing of the mixed form (same 40 RHS) for the comparison,
    # without timing events
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nrep = max(1, args.steps // 2)
    for _ in range(nrep):
        step(th_ref, precision=L.DOT_MIXED, full_path=False)
    torch.cuda.synchronize()
    solve_ms = (time.perf_counter() - t1) / nrep * 1e3

    # one more mixed solve of the same right-hand sides with every solver
    # kind timed: CG pass 1, the V-cycles and the binary64 residual sweeps
    op.profile_enable(True)
    step(th_ref, precision=L.DOT_MIXED, full_path=False)
    ms2s, n2s, cols2s = op.profile_read(L.DOT_PROF_PCG2_FP32)
    ms1, n1, cols1 = op.profile_read(L.DOT_PROF_PCG1_FP32)
    msv, nv, colsv = op.profile_read(L.DOT_PROF_VCYCLE_FP32)
    msr, nr, colsr = op.profile_read(L.DOT_PROF_RESID)
    op.profile_enable(False)
    bytes1 = cols1 * N * PASS_BYTES["pcg1_fp32"]
    achieved1 = bytes1 / (ms1 * 1e-3) / 1e9 if ms1 > 0 else 0.0
    # the whole solve's HBM-bound kernels: both CG passes, the V-cycles and
    # the binary64 residual replacements, algorithmic bytes over summed time
    vbytes = colsv * op.multigrid_cycle_bytes(L.DOT_MIXED)
    rbytes = colsr * N * PASS_BYTES["resid"]
    solve_bytes = bytes1 + cols2s * N * PASS_BYTES["pcg2_fp32"] + vbytes + rbytes
    solve_kms = ms1 + ms2s + msv + msr
    solve_kernels = {
        "bytes": solve_bytes, "ms": round(solve_kms, 3),
        "achieved_gbs": round(solve_bytes / (solve_kms * 1e-3) / 1e9, 1) if solve_kms > 0 else None,
        "frac": round(solve_bytes / (solve_kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if solve_kms > 0 else None,
        "vcycle_bytes_per_column": op.multigrid_cycle_bytes(L.DOT_MIXED),
        "vcycle_gbs": round(vbytes / (msv * 1e-3) / 1e9, 1) if msv > 0 else None,
        "resid_gbs": round(rbytes / (msr * 1e-3) / 1e9, 1) if msr > 0 else None,
        "what": "CG pass 1 (12 B/cell/col) + pass 2 (20) + V-cycles (vector streams of every "
                "level kernel) + binary64 residual replacements (28), binary32 vectors; summed "
                "HIP-event time of those launches in one timed mixed solve of the step's "
                "right-hand sides after the timed steps",
    }

    # ------------------------------------------- Jacobi-preconditioned leg
    # the same mixed solve with the Jacobi scaling alone (the preconditioner
    # the oracle's CG uses), for the multigrid comparison and the CPU baseline
    jacobi, rj = None, None
    if not args.no_jacobi_leg:
        step(th_ref, precision=L.DOT_MIXED, full_path=False, precond=L.DOT_PRECOND_JACOBI)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step(th_ref, precision=L.DOT_MIXED, full_path=False, precond=L.DOT_PRECOND_JACOBI)
        torch.cuda.synchronize()
        ejac = time.perf_counter() - t1
        rj = state["res"]
        jacobi = {"ms_per_solve": round(ejac * 1e3, 2), "rhs_per_s": round(k / ejac, 3),
                  "iters": int(rj.iters_max), "updates": int(rj.outer),
                  "relres_max": float(rj.relres.max())}
        log(f"[bench] Jacobi-preconditioned mixed solve: {ejac * 1e3:.1f} ms, iters={rj.iters_max}")

    # ---------------------------------------------------------- FP64 leg
    fp64 = None
    if not args.no_fp64_leg:
        wk64 = torch.empty(op.solve_workspace_bytes(k, L.DOT_FP64) + 256, dtype=torch.uint8,
                           device=dev)
        work_saved = work
        work = wk64[(-wk64.data_ptr()) % 256:]
        step(th_ref, precision=L.DOT_FP64, full_path=False)
        torch.cuda.synchronize()
        op.profile_enable(True)
        op.profile_kinds(L.DOT_PROF_PCG2_FP64)
        t1 = time.perf_counter()
        for _ in range(nrep):
            step(th_ref, precision=L.DOT_FP64, full_path=False)
        torch.cuda.synchronize()
        e64 = (time.perf_counter() - t1) / nrep
        m64, n64, c64 = op.profile_read(L.DOT_PROF_PCG2_FP64)
        op.profile_enable(False)
        r64 = state["res"]
        fp64 = {"rhs_per_s": round(k / e64, 3), "ms_per_solve": round(e64 * 1e3, 2),
                "iters": int(r64.iters_max), "relres_max": float(r64.relres.max()),
                "pcg2_fp64_achieved_gbs": round(c64 * N * PASS_BYTES["pcg2_fp64"] / (m64 * 1e-3) / 1e9, 1)
                if m64 > 0 else None}
        work = work_saved
        log(f"[bench] fp64 solve: {e64 * 1e3:.1f} ms, {k / e64:.2f} RHS/s, iters={r64.iters_max}")
        del wk64

    # ---------------------------------------------------------- Jacobian leg
    jac = None
    if not args.no_jacobian_leg:
        jac = jacobian_leg(dl, L, torch, dev)
        log(f"[bench] jacobian leg: {jac}")

    # ------------------------------------------------ frequency-domain leg
    frequency = None
    if not args.no_frequency_leg:
        frequency = frequency_leg(dl, L, torch, dev, op, cfg, wl, W, V)
        log(f"[bench] frequency leg: {frequency}")

    # ------------------------------------------------------- diffusion leg
    diffusion = None
    if not args.no_diffusion_leg:
        diffusion = diffusion_leg(dl, L, torch, dev, op, cfg, wl, pals, W, V)
        log(f"[bench] diffusion leg: {diffusion}")

    # ---------------------------------------------------------- inversion leg
    inversion = None
    if not args.no_inversion_leg:
        inversion = inversion_leg(dl, L, torch, dev)
        log(f"[bench] inversion leg: {inversion}")

    # ---------------------------------------------------------- CPU baseline
    cpu = None
    if cpu_proc is not None:
        log("[bench] waiting for the CPU baseline")
        outs, _ = cpu_proc.communicate(timeout=900)
        if cpu_proc.returncode != 0:
            raise RuntimeError(f"CPU baseline failed with code {cpu_proc.returncode}")
        cpu = json.loads(outs.strip().splitlines()[-1])
        log(f"[bench] cpu baseline: {cpu}")

    traffic = measured_traffic(cfg.name)
    out = {
        "metric": "RHS solves/sec at rel-res 1e-8 (128^3) + Jacobian TFLOP/s, mixed vs FP64",
        "value": round(value, 3),
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "step_phases_ms": step_phases,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: 3D DOT {cfg.n[0]}x{cfg.n[1]}x{cfg.n[2]} ({N} cells), "
                        f"{cfg.n_s} sources / {cfg.n_d} detectors, {ls}+{ld} simultaneous RHS "
                        f"({cfg.q_s} optimized + {ls - cfg.q_s} complementary random each), "
                        f"{cfg.m0} RBFs ({cfg.n_p} params), binary32 CG in binary64 refinement "
                        "to relres 1e-8; step = PaLS, RHS, solves, misfit, 3-part split-bf16 Jacobian, "
                        "gradient, Alg. 1 design, thin SVD and truncated-SVD Gauss-Newton step",
            "grid": list(cfg.n), "rhs_per_step": k, "rtol": 1e-8, "n_params": cfg.n_p,
        },
        "roofline": {
            "kernel": "sweep_kernel<PCG2, float> (CG pass 2, binary32)",
            "bound": "hbm",
            "achieved": round(achieved2, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved2 / HBM_PEAK_GBS, 4),
            "traffic": (traffic["pcg2_fp32_bytes_per_launch"] if traffic else None),
            "traffic_unit": "B per launch (FETCH_SIZE x 1.99983 + WRITE_SIZE)",
            "bytes_per_cell_column": PASS_BYTES["pcg2_fp32"],
            "algorithmic_bytes_per_launch": round(bytes2 / max(n2, 1)),
            "avg_launch_us": round(ms2 / max(n2, 1) * 1e3, 2),
            "launches": n2,
            "pass1_achieved_gbs": round(achieved1, 1),
            "pass1_avg_launch_us": round(ms1 / max(n1, 1) * 1e3, 2),
            "solve_kernels": solve_kernels,
        },
        "mixed": {"iters": int(res.iters_max), "updates": int(res.outer),
                  "relres_max": float(res.relres.max()), "ms_per_solve": round(solve_ms, 2),
                  "rhs_per_s_solve_only": round(k / (solve_ms * 1e-3), 3),
                  "preconditioner": f"multigrid V-cycle, {op.multigrid_levels} levels",
                  "vcycle_avg_us": round(msv / max(nv, 1) * 1e3, 1), "vcycles": nv},
        "jacobi_mixed": jacobi,
        "speedup_multigrid_vs_jacobi_solve": (round(jacobi["ms_per_solve"] / solve_ms, 3)
                                              if jacobi else None),
        "fp64": fp64,
        "speedup_mixed_vs_fp64_solve": (round(fp64["ms_per_solve"] / solve_ms, 3)
                                        if fp64 else None),
        "step_jacobian_ms": round(msj / max(nj, 1), 3),
        "step_jacobian_rel_err_vs_fp64": jac_err,
        "jacobian": jac,
        "frequency": frequency,
        "diffusion": diffusion,
        "inversion": inversion,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    op.close()


def jacobian_leg(dl, L, torch, dev):
    """1600 x 5000 sampled Jacobian on 128^3 with 1000 RBFs: the 3-part
    split-bf16 product form, the 2-part option and binary64; algorithmic
    TFLOP/s = 2 l_s l_d n_act (band pairs) / time, algorithmic HBM bytes =
    the fields at the band cells read once plus J_s written; error against
    binary64 on the same fields."""
    import synthetic

    cfg = synthetic.get_config("C5")
    wl = synthetic.make_workload(cfg)
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    th = torch.tensor(wl.theta_ref, device=dev)
    _, D = dl.pals_field(grid, pals, th, cfg.mus_prime)
    op = dl.Operator(grid, D)
    op.pals_mua(pals, th)
    W = torch.tensor(wl.w_signs / np.sqrt(cfg.l_s), device=dev)
    V = torch.tensor(wl.v_signs / np.sqrt(cfg.l_d), device=dev)
    # binary64 solves, so every binary32 CG pass of the run belongs to the
    # timed 128^3, 64-RBF workload
    U, Z = setup_fields(dl, L, torch, dev, cfg, wl, op, pals, W, V, L.DOT_FP64, 1e-8)
    pairs, nband = op.n_pairs, op.n_band_cells
    na = pals.n_act(grid.dim)
    flops = 2.0 * cfg.l_s * cfg.l_d * na * pairs
    hbm = 8.0 * nband * (cfg.l_s + cfg.l_d) + 8.0 * cfg.l_s * cfg.l_d * cfg.n_p
    out = {"workload": f"C5: 128^3, {cfg.m0} RBFs, {cfg.l_s}x{cfg.l_d} sampled rows, "
                       f"{cfg.n_p} params", "band_pairs": pairs, "band_cells": nband,
           "algorithmic_gflop": flops / 1e9, "algorithmic_hbm_bytes": hbm,
           "intensity_flop_per_byte": round(flops / hbm, 1)}
    Js = {}
    for prec, name in ((L.DOT_JAC_SPLIT_BF16X3, "split_bf16x3"), (L.DOT_JAC_SPLIT_BF16, "split_bf16"),
                       (L.DOT_JAC_FP64, "fp64")):
        Js[name] = op.jacobian(U, Z, prec)
        torch.cuda.synchronize()
        op.profile_enable(True)
        for _ in range(5):
            Js[name] = op.jacobian(U, Z, prec)
        ms, n, _ = op.profile_read(L.DOT_PROF_JACOBIAN)
        op.profile_enable(False)
        t = ms / n * 1e-3
        out[name] = {"ms": round(ms / n, 3), "tflops_algorithmic": round(flops / t / 1e12, 3),
                     "hbm_gbs_algorithmic": round(hbm / t / 1e9, 1),
                     "hbm_frac_algorithmic": round(hbm / t / 1e9 / HBM_PEAK_GBS, 4)}
    ref = Js["fp64"]
    for name in ("split_bf16x3", "split_bf16"):
        out[name]["rel_err_vs_fp64"] = float(torch.linalg.norm(Js[name] - ref) / torch.linalg.norm(ref))
        out[name]["frac_of_bf16_peak_algorithmic"] = round(
            out[name]["tflops_algorithmic"] / BF16_PEAK_TFLOPS, 5)
    out["split_bf16x3"]["role"] = "product form (error bound 1e-6)"
    out["split_bf16"]["role"] = "option (error bound 2e-5)"
    out["fp64"]["frac_of_fp64_peak"] = round(out["fp64"]["tflops_algorithmic"] / FP64_PEAK_TFLOPS, 4)
    # thin SVD of the 1600 x 5000 sampled Jacobian (Gauss-Newton model)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s, _, _ = dl.svd_thin(Js["split_bf16x3"], rcut=1e-10)
    torch.cuda.synchronize()
    out["svd_1600x5000_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    op.close()
    return out


# modulation frequency of the frequency-domain leg: kappa = omega / nu with
# omega = 2 pi 100 MHz and nu = c / 1.4 in tissue, in the unit box's length unit
# (1 mm for the 128^3 workload): kappa / mu_out is about 0.3, as in a 60 mm slab
KAPPA_100MHZ_PER_MM = 2.0 * np.pi * 100e6 / (3.0e11 / 1.4)


def frequency_leg(dl, L, torch, dev, op, cfg, wl, W, V, reps=3):
    """The step's 40 right-hand sides solved at 100 MHz modulation:
    (A + i kappa h^d I) X = [B W, C V] by binary64 COCG with the multigrid
    V-cycle on both parts (relres 1e-8), the V-cycle in binary64 or in
    binary32 with bfloat16 vectors.  Algorithmic bytes per cell, complex
    column and iteration: apply 32 (read p, write q), update 96 (read p, q,
    x, r; write x, r), r^T z 32, direction 48, plus the V-cycle on both
    parts; with the binary32 V-cycle the update also writes r / ||b|| in
    binary32 (+8) and r^T z and the direction read z in binary32 (-8 each)."""
    ls, ld = cfg.l_s, cfg.l_d
    k = ls + ld
    N = op.N
    rhs = torch.zeros((N, k), dtype=torch.complex128, device=dev)
    rhs[:, :ls] = op.form_rhs(wl.src_cells, W)
    rhs[:, ls:] = op.form_rhs(wl.det_cells, V)
    kappa = KAPPA_100MHZ_PER_MM
    out = {"kappa": kappa, "columns_complex": k,
           "preconditioner": f"multigrid V-cycle on real and imaginary parts, "
                             f"{op.multigrid_levels} levels"}
    for name, prec, per in (
            ("fp64_vcycle", L.DOT_FP64,
             32 + 96 + 32 + 48 + 2 * op.multigrid_cycle_bytes(L.DOT_FP64) / N),
            ("mixed_vcycle", L.DOT_MIXED,
             32 + 104 + 24 + 40 + 2 * op.multigrid_cycle_bytes(L.DOT_MIXED) / N)):
        res = op.solve_complex(rhs, kappa, rtol=1e-8, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = op.solve_complex(rhs, kappa, rtol=1e-8, precision=prec)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        it = int(res.iters_max)
        gbs = per * N * k * it / t / 1e9
        out[name] = {"ms_per_solve": round(t * 1e3, 2), "rhs_per_s": round(k / t, 2),
                     "iters": it, "relres_max": float(res.relres.max()),
                     "bytes_per_cell_column_iteration": round(per, 1),
                     "achieved_gbs_algorithmic": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def diffusion_leg(dl, L, torch, dev, op, cfg, wl, pals, W, V):
    """The sampled Jacobian with the diffusion inverted as well (face terms of
    dA/dp) on the step's fields: scattering contrast 2x inside the anomaly;
    binary64 and 3-part split-bf16, error of the latter against the former;
    algorithmic flop = 2 l_s l_d n_act (pairs x 7 rows)."""
    ls, ld = cfg.l_s, cfg.l_d
    th = torch.tensor(wl.theta_ref, device=dev)
    op.pals_mua_diffusion(pals, th, 2.0 * cfg.mus_prime, cfg.mus_prime)
    rhs = dl.empty_colmajor(op.N, ls + ld, dev)
    op.form_rhs(wl.src_cells, W, out=rhs[:, :ls])
    op.form_rhs(wl.det_cells, V, out=rhs[:, ls:])
    res = op.solve(rhs, rtol=1e-8, precision=L.DOT_MIXED, inner_rtol=0.01, check_every=2)
    U, Z = res.x[:, :ls], res.x[:, ls:]
    na = pals.n_act(op.grid.dim)
    rows = 1 + 2 * op.grid.dim
    flops = 2.0 * ls * ld * na * op.n_pairs * rows
    out = {"scattering_in_over_out": 2.0, "solve_iters": int(res.iters_max),
           "rows_per_pair": rows, "pairs": op.n_pairs, "algorithmic_gflop": flops / 1e9}
    Js = {}
    for prec, name in ((L.DOT_JAC_FP64, "fp64"), (L.DOT_JAC_SPLIT_BF16X3, "split_bf16x3")):
        Js[name] = op.jacobian(U, Z, prec)
        torch.cuda.synchronize()
        op.profile_enable(True)
        for _ in range(3):
            Js[name] = op.jacobian(U, Z, prec)
        ms, n, _ = op.profile_read(L.DOT_PROF_JACOBIAN)
        op.profile_enable(False)
        out[name] = {"ms": round(ms / n, 3), "tflops_algorithmic": round(flops / (ms / n * 1e-3) / 1e12, 2)}
    out["split_bf16x3"]["rel_err_vs_fp64"] = float(
        torch.linalg.norm(Js["split_bf16x3"] - Js["fp64"]) / torch.linalg.norm(Js["fp64"]))
    op.pals_mua(pals, th)
    return out


# Table T3 of the paper (Example 2: 32^3, 225 sources / 225 detectors, 27
# RBFs, 135 parameters, l = 12): iterations / function / Jacobian evaluations
# and total large solves, MATLAB, hardware not stated.
PAPER_T3 = {"all_sources_detectors": {"it": 25, "fe": 26, "je": 15, "solves": 9225},
            "saa_to_intermediate_tol": {"it": 4, "fe": 5, "je": 6, "solves": 132},
            "saa_plus_2_optimized": {"it": 12, "fe": 13, "je": 6, "solves": 726},
            "saa_plus_4_optimized": {"it": 9, "fe": 10, "je": 3, "solves": 762}}


def inversion_leg(dl, L, torch, dev, max_iter=30):
    """The outer driver on Example 2's shape (32^3 slab of 60 mm, 225 sources on
    top, 225 detectors at the bottom, 27 RBFs x 5 parameters, l = 12, 2
    optimized sources and detectors after the SAA phase, 0.1% noise): SAA
    Gauss-Newton to the intermediate tolerance, the full Jacobian (450
    solves) with Alg. 1 and the complement, then Gauss-Newton towards the
    final tolerance; counts beside table T3 and the wall time.  The data come
    from the library's own binary64 solves at the true parameters; the true
    misfit of each phase's end point is a check on the side (not counted)."""
    import synthetic

    cfg = synthetic.get_config("inv_x2")
    wl = synthetic.make_workload(cfg)
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    T = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), device=dev)  # noqa: E731
    _, D = dl.pals_field(grid, pals, T(wl.theta_ref), cfg.mus_prime)
    op = dl.Operator(grid, D)
    eye_s = torch.eye(cfg.n_s, dtype=torch.float64, device=dev)

    def measurements(theta):
        op.pals_mua(pals, theta)
        B = op.form_rhs(wl.src_cells, eye_s)
        return op.solve(B, rtol=1e-12).x[wl.det_cells.astype(np.int64), :]

    M_true = measurements(T(wl.theta_true))
    data = M_true * (1.0 + cfg.noise * T(wl.xi))
    dn2 = float(torch.sum(data * data).item())
    inv = dl.inversion
    sd = inv.SampledDOT(op, pals, T(wl.theta_ref), wl.src_cells, wl.det_cells, data,
                        rtol=cfg.rtol)
    p0 = sd.params_of(T(wl.theta_ref))
    opts = inv.TrustRegionOptions(radius0=0.5, max_iter=max_iter)

    def true_rel(p):
        R = measurements(sd.theta_of(p)) - data
        return float(torch.sum(R * R).item()) / dn2

    k_sk, sweeps = 8, 2
    draws = synthetic.sketch_draws(cfg.n_s, cfg.n_d, cfg.n_p, cfg.q_s, cfg.q_d, k_sk, sweeps, 1)
    draws = {key: ([T(x) for x in v] if isinstance(v, list) else T(v)) for key, v in draws.items()}
    runs = {}
    for design, sketch in (("full_jacobian", None), ("sketched", draws)):
        sd.solves = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = inv.invert(sd, p0, T(wl.w_signs / np.sqrt(cfg.l_s)),
                         T(wl.v_signs / np.sqrt(cfg.l_d)), cfg.q_s, cfg.q_d, T(wl.y_signs),
                         T(wl.z_signs), cfg.noise, opts, sketch=sketch)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phases = {}
        for name in ("saa", "opt"):
            ph = out.get(name)
            if ph is None:
                continue
            phases[name] = {"it": ph.it, "fe": ph.fe, "je": ph.je, "converged": ph.converged,
                            "sampled_rel_misfit": 2.0 * ph.f / dn2,
                            "true_rel_misfit": true_rel(ph.p)}
        n_up = cfg.n_s + cfg.n_d if sketch is None else inv.sketch_solves(k_sk, sweeps)
        runs[design] = {"phases": phases, "update_solves": n_up, "solves": out["solves"],
                        "solves_counted": out["counted"], "wall_s": round(wall, 3)}
        log(f"[bench] inversion ({design}): {runs[design]}")
    res = {"workload": f"inv_x2: 32^3, {cfg.n_s} sources / {cfg.n_d} detectors, {cfg.m0} RBFs "
                       f"({cfg.n_p} params), l = {cfg.l_s}, {cfg.q_s} optimized after SAA, "
                       f"delta = {cfg.noise}, binary64 solves to relres {cfg.rtol}",
           "tolerances_rel_misfit": {"intermediate": cfg.noise, "final": cfg.noise ** 2},
           "start_true_rel_misfit": true_rel(p0), "max_trial_steps_per_phase": max_iter,
           "sketch": {"test_vectors": k_sk, "sweeps": sweeps}, "runs": runs,
           "paper_T3": PAPER_T3}
    op.close()
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, repeats):
    """The oracle's Jacobi-PCG (scipy CSR SpMV, numpy vector updates) solving
    one right-hand side of the same workload to relative residual 1e-8,
    timed end to end, median of `repeats` runs.  BLAS is held to one thread
    (the CSR product is single-threaded anyway), so the baseline runs on one
    core; the host's core count and model are recorded beside it."""
    from threadpoolctl import threadpool_limits

    from oracle import estimators as oest
    from oracle import problem as oprob
    from oracle import solvers as osol

    t0 = time.perf_counter()
    prob = oprob.build(wl)
    A = prob.operator(wl.theta_ref)
    W = oest.sample_matrix(wl.w_signs)
    b = oest.simultaneous_rhs(prob.N, wl.src_cells, W[:, :1])[:, 0]
    t_setup = time.perf_counter() - t0
    times, iters, rels = [], [], []
    with threadpool_limits(limits=1):
        for _ in range(repeats):
            t1 = time.perf_counter()
            _, it, rel = osol.pcg_jacobi(A, b, rtol=1e-8, maxiter=5000)
            times.append(time.perf_counter() - t1)
            iters.append(it)
            rels.append(rel)
    per_rhs = float(np.median(times))
    return {"value": round(1.0 / per_rhs, 5), "unit": "RHS/s", "cores": 1, "kind": "oracle",
            "host_cpus": os.cpu_count(), "host_cpu_model": _cpu_model(),
            "seconds_per_solve": [round(t, 3) for t in times], "iters": iters[0],
            "relres": float(rels[0]),
            "sample": f"oracle Jacobi-PCG (scipy CSR SpMV, one thread) solving 1 of the 40 "
                      f"RHS of the 128^3 workload to relres 1e-8 ({iters[0]} iterations), "
                      f"median of {repeats} runs; oracle assembly ({t_setup:.1f} s) not timed"}


if __name__ == "__main__":
    main()
