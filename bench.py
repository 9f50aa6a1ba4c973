"""Benchmark of one step of the randomized DOT hot path on one MI355X.

Workload (the 128^3 configuration): 3D diffusion on 128^3 cells (2,097,152
unknowns), Robin top/bottom and Dirichlet lateral faces, 256 sources on the
top face and 256 detectors on the bottom face, l_s = l_d = 20 simultaneous
sources/detectors, PaLS absorption with 64 RBFs (320 parameters).  A step is
one pass of the whole hot path over that batch:
  PaLS absorption and A(theta) -> right-hand sides B W and C V -> the 40
  forward + adjoint solves to a per-column relative residual of 1e-8
  (binary32 CG inside binary64 refinement) -> sampled misfit -> sampled
  Jacobian (400 x 320) -> adjoint gradient.
The metric is right-hand sides solved per second over whole steps.  A second
leg times the same 40 solves in plain binary64 CG at the same 1e-8.

Printed: one JSON line (see keys below); progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell per column for each CG pass (vector streams only)
PASS_BYTES = {
    "pcg1_fp32": 12,   # read r, p_old; write p      (binary32)
    "pcg2_fp32": 20,   # read p, d, r; write d, r    (binary32)
    "pcg1_fp64": 24,
    "pcg2_fp64": 40,
}


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
    ap.add_argument("--cpu-iters", type=int, default=120)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path is built and measured on a single "
              "MI355X (the multi-GPU sharding is described in DESIGN.md, not run); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

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
    W = torch.tensor(wl.w_signs / np.sqrt(ls), device=dev)
    V = torch.tensor(wl.v_signs / np.sqrt(ld), device=dev)
    # synthetic data: all sources at theta_true, 0.1% relative noise
    op.pals_mua(pals, th_true)
    B = op.form_rhs(wl.src_cells, torch.eye(cfg.n_s, dtype=torch.float64, device=dev))
    # binary64 solves here, so the binary32 pass kernels run only in the timed workload
    full = op.solve(B, rtol=1e-10, precision=L.DOT_FP64)
    M_true = full.x.cpu().numpy()[wl.det_cells, :]
    data = torch.tensor(M_true * (1.0 + cfg.noise * wl.xi), device=dev)
    DW = dl.gemm(data, W)
    del B, full
    log("[bench] setup done (data synthesized with 256 solves)")

    rhs = dl.empty_colmajor(N, k, dev)
    x = dl.empty_colmajor(N, k, dev)
    work = torch.empty(op.solve_workspace_bytes(k, L.DOT_MIXED) + 256, dtype=torch.uint8,
                       device=dev)
    work = work[(-work.data_ptr()) % 256:]
    state = {}

    def step(theta, precision=L.DOT_MIXED, full_path=True):
        if full_path:
            op.pals_mua(pals, theta)
            op.form_rhs(wl.src_cells, W, out=rhs[:, :ls])
            op.form_rhs(wl.det_cells, V, out=rhs[:, ls:])
        res = op.solve(rhs, rtol=1e-8, precision=precision, inner_rtol=0.1, out=x, work=work)
        if not res.converged:
            raise RuntimeError(f"solve did not converge: {res.relres.max():.3e}")
        state["res"] = res
        if full_path:
            U, Z = x[:, :ls], x[:, ls:]
            Rs, f = op.sampled_misfit(wl.det_cells, U, V, DW)
            Js = op.jacobian(U, Z, L.DOT_JAC_FP64)
            g = op.grad_misfit(U, Z, Rs)
            state.update(f=f, Js=Js, g=g)

    for _ in range(args.warmup):
        step(th_ref)
    torch.cuda.synchronize()
    op.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(th_ref)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms2, n2, cols2 = op.profile_read(L.DOT_PROF_PCG2_FP32)
    ms1, n1, cols1 = op.profile_read(L.DOT_PROF_PCG1_FP32)
    op.profile_enable(False)
    res = state["res"]
    value = k * args.steps / elapsed
    log(f"[bench] mixed: {elapsed / args.steps * 1e3:.1f} ms/step, {value:.2f} RHS/s, "
        f"iters={res.iters_max}, updates={res.outer}, relres_max={res.relres.max():.2e}")

    # dominant kernel: CG pass 2 in binary32
    bytes2 = cols2 * N * PASS_BYTES["pcg2_fp32"]
    achieved2 = bytes2 / (ms2 * 1e-3) / 1e9 if ms2 > 0 else 0.0
    bytes1 = cols1 * N * PASS_BYTES["pcg1_fp32"]
    achieved1 = bytes1 / (ms1 * 1e-3) / 1e9 if ms1 > 0 else 0.0

    # ---------------------------------------------------------- FP64 leg
    fp64 = None
    if not args.no_fp64_leg:
        wk64 = torch.empty(op.solve_workspace_bytes(k, L.DOT_FP64) + 256, dtype=torch.uint8,
                           device=dev)
        work_saved = work
        work = wk64[(-wk64.data_ptr()) % 256:]
        op.pals_mua(pals, th_ref)
        step(th_ref, precision=L.DOT_FP64, full_path=False)
        torch.cuda.synchronize()
        op.profile_enable(True)
        t1 = time.perf_counter()
        nrep = max(1, args.steps // 2)
        for _ in range(nrep):
            step(th_ref, precision=L.DOT_FP64, full_path=False)
        torch.cuda.synchronize()
        e64 = (time.perf_counter() - t1) / nrep
        m64, n64, c64 = op.profile_read(L.DOT_PROF_PCG2_FP64)
        op.profile_enable(False)
        r64 = state["res"]
        fp64 = {"rhs_per_s": k / e64, "ms_per_solve": e64 * 1e3, "iters": int(r64.iters_max),
                "relres_max": float(r64.relres.max()),
                "pcg2_achieved_gbs": (c64 * N * PASS_BYTES["pcg2_fp64"] / (m64 * 1e-3) / 1e9)
                if m64 > 0 else None}
        work = work_saved
        log(f"[bench] fp64 solve: {e64 * 1e3:.1f} ms, {k / e64:.2f} RHS/s, iters={r64.iters_max}")
        del wk64

    # ---------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_iters, res)
        log(f"[bench] cpu baseline: {cpu}")

    out = {
        "metric": "RHS solves/sec at rel-res 1e-8 (128^3) + Jacobian TFLOP/s, mixed vs FP64",
        "value": round(value, 3),
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: 3D DOT {cfg.n[0]}x{cfg.n[1]}x{cfg.n[2]} "
                        f"({N} cells), {cfg.n_s} sources / {cfg.n_d} detectors, "
                        f"{ls}+{ld} simultaneous RHS, {cfg.m0} RBFs ({cfg.n_p} params), "
                        "binary32 CG in binary64 refinement to relres 1e-8",
            "grid": list(cfg.n), "rhs_per_step": k, "rtol": 1e-8, "n_params": cfg.n_p,
        },
        "roofline": {
            "kernel": "sweep_kernel<PCG2, float> (CG pass 2, binary32)",
            "bound": "hbm",
            "achieved": round(achieved2, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved2 / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_cell_column": PASS_BYTES["pcg2_fp32"],
            "avg_launch_us": round(ms2 / max(n2, 1) * 1e3, 2),
            "launches": n2,
            "pass1_achieved_gbs": round(achieved1, 1),
        },
        "mixed": {"iters": int(res.iters_max), "updates": int(res.outer),
                  "relres_max": float(res.relres.max())},
        "fp64": fp64,
        "speedup_mixed_vs_fp64": (round(value / fp64["rhs_per_s"], 3) if fp64 else None),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    op.close()


def cpu_baseline(wl, iters, gpu_res):
    """The oracle's Jacobi-PCG (scipy CSR) on one right-hand side of the same
    workload, run for a bounded number of iterations and scaled to the
    iteration count a full solve to 1e-8 needs."""
    import scipy.sparse.linalg  # noqa: F401

    from oracle import estimators as oest
    from oracle import problem as oprob
    from oracle import solvers as osol

    t0 = time.perf_counter()
    prob = oprob.build(wl)
    A = prob.operator(wl.theta_ref)
    W = oest.sample_matrix(wl.w_signs)
    b = oest.simultaneous_rhs(prob.N, wl.src_cells, W[:, :1])[:, 0]
    t_setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    _, it, rel = osol.pcg_jacobi(A, b, rtol=1e-30, maxiter=iters)
    t_it = (time.perf_counter() - t1) / it
    need = int(gpu_res.iters_max)   # the GPU binary32 run's count (matches binary64 CG within a few %)
    per_rhs = t_it * need
    return {"value": round(1.0 / per_rhs, 5), "unit": "RHS/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle Jacobi-PCG (scipy CSR, one thread) on 1 RHS of the 128^3 workload: "
                      f"{it} iterations timed ({t_it * 1e3:.1f} ms each), scaled to {need} "
                      f"iterations; operator assembly {t_setup:.1f} s not included"}


if __name__ == "__main__":
    main()
