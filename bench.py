"""Benchmark: Sternheimer solves/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload si16] [--no-cpu-baseline]

One step is one ``sternheimer_solve`` call over the whole workload: for the
si16 crystal (16-atom diamond fcc 2x2x2 supercell, 4015 plane waves, 48^3
grid) every one of 32 occupied bands x 50 plane-wave perturbations at one
seeded q x 64 frequencies in [0, 40] eV with eta = 0.05 eV, tol 1e-8 on the
true FP64 relative residual: 102,400 solves.  Inputs are resident in HBM
before the timed region; a solve counts when its true residual meets tol.

The JSON line carries the roofline of the dominant kernel (timed with HIP
events on the library's stream during the timed steps) and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)

WORKLOADS = {
    "si16": "si16: diamond fcc 2x2x2 (16 atoms), 4015 PW, 48^3 grid, 32 bands x 50 perts x 64 omega in [0,40] eV, "
            "eta 0.05 eV, tol 1e-8",
    "si2": "si2: diamond fcc primitive (2 atoms), 307 PW, 16^3 grid, 4 bands x 4 perts x 8 omega in [0,20] eV, "
           "eta 0.1 eV, tol 1e-10",
}

KERNELS = ["hx_sticks_inv", "hx_planes", "hx_sticks_fwd", "proj_dot", "proj_apply", "lanczos_step", "slot_init", "rhs_source",
           "tridiag", "combine", "residual", "permute"]


def fft_flops(n):
    return 5.0 * n * np.log2(n)


def kernel_model(problem, name):
    """Algorithmic flops per vector of the H.x kernels (5 N log2 N per complex N-point FFT)."""
    n0, n1, n2 = problem.grid
    m = problem.miller_kq
    n_row = int(m[:, 0].max() - m[:, 0].min() + 1)
    n_stick = len({(a, b) for a, b in m[:, :2]})
    if name == "hx_planes":
        per_plane = 2 * (n_row * fft_flops(n1) + n1 * fft_flops(n0)) + 2.0 * n0 * n1
        return per_plane * n2
    if name in ("hx_sticks_inv", "hx_sticks_fwd"):
        return n_stick * fft_flops(n2)
    return 0.0


def cpu_baseline(problem, n_pairs_sample, log):
    """Time the oracle (dense H_{k+q}, full eigendecomposition, spectral sums) on a sample of pairs."""
    import oracle
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 0) for i in info] + [0]) or os.cpu_count()
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    p = problem
    t0 = time.perf_counter()
    setup = oracle.spectral_setup(p.miller_kq, p.B, p.kvec + p.qvec, p.v_grid)
    t_setup = time.perf_counter() - t0
    log(f"cpu oracle: H_kq + eigh {t_setup:.1f} s")
    rng = np.random.default_rng(12345)
    all_pairs = [(v, q) for v in range(p.n_band) for q in range(p.n_pert)]
    idx = rng.choice(len(all_pairs), size=min(n_pairs_sample, len(all_pairs)), replace=False)
    pairs = [all_pairs[i] for i in idx]
    t0 = time.perf_counter()
    oracle.solve_pairs(setup, p.n_occ, p.psi_k, p.eps_k, p.miller_k, p.miller_kq, p.dv_miller, p.psi_kq, p.omega,
                       p.eta, pairs)
    t_pairs = time.perf_counter() - t0
    n_total_pairs = len(all_pairs)
    t_full = t_setup + t_pairs / len(pairs) * n_total_pairs
    value = n_total_pairs * p.n_omega / t_full
    return {"value": value, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": f"dense H_k+q + full eigh once ({t_setup:.1f} s) + spectral solves for {len(pairs)} of "
                      f"{n_total_pairs} (band, pert) pairs x {p.n_omega} omega ({t_pairs:.1f} s); value = "
                      f"all {n_total_pairs * p.n_omega} solves / (setup + per-pair time x {n_total_pairs})"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="si16", choices=sorted(WORKLOADS))
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-pairs", type=int, default=8)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n, "copies": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the (band, perturbation) pairs would be sharded across GPUs; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    import torch
    import synth
    from paper_1812_03717_amd import sgw
    from paper_1812_03717_amd.workload import DeviceProblem

    if not torch.cuda.is_available():
        log("no GPU available")
        sys.exit(1)
    sgw.load_library()
    t0 = time.perf_counter()
    problem = getattr(synth, args.workload)()
    log(f"generated {args.workload}: {problem.n_pw_kq} PW, grid {problem.grid}, {problem.n_solves} solves "
        f"({time.perf_counter() - t0:.1f} s)")
    ctx = sgw.sgw_ctx_create(0)
    dev = DeviceProblem(ctx, problem)
    ws = sgw.Workspace(ctx)
    opts = sgw.sgw_opts_default(slots=args.slots) if args.slots else sgw.sgw_opts_default()
    dpsi = torch.empty((problem.n_band, problem.n_pert, problem.n_omega, problem.n_pw_kq), dtype=torch.complex128,
                       device=ctx.device)
    info = torch.empty(problem.n_solves * sgw.INFO_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)

    # warmup (also identifies the dominant kernel)
    ctx.set_profiling("all")
    for w in range(max(args.warmup, 1)):
        t = time.perf_counter()
        st, _, _ = dev.solve(opts=opts, workspace=ws, dpsi=dpsi, info=info)
        torch.cuda.synchronize()
        log(f"warmup {w}: status {st}, {time.perf_counter() - t:.3f} s")
    stats = {k: ctx.kernel_stats(k) for k in KERNELS}
    total = sum(s["ms"] for s in stats.values())
    for k, s in sorted(stats.items(), key=lambda kv: -kv[1]["ms"]):
        if s["launches"]:
            log(f"  {k:14s} {s['ms']:9.2f} ms  {100 * s['ms'] / total:5.1f}%  launches {s['launches']}")
    dominant = max(stats, key=lambda k: stats[k]["ms"])

    # timed steps: events only around the dominant kernel
    ctx.reset_stats()
    ctx.set_profiling(dominant)
    inf = None
    n_ok = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, _, _ = dev.solve(opts=opts, workspace=ws, dpsi=dpsi, info=info)
        inf = sgw.info_to_numpy(info)
        n_ok += int(np.count_nonzero((inf["flags"] & sgw.FLAG_CONVERGED) != 0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_profiling(None)
    ks = ctx.kernel_stats(dominant)
    log(f"timed {args.steps} steps: {elapsed:.3f} s; converged {n_ok}/{problem.n_solves * args.steps}; "
        f"iters min/mean/max {inf['iters'].min()}/{inf['iters'].mean():.1f}/{inf['iters'].max()}; "
        f"max relres {inf['relres'].max():.3e}")

    avg_ms = ks["ms"] / max(ks["launches"], 1)
    bytes_per_launch = ks["bytes"] / max(ks["launches"], 1)
    gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    # vectors per launch from the charged bytes: flops model per vector x vectors
    roof = {"kernel": dominant, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "avg_launch_ms": round(avg_ms, 4),
            "launches": ks["launches"], "alg_bytes_per_launch": bytes_per_launch}
    fl = kernel_model(problem, dominant)
    if fl:
        n0, n1, n2 = problem.grid
        n_stick = len({(a, b) for a, b in problem.miller_kq[:, :2]})
        per_vec_bytes = n2 * n_stick * 32.0 if dominant == "hx_planes" else None
        if per_vec_bytes:
            vecs = (bytes_per_launch - n0 * n1 * n2 * 8.0) / per_vec_bytes
            tf = fl * vecs / (avg_ms * 1e-3) / 1e12
            roof["alu_achieved_tflops"] = round(tf, 2)
            roof["alu_peak_tflops"] = FP64_VECTOR_TFLOPS
            roof["alu_frac"] = round(tf / FP64_VECTOR_TFLOPS, 4)
    value = n_ok / elapsed
    out = {
        "metric": "Sternheimer solves/s (band x omega x pert) at true FP64 rel. residual <= tol",
        "value": round(value, 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "speedup_vs_plain_fp64": 1.0, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "solves_per_step": problem.n_solves,
                   "method": "plain FP64 multishift Lanczos-FOM, stored basis"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problem, args.cpu_sample_pairs, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
