"""Benchmark: Sternheimer solves/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload si64] [--no-cpu-baseline]

One step is one ``sternheimer_solve`` call over the whole workload.  The default workload is the
largest single-GPU configuration, si64: the 64-atom diamond cell (conventional cubic 2x2x2,
16,013 plane waves at k+q, 72^3 grid), every one of 128 occupied bands x 20 plane-wave
perturbations at one seeded q x 100 frequencies in [0, 40] eV with eta = 0.05 eV, tol 1e-8 on the
true FP64 relative residual: 256,000 solves.  The default method is the block solver in FP64 (one
block Krylov space per band over its 20 perturbations, at most 160 block steps), with the plain FP64
multishift solver (max_iter 3500) timed beside it on the same systems.  Inputs are resident in HBM
before the timed region; a solve counts when its true residual meets tol.

The JSON line carries the roofline of the dominant kernel (timed with HIP events on the
library's stream during the timed steps) and the CPU oracle timed on a bounded sample of the
same workload: for si64 the oracle's direct route (dense H_{k+q}, the shifted operator of one
band, one LU factorisation solving all perturbations at one frequency), scaled to the workload.

    python bench.py --workload si16 --precision mixed   # 16-atom cell, 48^3, 102,400 solves;
                                                        # a plain FP64 leg is timed beside it
    python bench.py --workload batch200                 # 200 uneven systems, sternheimer_solve_batch
    python bench.py --workload batch200e11              # the same at Ecut 11.46 Ha (inputs: GPU eigensolver)
                                                        # (block solver; --batch-solver multishift)
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
FP64_MFMA_TFLOPS = 78.6        # MI355X dense FP64 matrix

WORKLOADS = {
    "si16": "si16: diamond fcc 2x2x2 (16 atoms), 4015 PW, 48^3 grid, 32 bands x 50 perts x 64 omega in [0,40] eV, "
            "eta 0.05 eV, tol 1e-8",
    "si2": "si2: diamond fcc primitive (2 atoms), 307 PW, 16^3 grid, 4 bands x 4 perts x 8 omega in [0,20] eV, "
           "eta 0.1 eV, tol 1e-10",
    "si64": "si64: diamond conventional 2x2x2 (64 atoms), 16013 PW, 72^3 grid, 128 bands x 20 perts x 100 omega in "
            "[0,40] eV, eta 0.05 eV, tol 1e-8",
    "si64nl": "si64nl: si64 with synthetic separable non-local s and p projectors on every atom (256, "
              "Gaussian radial forms), 16013 PW, 72^3 grid, 128 bands x 20 perts x 100 omega in [0,40] eV, "
              "eta 0.05 eV, tol 1e-8",
    "batch200": "batch200: 200 independent diamond fcc n0 x n1 x n2 cells (n_d in 1..3, 2-54 atoms), grid 24 n_d "
                "per axis, Ecut 4 Ha (100-2800 PW), all ~2*atoms occupied bands, 16-128 omega in [0,40] eV, "
                "4-16 perts at an own seeded q, eta 0.05 eV, tol 1e-8",
    "batch200e11": "batch200e11: the same 200 systems' recipe at Ecut 11.46 Ha (531-13539 PW; grids 24^3-72^3), all "
                   "~2*atoms occupied bands (4-109), 16-128 omega in [0,40] eV, 4-16 perts at an own seeded q, "
                   "eta 0.05 eV, tol 1e-8",
}

KERNELS = ["hx_sticks_inv", "hx_planes", "hx_sticks_fwd", "proj_dot", "proj_apply", "lanczos_step", "slot_init", "rhs_source",
           "tridiag", "combine", "residual", "permute", "nl_dot", "nl_apply", "blk_product"]


def roofline(kernel, ks, workload, default_launch=True):
    """Roofline entry of the dominant kernel from the library's event timing.

    The library charges every launch with its algorithmic bytes (HBM data the
    kernel must move) and flops (5 N log2 N per complex N-point FFT, 2 per
    potential multiply).  The FFT plane pass runs out of LDS and registers and
    is bound by FP64 arithmetic, so its entry is "alu" against the FP64 vector
    peak; HBM figures are given beside it.  ``traffic`` comes from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, only while the kernel's sources
    still hash to the value recorded with those counters and the launches have
    the size they had there (``default_launch``: no --slots override, and the
    algorithmic bytes per launch within 2% of those of the counted run).
    """
    from paper_1812_03717_amd import profiling
    n = max(ks["launches"], 1)
    avg_s = ks["ms"] / n * 1e-3
    bytes_per_launch = ks["bytes"] / n
    flops_per_launch = ks["flops"] / n
    gbs = bytes_per_launch / avg_s / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if default_launch and os.path.exists(tfile):
        with open(tfile) as fh:
            t = json.load(fh)
        same_launch = abs(t.get("alg_bytes_per_launch", 0) - bytes_per_launch) <= 0.02 * bytes_per_launch
        if t.get("source_hash") == profiling.source_hash(kernel) and same_launch:
            traffic = round(t["fetch_bytes_per_dispatch"] + t["write_bytes_per_dispatch"])
    roof = {"kernel": kernel, "traffic": traffic, "avg_launch_ms": round(avg_s * 1e3, 4), "launches": ks["launches"],
            "alg_bytes_per_launch": round(bytes_per_launch), "hbm_achieved_gbs": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    if kernel == "blk_product":  # complex FP64 products on the matrix cores (rocBLAS zgemm)
        tf = flops_per_launch / avg_s / 1e12
        roof.update({"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / FP64_MFMA_TFLOPS, 4), "alg_flops_per_launch": round(flops_per_launch)})
    elif flops_per_launch > 0:
        tf = flops_per_launch / avg_s / 1e12
        roof.update({"bound": "alu", "achieved": round(tf, 2), "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / FP64_VECTOR_TFLOPS, 4), "alg_flops_per_launch": round(flops_per_launch)})
    else:
        roof.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4)})
    return roof


def _cpu_info():
    """(threads the BLAS pool uses, CPU model string)."""
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 0) for i in info] + [0]) or os.cpu_count()
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    return int(cores), model


def cpu_baseline_lu(problem, log):
    """Time the oracle's direct route on a bounded sample: the dense H_{k+q}, the shifted operator of
    the top band, and one LU factorisation of (A0 - z) solving every perturbation's right-hand side at
    one frequency.  Every (band, frequency) needs its own factorisation, so the whole workload costs
    t_H + n_band t_op + n_band n_omega t_LU."""
    import oracle.sternheimer_oracle as so
    cores, model = _cpu_info()
    p = problem
    v, j = p.n_band - 1, 0
    t0 = time.perf_counter()
    nl = None if p.e_kb is None else (p.beta_kq, p.e_kb)
    h = so.hamiltonian(p.miller_kq, p.B, p.kvec + p.qvec, p.v_grid, nl=nl)
    t_h = time.perf_counter() - t0
    t0 = time.perf_counter()
    a0 = so.coulomb_operator(h, p.psi_kq, p.eps_k[v], 1.0)
    del h
    bs = np.array([so.rhs(p.psi_k[v], p.miller_k, p.miller_kq, p.dv_miller[q], p.psi_kq) for q in range(p.n_pert)])
    t_op = time.perf_counter() - t0
    t0 = time.perf_counter()
    so.solve_lu(a0, bs.T, p.omega[j] + 1j * p.eta)
    t_lu = time.perf_counter() - t0
    del a0
    log(f"cpu oracle: H {t_h:.1f} s, operator + {p.n_pert} right-hand sides {t_op:.1f} s, one LU solve {t_lu:.1f} s")
    t_full = t_h + p.n_band * t_op + p.n_band * p.n_omega * t_lu
    return {"value": p.n_solves / t_full, "unit": "solves/s", "cores": cores, "kind": "oracle", "cpu": model,
            "sample": f"oracle direct route on the host: dense H_k+q ({p.n_pw_kq} PW, {t_h:.1f} s), operator of "
                      f"one band + its {p.n_pert} right-hand sides ({t_op:.1f} s), one LU factorisation solving "
                      f"the {p.n_pert} perturbations at one frequency ({t_lu:.1f} s); value = {p.n_solves} "
                      f"solves / (t_H + {p.n_band} t_op + {p.n_band * p.n_omega} t_LU)"}


def cpu_baseline(problem, n_pairs_sample, log):
    """Time the oracle (dense H_{k+q}, full eigendecomposition, spectral sums) on a sample of pairs."""
    import oracle
    cores, model = _cpu_info()
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
    return {"value": value, "unit": "solves/s", "cores": int(cores), "kind": "oracle", "cpu": model,
            "sample": f"dense H_k+q + full eigh once ({t_setup:.1f} s) + spectral solves for {len(pairs)} of "
                      f"{n_total_pairs} (band, pert) pairs x {p.n_omega} omega ({t_pairs:.1f} s); value = "
                      f"all {n_total_pairs * p.n_omega} solves / (setup + per-pair time x {n_total_pairs})"}


def bench_dielectric(args, log, problem, ctx, dev):
    """The screening path on one GPU: for each chunk of bands, the solves at z_j = omega_j + i eta and at
    -z_j, then the density response of the chunk added into chi (the chunks bound the memory of the two
    solution arrays); finally eps, eps^-1 and W_bar per frequency.  One step is the whole path;
    `value` counts the solves of both signs per second of it."""
    import torch
    from paper_1812_03717_amd import sgw
    p = problem
    nbc = min(args.dielectric, p.n_band)
    kw = solve_kw(args, "block")
    opts = sgw.sgw_opts_default(**kw)
    ws = sgw.Workspace(ctx)
    shape = (nbc, p.n_pert, p.n_omega, p.n_pw_kq)
    dp = torch.empty(shape, dtype=torch.complex128, device=ctx.device)
    dm = torch.empty(shape, dtype=torch.complex128, device=ctx.device)
    info = torch.empty(nbc * p.n_pert * p.n_omega * sgw.INFO_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)
    chi = torch.empty((p.n_omega, p.n_pert, p.n_pert), dtype=torch.complex128, device=ctx.device)
    consumer_s, solve_s, n_ok = [], [], 0

    def step():
        nonlocal n_ok
        t_solve = t_cons = 0.0
        for c0 in range(0, p.n_band, nbc):
            bands = list(range(c0, min(c0 + nbc, p.n_band)))
            nb = len(bands)
            psi = dev.psi_v[c0:c0 + nb].contiguous()
            eps_v = dev.eps_v[c0:c0 + nb]
            for sgn, out in ((1.0, dp), (-1.0, dm)):
                t = time.perf_counter()
                st, _, inf = sgw.sternheimer_solve(ctx, dev.h_kq, dev.psi_occ_kq, dev.h_k, psi, eps_v, p.dv_miller,
                                                   sgn * p.omega, sgn * p.eta, p.tol, opts=opts, workspace=ws,
                                                   dpsi=out[:nb], info=info[: nb * p.n_pert * p.n_omega *
                                                                              sgw.INFO_DTYPE.itemsize])
                inf = sgw.info_to_numpy(inf)
                n_ok += int(np.count_nonzero((inf["flags"] & sgw.FLAG_CONVERGED) != 0))
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                t_solve += dt
                log(f"  bands {c0}..{c0 + nb - 1} at {'+' if sgn > 0 else '-'}z: {dt:.3f} s, status {st}, "
                    f"iters max {inf['iters'].max()}")
            t = time.perf_counter()
            sgw.sgw_density_response(ctx, dev.h_kq, dev.psi_occ_kq, dev.h_k, psi, p.dv_miller, dp[:nb], dm[:nb],
                                     chi=chi, accumulate=c0 > 0)
            torch.cuda.synchronize()
            t_cons += time.perf_counter() - t
        t = time.perf_counter()
        out = sgw.sgw_screened_coulomb(ctx, dev.h_kq, dev.h_k, p.dv_miller, chi)
        torch.cuda.synchronize()
        t_cons += time.perf_counter() - t
        solve_s.append(t_solve)
        consumer_s.append(t_cons)
        return out

    ctx.set_profiling("chi_dot,dielectric")
    for w in range(args.warmup):
        step()
        log(f"warmup {w}: solves {solve_s[-1]:.3f} s, density response + W_bar {consumer_s[-1]:.3f} s")
    ctx.reset_stats()
    solve_s.clear()
    consumer_s.clear()
    n_ok = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        eps, inv, wbar = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n_total = 2 * p.n_solves * args.steps
    log(f"timed: {args.steps} steps in {el:.3f} s; converged {n_ok}/{n_total}; solves {sum(solve_s):.3f} s, "
        f"density response + W_bar {sum(consumer_s):.3f} s")
    split = {}
    for k in ("chi_dot", "dielectric"):
        s = ctx.kernel_stats(k)
        if s["launches"]:
            sec = s["ms"] * 1e-3
            split[k] = {"ms_per_step": round(s["ms"] / args.steps, 2), "launches_per_step": s["launches"] // args.steps,
                        "alg_GBps": round(s["bytes"] / sec / 1e9, 1),
                        "alg_TFLOPs": round(s["flops"] / sec / 1e12, 2)}
    w = wbar.cpu().numpy()
    print(json.dumps({
        "metric": "Sternheimer solves/s (band x omega x pert, at z and -z) through chi, eps^-1 and W_bar",
        "value": round(n_ok / el, 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + "; solves at z and -z, density response, eps^-1, W_bar",
                   "band_chunk": nbc, "solves_per_step": 2 * p.n_solves, "max_iter": kw.get("max_iter", 600),
                   "solver": "block" if "solver" in kw else "multishift"},
        "consumer_ms_per_step": round(1e3 * sum(consumer_s) / args.steps, 2),
        "solve_ms_per_step": round(1e3 * sum(solve_s) / args.steps, 2),
        "kernel_split": split, "wbar_head_w0": [float(w[0, 0, 0].real), float(w[0, 0, 0].imag)]}))


def solve_kw(args, default):
    """Solver options of the screening and self-energy paths: `default` ("block" or "multishift")
    unless --solver names one; the block solver takes at most 160 block steps for si64 (as the
    headline), the multishift solver 3500 Krylov steps."""
    from paper_1812_03717_amd import sgw
    si64 = args.workload in ("si64", "si64nl")
    if (args.solver or default) == "block":
        max_iter = args.max_iter or (160 if si64 else 0)
        return dict(solver=sgw.SOLVER_BLOCK, **({"max_iter": max_iter} if max_iter else {}))
    max_iter = args.max_iter or (3500 if si64 else 0)
    return {"max_iter": max_iter} if max_iter else {}


def bench_batch(args, log):
    """Batches of uneven systems: sternheimer_solve_batch over all of them (one step) after autotuning
    each system class; the same systems solved one after another with default options give the
    sequential reference."""
    import torch
    import synth
    from paper_1812_03717_amd import sgw
    from paper_1812_03717_amd.workload import DeviceProblem

    t0 = time.perf_counter()
    # at 11.46 Ha the bases reach 13,539 plane waves: the generator's eigensolver runs on the GPU from
    # 5,000 plane waves (the host pool takes the smaller systems meanwhile), and the large cells' levels
    # at the occupation edge are ~5e-4 Ha apart, so the smallest accepted gap there is 3e-4 Ha
    kw = dict(ecut=11.46, gpu_min_pw=5000, min_gap=3e-4) if args.workload == "batch200e11" else {}
    problems = synth.batch(200, workers=min(16, os.cpu_count() or 1), **kw)
    n_solves = sum(p.n_solves for p in problems)
    log(f"generated 200 systems, {n_solves} solves ({time.perf_counter() - t0:.1f} s)")
    ctx = sgw.sgw_ctx_create(0)
    devs = [DeviceProblem(ctx, p) for p in problems]
    ws = sgw.Workspace(ctx)
    # the outputs of all systems at 11.46 Ha (~0.3 TB) exceed the HBM beside the workspace: the systems
    # go in consecutive groups whose outputs fit one caller-owned buffer, one batched call per group
    # (one group at 4 Ha); the sequential reference writes into the same buffer
    sizes = [p.n_solves * p.n_pw_kq for p in problems]
    cap = max(max(sizes), (args.batch_output_gib << 30) // 16)
    groups, cur, acc = [], [], 0
    for i, n in enumerate(sizes):
        if cur and acc + n > cap:
            groups.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += n
    groups.append(cur)
    outbuf = torch.empty(max(sum(sizes[i] for i in g) for g in groups), dtype=torch.complex128, device=ctx.device)

    def views(g):
        off, vs = 0, []
        for i in g:
            p = problems[i]
            vs.append(outbuf[off:off + sizes[i]].view(p.n_band, p.n_pert, p.n_omega, p.n_pw_kq))
            off += sizes[i]
        return vs

    # the largest cells (72^3, ~110 bands, dense spectrum in the frequency window) need up to ~4000
    # Krylov steps for their upper bands; the slot count is fitted to the workspace
    block = args.batch_solver == "block"
    if block:  # one block space per band over its perturbations; no autotuning (multishift settings)
        opts = lambda: sgw.sgw_opts_default(solver=sgw.SOLVER_BLOCK, max_iter=args.batch_block_steps)
    else:
        opts = lambda: sgw.sgw_opts_default(max_iter=args.batch_max_iter)
    batches = []
    for g in groups:
        b = sgw.Batch(ctx)
        for i, v in zip(g, views(g)):
            d, p = devs[i], problems[i]
            b.add(d.h_kq, d.psi_occ_kq, d.h_k, d.psi_v, d.eps_v, p.dv_miller, p.omega, p.eta, p.tol, opts=opts(),
                  dpsi=v)
        batches.append(b)
    items = [it for b in batches for it in b.items]
    t = time.perf_counter()
    tune_ms = 0.0 if block else sum(b.autotune(i) for b in batches for i in range(len(b.items)))
    log(f"{len(groups)} group(s) of {[len(g) for g in groups]} systems; "
        f"autotune: {tune_ms / 1e3:.2f} s (wall {time.perf_counter() - t:.2f} s); steps_per_sync/graph chosen: "
        f"{sorted({(it['problem'].opts.steps_per_sync, it['problem'].opts.graph) for it in items})}; "
        f"plane kernel (1 line, 2 pair, 3 LDS, 4 three-thread) per grid: "
        f"{sorted({(tuple(devs[i].h_kq.grid), it['problem'].opts.fft_planes) for i, it in enumerate(items)})}")
    workers = args.batch_workers

    def ok_count(items):
        n = 0
        for it in items:
            inf = sgw.info_to_numpy(it["info"])
            n += int(np.count_nonzero((inf["flags"] & sgw.FLAG_CONVERGED) != 0))
        return n

    # one workspace for the sequential and the batched runs, sized once: growing it between systems
    # would hold the old and the new buffer together
    need = max([b.workspace_size(workers) for b in batches] +
               [sgw.sternheimer_workspace_size(ctx, devs[i].h_kq, problems[i].n_occ, problems[i].n_band,
                                               problems[i].n_pert, problems[i].n_omega, opts())
                for i in range(len(problems))])
    ws.get(need)
    log(f"workspace {need / 2**30:.1f} GiB")
    # sequential reference: one system at a time, default options, the library's own stream
    torch.cuda.synchronize()
    t = time.perf_counter()
    seq_ok = 0
    for g in groups:
        for i, v in zip(g, views(g)):
            st, _, info = devs[i].solve(workspace=ws, opts=opts(), dpsi=v)
            inf = sgw.info_to_numpy(info)
            seq_ok += int(np.count_nonzero((inf["flags"] & sgw.FLAG_CONVERGED) != 0))
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t
    log(f"sequential: {seq_s:.3f} s, converged {seq_ok}/{n_solves}")
    for w in range(max(args.warmup, 1)):
        t = time.perf_counter()
        st = [b.solve(n_workers=workers, workspace=ws) for b in batches]
        torch.cuda.synchronize()
        log(f"warmup {w}: status {st}, {time.perf_counter() - t:.3f} s")
    ctx.reset_stats()
    ctx.set_profiling("hx_planes")
    n_ok = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for b in batches:
            b.solve(n_workers=workers, workspace=ws)
            n_ok += ok_count(b.items)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_profiling(None)
    ks = ctx.kernel_stats("hx_planes")
    value = n_ok / elapsed
    log(f"batch: {elapsed / args.steps:.3f} s per step, converged {n_ok}/{n_solves * args.steps}")
    out = {
        "metric": "Sternheimer solves/s (band x omega x pert) at true FP64 rel. residual <= tol",
        "value": round(value, 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "speedup_vs_sequential": round(value / (seq_ok / seq_s), 3), "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "solves_per_step": n_solves, "workers": workers,
                   "groups": len(groups),
                   "autotune_s": round(tune_ms / 1e3, 3), "sequential_solves_per_s": round(seq_ok / seq_s, 1),
                   "max_iter": args.batch_block_steps if block else args.batch_max_iter,
                   "method": ("FP64 block Lanczos-FOM over each band's perturbations, batched over worker "
                              "streams" if block else
                              "plain FP64 multishift Lanczos-FOM, batched over worker streams, autotuned")},
        "roofline": roofline("hx_planes", ks, args.workload),
    }
    print(json.dumps(out), flush=True)


def bench_learned(args, log):
    """The learned preconditioner and guess on held-out cells.  The model is trained on the GPU (the
    library's kernels) from per-shift residual histories of a 16-atom subset (5 bands x 4
    perturbations x 16 omega of the si16 workload) and three cells of the batch recipe (4 Ha); it
    is then evaluated on cells with seeds of their own, 16, 36 and 64 atoms at 48^3 to 72^3 with
    64 frequencies (bands lowest, middle and highest x 4 perturbations x 64 omega each), as the
    per-shift solver's preconditioner against the Teter diagonal (the fallback), with the multishift
    solver beside them.  Every solve is decided by its true FP64 residual (tol 1e-8)."""
    import torch
    import synth
    from paper_1812_03717_amd import sgw, training
    from paper_1812_03717_amd.workload import DeviceProblem
    ctx = sgw.sgw_ctx_create(0)
    ws = sgw.Workspace(ctx)
    t0 = time.perf_counter()
    train_sets = [(synth.si16(), [0, 8, 16, 24, 31], range(4), slice(None, None, 4))]
    train_sets += [(p, range(p.n_band), range(p.n_pert), slice(None)) for p in
                   synth.batch(3, seed0=9600, cells_max=2, n_omega_range=(16, 32), n_pert_range=(4, 6), workers=3)]
    feats, tgts = [], []
    for p, bands, perts, osel in train_sets:
        d = DeviceProblem(ctx, p)
        f, t = training.collect_rows(ctx, d, bands, perts, p.omega[osel], workspace=ws)
        feats.append(f)
        tgts.append(t)
        del d
    feat, tgt = torch.cat(feats), torch.cat(tgts)
    del feats, tgts
    mlp = sgw.sgw_mlp_create(ctx, seed=1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = training.train(ctx, mlp, feat, tgt, steps=2000, lr=2e-3, batch=32768)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    log(f"training: {feat.shape[0]} rows from {len(train_sets)} systems ({t1 - t0:.1f} s), 2000 Adam steps "
        f"{train_s:.2f} s, loss {losses[0]:.4f} -> {np.mean(losses[-20:]):.4f}")
    del feat, tgt
    # iteration limits that let the near-resonant top bands converge in every mode (a multishift Krylov
    # step is one operator application, a BiCGStab iteration two)
    modes = {"multishift": dict(max_iter=4000),
             "teter": dict(solver=sgw.SOLVER_PER_SHIFT, precond=sgw.PC_TETER, ps_max_iter=4000),
             "learned": dict(solver=sgw.SOLVER_PER_SHIFT, precond=sgw.PC_LEARNED, mlp=mlp, ps_max_iter=4000)}
    cells = {}
    tot = {m: [0, 0.0] for m in modes}
    for name, seed in (("fcc222", 9801), ("fcc233", 9802), ("conv222", 9803)):
        p = synth.held_out(name, seed)
        d = DeviceProblem(ctx, p)
        bands = [0, p.n_occ // 2, p.n_occ - 1]
        res = {}
        for m, kw in modes.items():
            opts = sgw.sgw_opts_default(**kw)
            d.solve(opts=opts, workspace=ws, bands=bands)   # warm-up (slots, graphs, workspace)
            torch.cuda.synchronize()
            t = time.perf_counter()
            st, _, info = d.solve(opts=opts, workspace=ws, bands=bands)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            inf = sgw.info_to_numpy(info)
            conv = int(np.count_nonzero(inf["flags"] & sgw.FLAG_CONVERGED))
            res[m] = {"iterations": int(inf["iters"].sum()), "converged": conv, "solves": int(inf.size),
                      "s": round(dt, 3), "solves_per_s": round(conv / dt, 1)}
            tot[m][0] += conv
            tot[m][1] += dt
        log(f"{p.name}: {p.n_pw_kq} PW, grid {p.grid}, n_occ {p.n_occ}, bands {bands}: {res}")
        cells[p.name] = {"n_pw": p.n_pw_kq, "grid": list(p.grid), "n_occ": p.n_occ, "bands": bands, **res}
    ratio = [cells[c]["learned"]["iterations"] / cells[c]["teter"]["iterations"] for c in cells]
    print(json.dumps({
        "metric": "per-shift solves/s at true FP64 rel. residual <= 1e-8 with the learned preconditioner and guess "
                  "on held-out cells (Teter fallback and the multishift solver beside it)",
        "value": round(tot["learned"][0] / tot["learned"][1], 1), "unit": "solves/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "held-out diamond cells, seeds 9801-9803: fcc 2x2x2 (16 atoms, 48^3), fcc 2x3x3 "
                               "(36 atoms, 48x72x72), conventional 2x2x2 (64 atoms, 72^3), Ecut 11.46 Ha, 3 bands x "
                               "4 perts x 64 omega in [0,40] eV each, eta 0.05 eV, tol 1e-8; model 5-64-64-4 trained "
                               "on si16 and batch-recipe cells (other seeds)",
                   "train_s": round(train_s, 2)},
        "learned_over_teter_iterations": [round(r, 3) for r in ratio],
        "teter_solves_per_s": round(tot["teter"][0] / tot["teter"][1], 1),
        "multishift_solves_per_s": round(tot["multishift"][0] / tot["multishift"][1], 1),
        "cells": cells}), flush=True)
    mlp.close()


def sigma_frequencies(n_int=32, n_out=12, h=0.25):
    """Imaginary-axis meshes of the self-energy path: integration frequencies w'_j = h (j + 1/2),
    j = -n_int/2 .. n_int/2 - 1 (midpoint rule, weight h each), outputs w_k = h k, k < n_out; the
    differences w'_j - w_k all lie on the half-integer mesh h (m + 1/2), where W_bar is needed.
    Returns (w_int, weights, w_out, nu, w_index)."""
    j = np.arange(-(n_int // 2), n_int - n_int // 2)
    w_int = h * (j + 0.5)
    w_out = h * np.arange(n_out)
    m = j[None, :] - np.arange(n_out)[:, None]
    m_all = np.arange(m.min(), m.max() + 1)
    return w_int, np.full(n_int, h), w_out, h * (m_all + 0.5), (m - m.min()).astype(np.int32)


def bench_sigma(args, log, problem, ctx, dev):
    """The correlation self-energy path of the top STATES bands on one GPU (Eq. 10).  Imaginary axis
    (default): W_bar on the imaginary-axis mesh first, untimed (solves at +-i nu over all bands,
    density response, eps^-1); one step is then the Green's function pair elements (multishift solves
    at mu + i w'_j for every state and wave vector), the frequency convolution Sigma^c(i w_k), an AAA
    fit per state, the spectral function on 2001 real frequencies and the quasiparticle energies.
    Real axis (--sigma-axis real): W_bar at the real differences nu + i eta (eta = 0.15 eV), untimed;
    one step is the pair elements at the time-ordered w'_j + i eta sgn(w'_j - mu) and Sigma^c(w_k)
    with alpha = i.  `value` counts the pair-element solves per second of the step."""
    import torch
    from paper_1812_03717_amd import sgw
    p = problem
    real = args.sigma_axis == "real"
    n_st = min(args.sigma, p.n_band)
    # the pair elements are a small problem (16 states x 20 wave vectors per launch): the multishift
    # solver is the faster there (measured: 75.5k against 67.8k solves/s with the block solver)
    kw = solve_kw(args, "multishift")
    mu = 0.5 * (p.eps_kq[p.n_occ - 1] + p.eps_kq[p.n_occ])
    eta_r = 0.15 / 27.211386245988
    if real:
        # w'_j = mu + h (j + 1/2), j = -32..31 (h = 0.125 Ha), outputs mu + h k, k = -8..7
        w_int, q_int, w_out, nu, w_index = sigma_frequencies(n_int=64, n_out=16, h=0.125)
        w_int, w_out = mu + w_int, mu + w_out - 8 * 0.125
        diff = w_int[None, :] - w_out[:, None]
        nu, inv = np.unique(np.round(diff, 12), return_inverse=True)
        w_index = inv.reshape(diff.shape).astype(np.int32)
    else:
        w_int, q_int, w_out, nu, w_index = sigma_frequencies()
    ws = sgw.Workspace(ctx)
    # W_bar from all bands, in chunks of 32 bands (untimed)
    t = time.perf_counter()
    nbc = min(32, p.n_band)
    zero = np.zeros(len(nu))
    chi = torch.empty((len(nu), p.n_pert, p.n_pert), dtype=torch.complex128, device=ctx.device)
    for c0 in range(0, p.n_band, nbc):
        nb = min(nbc, p.n_band - c0)
        psi = dev.psi_v[c0:c0 + nb].contiguous()
        sols = []
        for sgn in (1.0, -1.0):
            if real:
                o = sgw.sgw_opts_default(**kw)
                st, x, _ = sgw.sternheimer_solve(ctx, dev.h_kq, dev.psi_occ_kq, dev.h_k, psi, dev.eps_v[c0:c0 + nb],
                                                 p.dv_miller, sgn * nu, sgn * eta_r, p.tol, opts=o, workspace=ws)
            else:
                o = sgw.sgw_opts_default(shift_imag=sgn * nu, **kw)
                st, x, _ = sgw.sternheimer_solve(ctx, dev.h_kq, dev.psi_occ_kq, dev.h_k, psi, dev.eps_v[c0:c0 + nb],
                                                 p.dv_miller, zero, 0.0, p.tol, opts=o, workspace=ws)
            sols.append(x)
        sgw.sgw_density_response(ctx, dev.h_kq, dev.psi_occ_kq, dev.h_k, psi, p.dv_miller, sols[0], sols[1], chi=chi,
                                 accumulate=c0 > 0)
        del sols
        log(f"  W_bar: bands {c0}..{c0 + nb - 1} at +-{'(nu + i eta)' if real else 'i nu'} ({len(nu)} frequencies), "
            f"status {st}")
    _, _, wbar = sgw.sgw_screened_coulomb(ctx, dev.h_kq, dev.h_k, p.dv_miller, chi)
    torch.cuda.synchronize()
    log(f"W_bar on {len(nu)} {'real' if real else 'imaginary'} frequencies: {time.perf_counter() - t:.1f} s (untimed)")
    states = list(range(p.n_band - n_st, p.n_band))
    psi_n = dev.psi_v[states[0]:].contiguous()
    eps_n = np.asarray(p.eps_k[states], np.float64)
    z_g = w_int + 1j * eta_r * np.sign(w_int - mu) if real else mu + 1j * w_int
    opts = sgw.sgw_opts_default(**kw)
    omega = np.linspace(-1.0, 1.0, 2001)
    vol = float(abs(np.linalg.det(p.A)))
    stage = {"pair_elements": [], "sigma_c": [], "aaa": [], "spectral": []}
    n_ok = 0

    def step():
        nonlocal n_ok
        t0 = time.perf_counter()
        st, m, info = sgw.sgw_green_pair_elements(ctx, dev.h_kq, dev.h_k, psi_n, p.dv_miller, z_g, p.tol, opts=opts,
                                                  workspace=ws)
        inf = sgw.info_to_numpy(info)
        n_ok += int(np.count_nonzero((inf["flags"] & sgw.FLAG_CONVERGED) != 0))
        t1 = time.perf_counter()
        sig = sgw.sgw_sigma_c(ctx, m, q_int, wbar, w_index, vol, alpha=1j if real else -1.0).cpu().numpy()
        t2 = time.perf_counter()
        qp = []
        if not real:
            fits = [sgw.sgw_aaa_fit(1j * w_out, sig[n], tol=1e-12) for n in range(n_st)]
        t3 = time.perf_counter()
        if not real:
            _, a = sgw.sgw_spectral_function(ctx, fits, omega, 1e-3, eps_n, np.zeros(n_st))
            qp = [sgw.sgw_quasiparticle(f, e, 0.0) for f, e in zip(fits, eps_n)]
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for k, dt in zip(stage, (t1 - t0, t2 - t1, t3 - t2, t4 - t3)):
            stage[k].append(dt)
        log(f"  pair elements {t1 - t0:.3f} s (status {st}, iters max {inf['iters'].max()}), Sigma^c {t2 - t1:.4f} s, "
            f"AAA {t3 - t2:.4f} s, A(w) + E_qp {t4 - t3:.4f} s")
        return sig, qp

    for _ in range(args.warmup):
        step()
    for v in stage.values():
        v.clear()
    n_ok = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sig, qp = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n_solves = n_st * p.n_pert * len(w_int)
    log(f"timed: {args.steps} steps in {el:.3f} s; converged {n_ok}/{n_solves * args.steps}")
    if real:
        desc = (f"; Sigma^c of the top {n_st} bands along the real axis: pair elements at w' + i eta sgn(w' - mu) "
                f"({len(w_int)} frequencies, h 0.125 Ha, eta 0.15 eV), W_bar at {len(nu)} frequencies nu + i eta "
                f"(untimed), Sigma^c at {len(w_out)} frequencies (alpha = i)")
    else:
        desc = (f"; Sigma^c of the top {n_st} bands: pair elements at mu + i w' ({len(w_int)} midpoint frequencies, "
                f"h 0.25 Ha), W_bar at {len(nu)} frequencies (untimed), Sigma^c at {len(w_out)} frequencies, AAA, "
                f"A(w) on 2001 points")
    out = {
        "metric": "Green's function pair-element solves/s (state x wave vector x frequency) through Sigma^c"
                  + ("" if real else ", AAA continuation and A(w)"),
        "value": round(n_ok / el, 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + desc, "axis": args.sigma_axis,
                   "solves_per_step": n_solves, "max_iter": kw.get("max_iter", 600),
                   "solver": "block" if "solver" in kw else "multishift"},
        "stage_ms_per_step": {k: round(1e3 * sum(v) / args.steps, 3) for k, v in stage.items()},
        "sigma_c_top_state_w0": [float(sig[-1, 0].real), float(sig[-1, 0].imag)]}
    if qp:
        out["z_factors"] = [round(z, 4) for _, z in qp]
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="si64", choices=sorted(WORKLOADS))
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--max-iter", type=int, default=0,
                    help="Krylov steps per pair before a solve is flagged (0: 3500 for si64, else the library "
                         "default)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="the timed method; mixed: FP32 potential matvecs once a pair's residuals are small, "
                         "FP64 refinement, with a plain FP64 leg timed beside it")
    ap.add_argument("--mixed-switch", type=float, default=0.0)
    ap.add_argument("--solver", choices=["multishift", "block"], default=None,
                    help="block (default in FP64): one block Krylov space per band over its perturbations "
                         "(max_iter then limits the block steps, 0: 160 for si64), with the multishift solver "
                         "timed beside it; multishift (default with --precision mixed): one Krylov space per "
                         "(band, perturbation)")
    ap.add_argument("--compare-steps", type=int, default=2,
                    help="timed steps of the multishift solver beside the block solver (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-workers", type=int, default=4)
    ap.add_argument("--batch-max-iter", type=int, default=4000)
    ap.add_argument("--batch-solver", choices=["multishift", "block"], default="block",
                    help="solver of the batch workloads (block: at most --batch-block-steps block steps; "
                         "multishift: --batch-max-iter Krylov steps, autotuned)")
    ap.add_argument("--batch-block-steps", type=int, default=600)
    ap.add_argument("--batch-output-gib", type=int, default=100,
                    help="device memory for the batch outputs; systems are grouped to fit it")
    ap.add_argument("--cpu-sample-pairs", type=int, default=160)
    ap.add_argument("--dielectric", type=int, default=0, metavar="BANDS",
                    help="time the screening path instead: solves at z and -z for BANDS bands at a time, the "
                         "density response accumulated over the band chunks, eps, eps^-1 and W_bar")
    ap.add_argument("--learned", action="store_true",
                    help="train the learned preconditioner and compare it with the Teter fallback on held-out "
                         "16-, 36- and 64-atom cells with 64 frequencies")
    ap.add_argument("--sigma", type=int, default=0, metavar="STATES",
                    help="time the self-energy path of the top STATES bands instead (W_bar untimed): Green's "
                         "function pair elements, Sigma^c on the imaginary axis, AAA, A(w), E_qp")
    ap.add_argument("--sigma-axis", choices=["imag", "real"], default="imag",
                    help="frequency convolution of --sigma along the imaginary axis (then AAA) or the real axis")
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
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(across GPUs each would take a slice of the (band, perturbation) pair queue)", file=sys.stderr)
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
    if args.learned:
        return bench_learned(args, log)
    if args.workload in ("batch200", "batch200e11"):
        return bench_batch(args, log)
    t0 = time.perf_counter()
    problem = getattr(synth, args.workload)()
    log(f"generated {args.workload}: {problem.n_pw_kq} PW, grid {problem.grid}, {problem.n_solves} solves "
        f"({time.perf_counter() - t0:.1f} s)")
    ctx = sgw.sgw_ctx_create(0)
    dev = DeviceProblem(ctx, problem)
    if args.dielectric:
        return bench_dielectric(args, log, problem, ctx, dev)
    if args.sigma:
        return bench_sigma(args, log, problem, ctx, dev)
    ws = sgw.Workspace(ctx)
    prec = sgw.MIXED if args.precision == "mixed" else sgw.FP64
    kw = dict(precision=prec)
    if args.slots:
        kw["slots"] = args.slots
    if args.solver is None:
        args.solver = "block" if args.precision == "fp64" else "multishift"
    block = args.solver == "block"
    if block:
        if prec != sgw.FP64:
            log("the block solver runs in FP64 only")
            sys.exit(2)
        kw["solver"] = sgw.SOLVER_BLOCK
    max_iter = args.max_iter or ((160 if block else 3500) if args.workload in ("si64", "si64nl") else 0)
    if max_iter:
        kw["max_iter"] = max_iter
    if args.mixed_switch:
        kw["mixed_switch"] = args.mixed_switch
    opts = sgw.sgw_opts_default(**kw)
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
    n_warm = max(args.warmup, 1)
    split = {}  # per kernel, over the warmup solves (every launch timed): ms per step and achieved rates
    for k, s in sorted(stats.items(), key=lambda kv: -kv[1]["ms"]):
        if s["launches"]:
            log(f"  {k:14s} {s['ms']:9.2f} ms  {100 * s['ms'] / total:5.1f}%  launches {s['launches']}")
            sec = s["ms"] * 1e-3
            split[k] = {"ms_per_step": round(s["ms"] / n_warm, 1), "launches_per_step": s["launches"] // n_warm,
                        "alg_GBps": round(s["bytes"] / sec / 1e9, 1),
                        "alg_TFLOPs": round(s["flops"] / sec / 1e12, 2) if s["flops"] else None}
    dominant = max(stats, key=lambda k: stats[k]["ms"])

    step_s = []

    def timed(o, profile):
        """Run args.steps solves; returns (elapsed s, converged solves, last info).  Each solve ends
        with its stream synchronised and its info copied to the host, so the per-step times kept in
        step_s are exact."""
        ctx.reset_stats()
        ctx.set_profiling(profile)
        n_ok, inf = 0, None
        step_s.clear()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            dev.solve(opts=o, workspace=ws, dpsi=dpsi, info=info)
            inf = sgw.info_to_numpy(info)
            step_s.append(time.perf_counter() - ts)
            n_ok += int(np.count_nonzero((inf["flags"] & sgw.FLAG_CONVERGED) != 0))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.set_profiling(None)
        return el, n_ok, inf

    def report(tag, el, n_ok, inf, steps=None):
        steps = steps or args.steps
        log(f"{tag}: {steps} steps in {el:.3f} s; converged {n_ok}/{problem.n_solves * steps}; "
            f"iters min/mean/max {inf['iters'].min()}/{inf['iters'].mean():.1f}/{inf['iters'].max()}; "
            f"max relres {inf['relres'].max():.3e}; refined per shift "
            f"{int(np.count_nonzero((inf['flags'] & sgw.FLAG_PER_SHIFT) != 0))}")

    # timed steps of the chosen method; plain FP64 beside it, with events around the dominant kernel
    multishift = None
    if block:
        elapsed, n_ok, inf = timed(opts, dominant)
        med_ms = 1e3 * float(np.median(step_s))
        report("timed (block fp64)", elapsed, n_ok, inf)
        p_el, p_ok = elapsed, n_ok
        ks = ctx.kernel_stats(dominant)
        if args.compare_steps > 0:
            # the multishift solver on the same systems (its own max_iter), fewer steps
            mkw = {k: v for k, v in kw.items() if k != "solver"}
            mkw["max_iter"] = args.max_iter or (3500 if args.workload in ("si64", "si64nl") else 600)
            mopts = sgw.sgw_opts_default(**mkw)
            dev.solve(opts=mopts, workspace=ws, dpsi=dpsi, info=info)
            torch.cuda.synchronize()
            saved = args.steps
            args.steps = args.compare_steps
            m_el, m_ok, m_inf = timed(mopts, None)
            args.steps = saved
            report("timed (multishift fp64)", m_el, m_ok, m_inf, steps=args.compare_steps)
            multishift = {"value": round(m_ok / m_el, 1), "steps": args.compare_steps,
                          "ms_per_step": round(1e3 * m_el / args.compare_steps, 3), "max_iter": mkw["max_iter"],
                          "converged": m_ok}
    elif prec == sgw.FP64:
        elapsed, n_ok, inf = timed(opts, dominant)
        med_ms = 1e3 * float(np.median(step_s))
        report("timed (plain fp64)", elapsed, n_ok, inf)
        p_el, p_ok = elapsed, n_ok
    else:
        elapsed, n_ok, inf = timed(opts, None)
        med_ms = 1e3 * float(np.median(step_s))
        report(f"timed ({args.precision})", elapsed, n_ok, inf)
        plain = sgw.sgw_opts_default(**{k: v for k, v in kw.items() if k in ("slots", "max_iter")})
        p_el, p_ok, p_inf = timed(plain, dominant)
        report("timed (plain fp64)", p_el, p_ok, p_inf)
    if not block:
        ks = ctx.kernel_stats(dominant)
    roof = roofline(dominant, ks, args.workload, default_launch=not args.slots)
    roof["leg"] = "block FP64 timed steps" if block else "plain FP64 timed steps"
    value = n_ok / elapsed
    plain_value = p_ok / p_el
    out = {
        "metric": "Sternheimer solves/s (band x omega x pert) at true FP64 rel. residual <= tol",
        "value": round(value, 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "step_ms_median": round(med_ms, 3),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == sgw.FP64 else "f64+f32", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "solves_per_step": problem.n_solves,
                   "max_iter": max_iter or 600,
                   "method": ("block Lanczos-FOM over each band's perturbations (block steps <= max_iter), FP64, "
                              "per-shift refinement of any shift whose true residual misses tol") if block else
                             "multishift Lanczos-FOM, stored basis, " +
                             ("FP64" if prec == sgw.FP64 else "FP64 with FP32 potential matvecs once a pair's "
                              "shift residuals are below 1e4*tol, FP64 per-shift refinement of any shift above tol")},
        "roofline": roof,
        "kernel_split": split,
    }
    if block:
        if multishift:
            out["multishift_fp64"] = multishift
            out["speedup_vs_multishift"] = round(value / multishift["value"], 4)
            # the metric's "speedup vs plain FP64": the reference is the plain FP64 multishift solver on
            # the same systems (the block solver is FP64 as well)
            out["speedup_vs_plain_fp64"] = out["speedup_vs_multishift"]
            out["plain_fp64_value"] = multishift["value"]
            out["plain_fp64_reference"] = "multishift solver, FP64, same systems"
    else:
        out["speedup_vs_plain_fp64"] = round(value / plain_value, 4)
        out["plain_fp64_value"] = round(plain_value, 1)
    if not args.no_cpu_baseline:
        if args.workload in ("si64", "si64nl"):
            out["cpu_baseline"] = cpu_baseline_lu(problem, log)
        else:
            out["cpu_baseline"] = cpu_baseline(problem, args.cpu_sample_pairs, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
