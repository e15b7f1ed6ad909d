"""Summaries of rocprofv3 results (rocpd SQLite databases) for the library's kernels.

    python -m paper_1812_03717_amd.profiling top DB [--since KERNEL]
    python -m paper_1812_03717_amd.profiling pmc DB
    python -m paper_1812_03717_amd.profiling traffic --kernel k_planes --fetch DB --write DB \
        --copy-fetch DB --copy-write DB --copy-bytes N [--bench-line FILE] [--out FILE.json]
    python -m paper_1812_03717_amd.profiling mfma --pmc DB --trace DB --kernel k_proj_dot [--kernel ...]
    python -m paper_1812_03717_amd.profiling valu --pmc DB --trace DB --kernel k_planes_line [--alg-flops F]
    python -m paper_1812_03717_amd.profiling stalls --pmc DB [--pmc DB ...] --kernel k_planes_pair
    python -m paper_1812_03717_amd.profiling blkprod DB

``traffic`` scales the per-dispatch FETCH_SIZE and WRITE_SIZE averages (KiB) of
one kernel by what the same counters read for a plain device copy of known
size, and records a hash of the kernel's sources so that a later change of the
kernel marks the numbers stale (``source_hash``).  With ``--bench-line`` (a file
holding the JSON line that the counted bench run printed) it also records the
algorithmic bytes per launch of that run, so that a later run whose launches
have another size (another workspace budget, another batch) can tell that the
counters do not describe its launches.

``mfma`` reports, per kernel, the FP64 matrix flops per dispatch
(SQ_INSTS_VALU_MFMA_MOPS_F64 counts units of 512 flops), the achieved rate over
the traced average duration, and the fraction of SIMD cycles the matrix units
were busy (SQ_VALU_MFMA_BUSY_CYCLES, summed over the SIMDs, against the traced
duration on all 1024 SIMDs at the 2.4 GHz peak clock).
"""
from __future__ import annotations

import argparse
import collections
import functools
import hashlib
import json
import os
import re
import sqlite3

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# sources that define each timed kernel
KERNEL_SOURCES = {
    "hx_planes": ["planes.h", "fft_reg.h", "fft_lds.h", "twiddle_const.h", "hx.hip"],
    "hx_sticks_inv": ["hx.hip", "planes.h", "fft_reg.h", "fft_lds.h", "twiddle_const.h", "sgw_internal.h"],
    "hx_sticks_fwd": ["hx.hip", "planes.h", "fft_reg.h", "fft_lds.h", "twiddle_const.h", "sgw_internal.h"],
    "proj_dot": ["projector.hip"],
    "proj_apply": ["projector.hip"],
    # rocBLAS products whose shapes and count the block solver sets
    "blk_product": ["block.hip"],
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def short_name(n: str) -> str:
    """Kernel symbol with its template arguments, e.g. k_planes<double2, 48, 48>."""
    n = n.replace("HIP_vector_type<double, 2u>", "double2").replace("HIP_vector_type<float, 2u>", "float2")
    m = re.search(r"k_\w+", n)
    if not m:
        return n[:60]
    out, i = m.group(0), m.end()
    if i < len(n) and n[i] == "<":
        depth = 0
        for j in range(i, len(n)):
            depth += (n[j] == "<") - (n[j] == ">")
            if depth == 0:
                out += n[i:j + 1]
                break
    return out


def top(db: str, since: str | None = None):
    """(kernel, calls, total_us, avg_us, pct) by total duration; with `since`, only the dispatches from
    the first one whose name contains `since` on (e.g. the solves, without the input generation)."""
    c = sqlite3.connect(db)
    if not since:
        rows = c.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                         "order by total_duration desc").fetchall()
        return [(short_name(n), calls, tot, avg, pct) for n, calls, tot, avg, pct in rows]
    agg = collections.defaultdict(lambda: [0, 0.0])
    on = False
    for name, dur in c.execute("select name, duration from kernels order by start"):
        on = on or since in name
        if on:
            k = name.split("_MI")[0][:40] if name.startswith("Cijk") else short_name(name)
            agg[k][0] += 1
            agg[k][1] += dur / 1e3  # ns -> us
    tot_all = sum(v[1] for v in agg.values()) or 1.0
    return sorted(((k, n, t, t / n, 100.0 * t / tot_all) for k, (n, t) in agg.items()), key=lambda r: -r[2])


@functools.lru_cache(maxsize=None)
def pmc(db: str):
    """{(kernel, counter): (dispatches, average value)} (read once per database)"""
    c = sqlite3.connect(db)
    agg = collections.defaultdict(lambda: [0, 0.0])
    for name, cn, val in c.execute("select kernel_name, counter_name, value from counters_collection"):
        k = (short_name(name), cn)
        agg[k][0] += 1
        agg[k][1] += val
    return {k: (n, s / n) for k, (n, s) in agg.items()}


def _avg(db, kernel_prefix, counter):
    """(dispatches, average per dispatch) of a counter over every kernel whose name starts with
    kernel_prefix (all template instances of it)"""
    n_all, tot = 0, 0.0
    for (k, cn), (n, avg) in pmc(db).items():
        if cn == counter and k.startswith(kernel_prefix):
            n_all += n
            tot += n * avg
    if not n_all:
        raise KeyError(f"{kernel_prefix}/{counter} not in {db}")
    return n_all, tot / n_all


def traffic(kernel_prefix, fetch_db, write_db, copy_fetch_db, copy_write_db, copy_bytes):
    nf, fetch_kib = _avg(fetch_db, kernel_prefix, "FETCH_SIZE")
    nw, write_kib = _avg(write_db, kernel_prefix, "WRITE_SIZE")
    _, cf = _avg(copy_fetch_db, "__amd_rocclr_copyBuffer", "FETCH_SIZE")
    _, cw = _avg(copy_write_db, "__amd_rocclr_copyBuffer", "WRITE_SIZE")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    return {"fetch_bytes_per_dispatch": fetch_kib * 1024.0 * f_scale,
            "write_bytes_per_dispatch": write_kib * 1024.0 * w_scale,
            "fetch_scale": f_scale, "write_scale": w_scale, "dispatches": [nf, nw]}


N_SIMD = 256 * 4      # MI355X: 256 compute units of 4 SIMDs
CLOCK_HZ = 2.4e9      # peak engine clock
FP64_MFMA_PEAK = 78.6e12


def mfma(pmc_db, trace_db, kernel_prefix):
    """{dispatches, avg_us, flops, tflops, frac_peak, busy_frac} of one kernel."""
    durs = [(calls, avg) for n, calls, tot, avg, pct in top(trace_db) if n.startswith(kernel_prefix)]
    if not durs:
        raise KeyError(f"{kernel_prefix} not in {trace_db}")
    calls = sum(c for c, _ in durs)
    avg_us = sum(c * a for c, a in durs) / calls
    n, mops = _avg(pmc_db, kernel_prefix, "SQ_INSTS_VALU_MFMA_MOPS_F64")
    _, busy = _avg(pmc_db, kernel_prefix, "SQ_VALU_MFMA_BUSY_CYCLES")
    flops = mops * 512.0
    return {"dispatches": n, "avg_us": avg_us, "flops": flops, "tflops": flops / (avg_us * 1e-6) / 1e12,
            "frac_peak": flops / (avg_us * 1e-6) / FP64_MFMA_PEAK,
            "busy_frac": busy / (avg_us * 1e-6 * CLOCK_HZ * N_SIMD)}


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                 "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_WAVES")


def valu(pmc_db, trace_db, kernel_prefix):
    """Per-dispatch instruction counts of one kernel (per wavefront instruction issued) and the share
    of the SIMDs' cycles its VALU instructions occupy: a wave64 VALU instruction takes 4 cycles of
    a 16-lane SIMD, against the traced duration on all 1024 SIMDs at the 2.4 GHz peak clock."""
    durs = [(calls, avg) for n, calls, tot, avg, pct in top(trace_db) if n.startswith(kernel_prefix)]
    if not durs:
        raise KeyError(f"{kernel_prefix} not in {trace_db}")
    calls = sum(c for c, _ in durs)
    avg_us = sum(c * a for c, a in durs) / calls
    r = {"avg_us": avg_us}
    for c in VALU_COUNTERS:
        r[c] = _avg(pmc_db, kernel_prefix, c)[1]
    f64 = r["SQ_INSTS_VALU_ADD_F64"] + r["SQ_INSTS_VALU_MUL_F64"] + r["SQ_INSTS_VALU_FMA_F64"]
    cyc = avg_us * 1e-6 * CLOCK_HZ * N_SIMD
    r["fp64_share"] = f64 / r["SQ_INSTS_VALU"]
    r["valu_busy"] = 4.0 * r["SQ_INSTS_VALU"] / cyc
    r["fp64_busy"] = 4.0 * f64 / cyc
    # flops the FP64 instructions would do with all 64 lanes active (FMA = 2)
    r["fp64_flops_full_lanes"] = 64.0 * (r["SQ_INSTS_VALU_ADD_F64"] + r["SQ_INSTS_VALU_MUL_F64"] +
                                         2.0 * r["SQ_INSTS_VALU_FMA_F64"])
    return r


STALL_COUNTERS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                  "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
                  "SQ_ACTIVE_INST_SCA", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_LDS_BANK_CONFLICT",
                  "SQ_LDS_IDX_ACTIVE")


def stalls(pmc_dbs, kernel_prefix):
    """Per-dispatch SQ counters of one kernel gathered from several counter passes, and the shares
    of the waves' lifetime (SQ_WAVE_CYCLES) spent issuing VALU or LDS instructions and waiting."""
    r = {}
    for c in STALL_COUNTERS:
        for db in pmc_dbs:
            try:
                r[c] = _avg(db, kernel_prefix, c)[1]
                break
            except KeyError:
                continue
    wc = r.get("SQ_WAVE_CYCLES")
    if wc:
        for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_ANY",
                  "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS"):
            if c in r:
                r[c + "/wave_cycles"] = r[c] / wc
    if r.get("SQ_WAVES") and "SQ_INSTS_VALU" in r:
        r["valu_insts_per_wave"] = r["SQ_INSTS_VALU"] / r["SQ_WAVES"]
    if r.get("SQ_LDS_IDX_ACTIVE") and "SQ_LDS_BANK_CONFLICT" in r:
        r["lds_conflict/lds_active"] = r["SQ_LDS_BANK_CONFLICT"] / r["SQ_LDS_IDX_ACTIVE"]
    return r


def blk_products(db: str):
    """The block solver's final products: rocBLAS kernels (Cijk_*) whose latest preceding block-solver
    kernel (k_blk_*) is k_blk_solve or k_blk_final, i.e. the launches timed as "blk_product".
    Returns {dispatches, total_ms, avg_us, kernels}."""
    c = sqlite3.connect(db)
    last, durs, names = None, [], collections.Counter()
    for name, dur in c.execute("select name, duration from kernels order by start"):
        m = re.search(r"k_blk_\w+", name)
        if m:
            last = m.group(0)
        elif name.startswith("Cijk") and last in ("k_blk_solve", "k_blk_final"):
            durs.append(dur)
            names[name.split("_MT")[0] + "_MT" + name.split("_MT")[1].split("_")[0]] += 1
    tot = sum(durs)
    return {"dispatches": len(durs), "total_ms": tot / 1e6, "avg_us": tot / max(len(durs), 1) / 1e3,
            "kernels": dict(names)}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("top")
    t.add_argument("db")
    t.add_argument("--since", help="only dispatches from the first kernel whose name contains this on")
    p = sub.add_parser("pmc")
    p.add_argument("db")
    r = sub.add_parser("traffic")
    r.add_argument("--kernel", required=True, help="kernel symbol prefix, e.g. k_planes")
    r.add_argument("--name", required=True, help="library kernel name, e.g. hx_planes")
    for k in ("fetch", "write", "copy-fetch", "copy-write"):
        r.add_argument(f"--{k}", required=True)
    r.add_argument("--copy-bytes", type=float, required=True)
    r.add_argument("--bench-line", help="file with the JSON line the counted bench run printed")
    r.add_argument("--out")
    m = sub.add_parser("mfma")
    m.add_argument("--pmc", required=True)
    m.add_argument("--trace", required=True)
    m.add_argument("--kernel", action="append", required=True)
    v = sub.add_parser("valu")
    v.add_argument("--pmc", required=True)
    v.add_argument("--trace", required=True)
    v.add_argument("--kernel", required=True)
    v.add_argument("--alg-flops", type=float, default=0.0, help="algorithmic flops per dispatch, if known")
    b = sub.add_parser("blkprod")
    b.add_argument("db")
    s = sub.add_parser("stalls")
    s.add_argument("--pmc", action="append", required=True)
    s.add_argument("--kernel", required=True)
    a = ap.parse_args()
    if a.cmd == "top":
        # rocpd reports durations in microseconds
        print(f"{'kernel':40s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>9s} {'pct':>6s}")
        for n, calls, tot, avg, pct in top(a.db, a.since):
            print(f"{n:40s} {calls:7d} {tot / 1e3:10.2f} {avg:9.2f} {pct:6.2f}")
    elif a.cmd == "blkprod":
        r = blk_products(a.db)
        print(f"block solver final products: {r['dispatches']} dispatches, {r['total_ms']:.2f} ms, "
              f"avg {r['avg_us']:.2f} us")
        for k, n in r["kernels"].items():
            print(f"  {k}: {n}")
    elif a.cmd == "pmc":
        for (k, cn), (n, avg) in sorted(pmc(a.db).items()):
            unit = " KiB" if cn in ("FETCH_SIZE", "WRITE_SIZE") else ""
            print(f"{k:40s} {cn:12s} dispatches {n:6d} avg {avg:14.1f}{unit}")
    elif a.cmd == "mfma":
        print(f"{'kernel':24s} {'dispatches':>10s} {'avg_us':>8s} {'GFLOP/disp':>10s} {'TFLOP/s':>8s} "
              f"{'of_peak':>7s} {'mfma_busy':>9s}")
        for k in a.kernel:
            r = mfma(a.pmc, a.trace, k)
            print(f"{k:24s} {r['dispatches']:10d} {r['avg_us']:8.2f} {r['flops'] / 1e9:10.3f} {r['tflops']:8.2f} "
                  f"{r['frac_peak']:7.3f} {r['busy_frac']:9.3f}")
    elif a.cmd == "valu":
        r = valu(a.pmc, a.trace, a.kernel)
        print(f"{a.kernel}: {r['avg_us']:.2f} us per dispatch, {r['SQ_WAVES']:.0f} waves")
        for c in VALU_COUNTERS[:-1]:
            print(f"  {c:24s} {r[c]:16.0f}")
        print(f"  FP64 share of VALU instructions   {r['fp64_share']:.3f}")
        print(f"  VALU issue / SIMD cycles          {r['valu_busy']:.3f}   (FP64 alone {r['fp64_busy']:.3f})")
        print(f"  FP64 flops at full lanes          {r['fp64_flops_full_lanes'] / 1e9:.3f} GFLOP per dispatch")
        if a.alg_flops:
            print(f"  algorithmic / full-lane FP64 flops {a.alg_flops / r['fp64_flops_full_lanes']:.3f}")
    elif a.cmd == "stalls":
        print(f"{a.kernel}: per dispatch")
        for k, v in stalls(a.pmc, a.kernel).items():
            print(f"  {k:34s} {v:16.3f}" if v < 100 else f"  {k:34s} {v:16.0f}")
    else:
        res = traffic(a.kernel, a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes)
        res["kernel"] = a.name
        if a.bench_line:
            with open(a.bench_line) as fh:
                line = [ln for ln in fh if ln.lstrip().startswith("{")][-1]
            roof = json.loads(line)["roofline"]
            if roof.get("kernel") != a.name:
                raise SystemExit(f"the bench line's dominant kernel is {roof.get('kernel')}, not {a.name}")
            res["alg_bytes_per_launch"] = roof["alg_bytes_per_launch"]
        res["source_hash"] = source_hash(a.name)
        print(json.dumps(res, indent=1))
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(res, fh, indent=1)
                fh.write("\n")


if __name__ == "__main__":
    main()
