"""Benchmark of the gfx950 SpGEMM path on one MI355X.

One step = the whole product C = A*B as the paper times it (setup + symbolic +
numeric, Section 4.2): plan (setup, precise symbolic phase), allocation of C,
numeric phase, release.  Inputs are resident in device memory before the
timed region starts.

Default workload: C = A*A with A the scale-20 R-MAT matrix (2^20 rows,
a=.57, b=c=.19, d=.05, 16 draws per row, duplicates merged, f64 values
uniform in [-1, 1), int32 indices, int64 row pointers for C), the R-MAT
workload of Section 4.2 / Table 3.

The JSON line carries:
  value        GFLOP/s = 2 * intermediate products / time per step
  roofline     the dominant kernel's algorithmic bytes per launch over its
               event-timed duration, against the 8 TB/s HBM peak
  ideal_volume the paper's ideal data volume (Eqs. 8-9) over the step time
  cpu_baseline the CPU oracle timed on a bounded sample of the same rows
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpGEMM GFLOP/s + % HBM roofline; batched/served vs per-call, p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def src_digest() -> str:
    h = hashlib.sha1()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2501_07056_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:12]


def workload(name: str, mer_d: int = 1024):
    import workloads as wl
    if name.startswith("mer"):
        lg = int(name[3:])
        A, B = wl.massive_er(lg, d=mer_d)
        return A, B, {"workload": f"uniform random, C = A*B with 4096 rows and 2^{lg} columns, "
                                  f"{mer_d} per row of A and of every referenced row of B",
                      "n": A.nrows, "m_C": 1 << lg, "d": mer_d, "values": "f32 uniform [-1,1)",
                      "index": f"{np.dtype(B.col.dtype).name} col, int64 rowptr",
                      "c_rowptr": "int64"}
    if name == "rmat20":
        A, B = wl.config2(20)
        return A, B, {"workload": "R-MAT scale 20, C = A*A", "n": A.nrows, "edge_factor": 16,
                      "rmat_abcd": [0.57, 0.19, 0.19, 0.05], "values": "f64 uniform [-1,1)",
                      "index": "int32", "c_rowptr": "int64"}
    if name.startswith("rmat"):
        sc = int(name[4:])
        A, B = wl.config2(sc)
        return A, B, {"workload": f"R-MAT scale {sc}, C = A*A", "n": A.nrows, "index": "int32",
                      "values": "f64", "c_rowptr": "int64"}
    if name.startswith("er"):
        lg = int(name[2:])
        A, B = wl.config3(lg)
        return A, B, {"workload": f"Erdos-Renyi 2^{lg} x 2^{lg}, 16 per row, C = A*B",
                      "n": A.nrows, "values": "f32 uniform [-1,1)", "index": "int32 col, int64 rowptr",
                      "c_rowptr": "int64"}
    if name == "cfg1":
        A, B = wl.config1()
        return A, B, {"workload": "Erdos-Renyi 4096 x 4096, 8 per row, integer f64, C = A*A",
                      "n": A.nrows, "index": "int32", "c_rowptr": "int64"}
    raise SystemExit(f"unknown workload {name}")


def ideal_volume(A, B, ip, nnz_c, c_rp_bytes=8):
    # Eqs. 8-9 with each array's own width
    import oracle
    r, w = oracle.ideal_volume(A.nrows, A.nnz, ip, A.nrows, nnz_c,
                               s_rp_a=A.rowptr.dtype.itemsize, s_rp_b=B.rowptr.dtype.itemsize,
                               s_col_a=A.col.dtype.itemsize, s_col_b=B.col.dtype.itemsize,
                               s_val=A.val.dtype.itemsize, s_rp_c=c_rp_bytes,
                               s_col_c=B.col.dtype.itemsize)
    return r + w


def stored_traffic(kernel: str, wl_name: str):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter
    summaries, if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{wl_name}.md")
    if not os.path.exists(path):
        return None, None
    for line in open(path):
        if line.startswith("traffic-json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("src_sha") != src_digest():
                return None, "stale"
            k = d.get("kernels", {}).get(kernel)
            if k is None:
                return None, "absent"
            return float(k["bytes_per_launch"]), d.get("note")
    return None, None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def config1_oracle_times():
    """The oracle on the whole of config 1 (C = A*A, 4096 x 4096, 8 per row):
    one thread and all the process's cores, the mean of 10 runs after one."""
    import oracle
    import workloads as wl
    A, _ = wl.config1()
    cores = len(os.sched_getaffinity(0))
    out = {}
    for name, nt in (("one_thread", 1), ("all_cores", cores)):
        oracle.spgemm(A, A, nthreads=nt)
        t0 = time.perf_counter()
        for _ in range(10):
            oracle.spgemm(A, A, nthreads=nt)
        out[name + "_us"] = round((time.perf_counter() - t0) / 10 * 1e6, 1)
    out["cores"] = cores
    return out


def cpu_baseline(A, B, ip_rows, seconds: float, seed: int = 7):
    """Oracle rate on rows drawn with probability proportional to their
    intermediate-product count (so the sample has the workload's mix)."""
    import numpy as np

    import oracle
    cores = len(os.sched_getaffinity(0))
    cum = np.cumsum(ip_rows.astype(np.float64))
    total = cum[-1]
    rng = np.random.default_rng(seed)

    def pick(budget):
        rows, got = set(), 0
        while got < budget and len(rows) < len(ip_rows):
            r = int(np.searchsorted(cum, rng.random() * total, side="right"))
            r = min(r, len(ip_rows) - 1)
            if r not in rows and ip_rows[r] > 0:
                rows.add(r)
                got += int(ip_rows[r])
        return np.array(sorted(rows), dtype=np.int64)

    # grow a calibration sample until it runs for a tenth of the budget, then
    # size the measured sample for about `seconds`
    budget, rate = 4e6, None
    while True:
        cal = pick(budget)
        t0 = time.perf_counter()
        oracle.spgemm(A, B, cal, nthreads=cores)
        dt = time.perf_counter() - t0
        rate = max(1.0, ip_rows[cal].sum() / max(1e-6, dt))
        if dt >= 0.1 * seconds or budget >= 0.25 * total:
            break
        budget *= 4
    # a larger sample spreads over the threads better and runs faster than the
    # calibration predicted: re-size it from the measured rate (at most twice)
    for _ in range(3):
        rows = pick(min(rate * seconds, 0.5 * total))
        t0 = time.perf_counter()
        ref = oracle.spgemm(A, B, rows, nthreads=cores)
        dt = time.perf_counter() - t0
        ipw = int(ip_rows[rows].sum())
        if dt >= 0.6 * seconds or ipw >= 0.5 * total - 1:
            break
        rate = max(1.0, ipw / max(1e-6, dt))
    res = {"value": 2.0 * ipw / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"{len(rows)} rows drawn with probability proportional to their "
                     f"intermediate products ({ipw} products, {dt:.1f} s)",
           "seconds": dt, "cpu_model": cpu_model()}
    return res, rows, ref


# library profile names -> kernel symbols they launch (a symbol matches when
# it contains every string of one of the tuples)
KERNEL_SYMBOLS = {
    "bin_scatter (numeric reorder)": [("k_bin_scatter2<", "unsigned short, true")],
    "bin_accum (numeric, dense+sort chunks)": [("k_accum_dense<", "true>"),
                                               ("k_accum_sort<", "true, false>")],
    "bin_scatter_det (ordered reorder)": [("k_bin_scatter_det<",)],
    "det_counts (symbolic, segment chunks)": [("k_det_seg_hist<",)],
    "bin_accum_det (ordered dense+sort)": [("k_accum_dense_det<",),
                                           ("k_accum_sort<", "true, true>")],
    "row_bitmap (symbolic, chunked rows)": [("k_row_bitmap<",)],
    "sort_rows (numeric)": [("k_sort_rows<",)],
    "rowinfo (setup)": [("k_rowinfo<",)],
    "coarse_scatter (numeric, level 1)": [("k_bin_scatter2<", "unsigned int, true")],
    "fine_scatter (numeric, level 2)": [("k_l2_scatter<", "true>")],
    "coarse_reorder (symbolic, level 1)": [("k_bin_hist<",),
                                           ("k_bin_scatter2<", "unsigned int, false")],
    "coarse_reorder (symbolic, L1, values)": [("k_bin_hist<",),
                                                   ("k_bin_scatter2<", "unsigned int, true")],
    "coarse_sort (symbolic, small chunks)": [("k_vrow_sort<", "false>")],
    "coarse_sort (numeric, small chunks)": [("k_vrow_sort<", "true>")],
    "coarse_bitmap (symbolic, level 2)": [("k_vrow_bitmap",)],
    "coarse_count (symbolic, level 2)": [("k_l2_hist<",), ("k_l2_scatter<", "false>")],
    "run_bin (symbolic, runs per chunk)": [("k_run_rows<",)],
    "run_count (symbolic, chunks from runs)": [("k_run_dense<", "false>"),
                                               ("k_run_sort<", "false>")],
    "run_accum (numeric, chunks from runs)": [("k_run_dense<", "true>"),
                                                         ("k_run_sort<", "true>")],
}

# gfx950 (MI355X) unit counts used by the counter-derived figures
N_XCD, N_CU, N_SIMD = 8, 256, 1024


def _match(name, pats):
    return any(all(p in name for p in tup) for tup in pats)


def _counter_rows(d):
    """(dispatch id, kernel name, counter, value) of every counter sample
    under d, from rocprofv3's CSV output or its rocpd SQLite database."""
    import csv
    import sqlite3
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            yield r["Dispatch_Id"], r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])
    for f in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
        con = sqlite3.connect(f)
        q = "select dispatch_id, kernel_name, counter_name, value from counters_collection"
        for did, kn, cn, v in con.execute(q):
            yield str(did), kn, cn, float(v)
        con.close()


def _pmc_totals(d, counter):
    tot = {}
    for did, name, cn, v in _counter_rows(d):
        if cn != counter:
            continue
        t = tot.setdefault(name, [0.0, set()])
        t[0] += v
        t[1].add(did)
    return {k: (v[0], len(v[1])) for k, v in tot.items()}


SQ_PASSES = (
    "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY SQ_INSTS_VALU SQ_INSTS_LDS "
    "SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_LDS GRBM_GUI_ACTIVE",
    "SQ_ACTIVE_INST_VALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SALU SQ_WAIT_ANY "
    "SQ_ACTIVE_INST_ANY SQ_INSTS_BRANCH SQ_INST_CYCLES_VMEM GRBM_GUI_ACTIVE",
)


def sq_summary(args):
    """Occupancy, waits, VALU and LDS figures per library kernel from two
    rocprofv3 --pmc runs of one bench step (SQ_PASSES), written to
    profiles/counters_<workload>.md."""
    per = {}   # kernel (name with template arguments) -> counter -> dispatch -> value
    wanted = [p for pats in KERNEL_SYMBOLS.values() for p in pats]
    for di, d in enumerate(args.sq_summary):
        for did0, name, cn, v in _counter_rows(d):
            did = (di, did0)  # dispatch ids restart in every run
            if not _match(name, wanted):
                continue
            key = name.split("(")[0].replace("void ", "").replace("mg::", "").strip()
            per.setdefault(key, {}).setdefault(cn, {}).setdefault(did, 0.0)
            per[key][cn][did] += v
    # the sources the profiled run was built from: its bench line's digest
    sha = src_digest()
    logf = args.sq_summary[0].rstrip("/") + ".log"
    if os.path.exists(logf):
        for line in open(logf):
            if line.startswith("{") and '"src_sha"' in line:
                sha = json.loads(line)["src_sha"]
    rows, js = [], {}
    for lib_name, cs in per.items():
        def tot(c):
            return sum(cs.get(c, {}).values())
        # GRBM_GUI_ACTIVE counts every XCD's busy cycles: one XCD's share is
        # the kernel's cycles; wave cycles and VALU-active cycles count in
        # units of 4 cycles
        launches = max(len(cs.get("SQ_WAVES", {})), 1)
        grbm_a = sum(v for k, v in cs.get("GRBM_GUI_ACTIVE", {}).items()
                     if k in cs.get("SQ_WAVES", {}))
        grbm_b = sum(v for k, v in cs.get("GRBM_GUI_ACTIVE", {}).items()
                     if k in cs.get("SQ_WAIT_ANY", {}))
        cyc_a, cyc_b = grbm_a / N_XCD, grbm_b / N_XCD
        if cyc_a <= 0 or cyc_b <= 0:
            continue
        waves = tot("SQ_WAVES")
        occ = 4.0 * tot("SQ_WAVE_CYCLES") / (cyc_a * N_CU)
        wait = tot("SQ_WAIT_ANY") / max(1.0, tot("SQ_WAVE_CYCLES") * cyc_b / cyc_a)
        valu_busy = 4.0 * tot("SQ_ACTIVE_INST_VALU") / (cyc_b * N_SIMD)
        bank = tot("SQ_LDS_BANK_CONFLICT") / (cyc_a * N_CU)
        d = {"launches": launches, "waves_per_launch": waves / launches,
             "mean_waves_per_cu": occ, "wait_frac": wait, "valu_busy": valu_busy,
             "lds_bank_conflict_frac": bank,
             "valu_per_wave": tot("SQ_INSTS_VALU") / max(waves, 1),
             "lds_per_wave": tot("SQ_INSTS_LDS") / max(waves, 1),
             "vmem_rd_per_wave": tot("SQ_INSTS_VMEM_RD") / max(waves, 1) * cyc_a / cyc_b,
             "vmem_wr_per_wave": tot("SQ_INSTS_VMEM_WR") / max(waves, 1) * cyc_a / cyc_b,
             "kernel_ms_per_launch": cyc_a / launches / 2.4e6}
        js[lib_name] = d
        if d["kernel_ms_per_launch"] * launches < 0.5:
            continue  # sub-millisecond kernels: figures dominated by launch edges
        rows.append(f"| {lib_name} | {launches} | {d['kernel_ms_per_launch']:.2f} | "
                    f"{d['waves_per_launch']:.4g} | {occ:.1f} | {100 * wait:.0f}% | "
                    f"{100 * valu_busy:.1f}% | {100 * bank:.1f}% | {d['valu_per_wave']:.4g} | "
                    f"{d['lds_per_wave']:.4g} |")
    out = os.path.join(ROOT, "profiles", f"counters_{args.workload}.md")
    cmd = f"python bench.py --workload {args.workload} --steps 1 --warmup 0 --no-cpu"
    with open(out, "w") as fh:
        fh.write(f"# SQ counters per kernel, workload {args.workload}\n\n")
        fh.write("Two counter runs of one bench step (each its own process):\n\n")
        for i, ps in enumerate(SQ_PASSES):
            fh.write(f"- `rocprofv3 --pmc {ps} -d <dir{i}> -o run -- {cmd}`\n")
        fh.write(f"\nthen `python bench.py --workload {args.workload} --sq-summary <dir0> <dir1>`.\n\n")
        fh.write("Definitions (gfx950: 8 XCDs, 256 CUs, 1024 SIMDs; GRBM_GUI_ACTIVE sums the busy "
                 "cycles of every XCD, so one XCD's share is the kernel's cycles T; "
                 "SQ_WAVE_CYCLES and SQ_ACTIVE_INST_VALU count units of 4 cycles):\n\n"
                 "- waves/CU = 4 * SQ_WAVE_CYCLES / (T * 256), the mean resident waves per CU;\n"
                 "- wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES, the share of wave time spent waiting;\n"
                 "- VALU busy = 4 * SQ_ACTIVE_INST_VALU / (T * 1024);\n"
                 "- LDS bank conflicts = SQ_LDS_BANK_CONFLICT / (T * 256), the share of each "
                 "CU's cycles its LDS spent on bank conflicts;\n"
                 "- VALU and LDS instructions per wave = SQ_INSTS_* / SQ_WAVES.\n\n")
        fh.write(f"Sources of the profiled run: `src_sha {sha}` (the bench line's digest).\n\n")
        fh.write("| kernel | launches | ms/launch (T) | waves/launch | waves/CU | wait | VALU busy "
                 "| LDS bank conflicts | VALU instr/wave | LDS instr/wave |\n"
                 "|---|---|---|---|---|---|---|---|---|---|\n")
        fh.write("\n".join(rows) + "\n\n(Kernels under 0.5 ms in total are in the JSON line only.)\n\n")
        fh.write("counters-json:" + json.dumps({"src_sha": sha, "kernels": js}) + "\n")
    log(f"[bench] wrote {out}")


def pmc_summary(args):
    fetch_d, write_d, cf_d, cw_d = args.pmc_summary
    fetch, write = _pmc_totals(fetch_d, "FETCH_SIZE"), _pmc_totals(write_d, "WRITE_SIZE")
    cfe, cwr = _pmc_totals(cf_d, "FETCH_SIZE"), _pmc_totals(cw_d, "WRITE_SIZE")
    ck = [k for k in cfe if "k_stream_copy" in k]
    cw = [k for k in cwr if "k_stream_copy" in k]
    f_fetch = args.copy_bytes * cfe[ck[0]][1] / (cfe[ck[0]][0] * 1024.0)
    f_write = args.copy_bytes * cwr[cw[0]][1] / (cwr[cw[0]][0] * 1024.0)
    kernels = {}
    lines = []
    # only the library kernels the profiled run reported (several names map
    # to the same kernel symbols in different modes)
    seen = None
    if args.pmc_names:
        d = json.loads(open(args.pmc_names).read().strip().splitlines()[-1])
        seen = {k["name"] for k in d.get("kernels", [])}
    for lib_name, pats in KERNEL_SYMBOLS.items():
        if seen is not None and lib_name not in seen:
            continue
        fk = sum(v[0] for k, v in fetch.items() if _match(k, pats))
        wk = sum(v[0] for k, v in write.items() if _match(k, pats))
        # dispatches of the first matching symbol = launches of the grouped kernel
        nd = max([v[1] for k, v in fetch.items() if _match(k, pats[:1])] or [0])
        if nd == 0:
            continue
        b = (fk * f_fetch + wk * f_write) * 1024.0 / nd
        kernels[lib_name] = {"bytes_per_launch": b, "fetch_kib_per_launch": fk / nd,
                             "write_kib_per_launch": wk / nd, "launches": nd}
        lines.append(f"| {lib_name} | {nd} | {fk / nd:.4g} | {wk / nd:.4g} | {b / 1e9:.3f} |")
    d = {"src_sha": src_digest(), "copy_factor_fetch": f_fetch, "copy_factor_write": f_write,
         "kernels": kernels,
         "note": "FETCH_SIZE / WRITE_SIZE KiB per dispatch scaled by the plain copy kernel's factors"}
    out = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.md")
    with open(out, "w") as fh:
        fh.write(f"# HBM traffic per launch, workload {args.workload}\n\n")
        fh.write("Counters: `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` (separate runs) of\n"
                 f"`python bench.py --workload {args.workload} --steps 1 --warmup 0 --no-cpu`, and of\n"
                 f"`python bench.py --copy-probe {args.copy_bytes}` for the scale factors\n"
                 f"(copy of {args.copy_bytes} bytes: fetch factor {f_fetch:.4f}, write factor {f_write:.4f}).\n\n")
        fh.write("| kernel | launches | FETCH KiB/launch | WRITE KiB/launch | scaled GB/launch |\n|---|---|---|---|---|\n")
        fh.write("\n".join(lines) + "\n\n")
        fh.write("traffic-json:" + json.dumps(d) + "\n")
    log(f"[bench] wrote {out}")


def trace_summary(args):
    import csv
    files = glob.glob(os.path.join(args.trace_summary, "**", "*kernel_stats.csv"), recursive=True)
    rows = list(csv.DictReader(open(files[0])))
    out = os.path.join(ROOT, "profiles", f"kernels_{args.workload}.md")
    with open(out, "w") as fh:
        fh.write(f"# Kernel time, workload {args.workload}\n\n")
        fh.write(f"Command: `{args.trace_command}`\n\n")
        fh.write("| kernel | calls | total ms | average us | % |\n|---|---|---|---|---|\n")
        for r in rows[:25]:
            name = r["Name"].replace("|", "/")
            if len(name) > 90:
                name = name[:90] + "..."
            fh.write(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |\n")
    log(f"[bench] wrote {out}")


def batch_main(args, opts):
    """Batched products (512 independent C_b = A_b * A_b, A_b Erdos-Renyi with
    n log-uniform in [1024, 65536] and 4..32 entries per row, f32 values,
    int32 indices): one batch per step against the same products called one
    at a time through the single-product calls, both timed with the whole
    plan + execute; then the numeric phase alone, replayed from a kept plan
    (captured graph vs the same launches issued eagerly vs per-call)."""
    import numpy as np
    import torch

    import oracle
    import paper_2501_07056_amd as mg
    from paper_2501_07056_amd import autotune
    import workloads as wl

    t0 = time.time()
    count = args.batch_count
    pairs_host = wl.config4(count)
    log(f"[bench] batch of {count} generated in {time.time() - t0:.1f} s, "
        f"nnz(A) total {sum(A.nnz for A, _ in pairs_host)}")
    pairs = []
    for A, _ in pairs_host:
        dA = mg.DeviceCSR.from_host(A)
        pairs.append((dA, dA))
    ctx = mg.Context(0, **opts)
    torch.cuda.synchronize()

    tuned = None
    if not args.no_tune:
        tuned = autotune.tune(ctx, pairs, cache_path=args.tune_cache, log=log)
        ctx.set_options(dense_block=tuned["dense_block"], chunk_shift=tuned["chunk_shift"],
                        bin_dense_min=tuned["bin_dense_min"],
                        sort_group_max=tuned["sort_group_max"])
    sort_max = tuned["sort_max"] if tuned else None

    def batched_step(graph=True):
        bp = ctx.batch_plan(pairs, sort_max=sort_max)
        outs = bp.execute(graph=graph)
        info = bp.info.as_dict()
        bp.destroy()
        return outs, info

    def per_call_step():
        # one magnus_spgemm call per product (plan with its readbacks, C from
        # the allocator, execute), C freed after the step
        outs = []
        for b, (dA, dB) in enumerate(pairs):
            if sort_max is not None:
                ctx.set_options(sort_max=sort_max[b])
            outs.append(ctx.spgemm_lib(dA, dB, rowptr_dtype=torch.int64))
        return outs

    def timed(fn, steps, warmup):
        res = None
        for _ in range(warmup):
            res = fn()
            del res
            torch.cuda.synchronize()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            res = fn()
            if i + 1 < steps:
                del res
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / steps, res

    ms_b, (outs, info) = timed(batched_step, args.steps, args.warmup)
    ip = int(info["ip_total"])
    log(f"[bench] batched: {ms_b:.2f} ms/step, {2 * ip / ms_b / 1e6:.1f} GFLOP/s")
    del outs
    ms_p, outs_p = timed(per_call_step, args.steps, args.warmup)
    ctx.set_options(sort_max=0)
    log(f"[bench] per-call: {ms_p:.2f} ms/step, {2 * ip / ms_p / 1e6:.1f} GFLOP/s")
    del outs_p

    # numeric phase only, replayed from a kept plan
    bp = ctx.batch_plan(pairs, sort_max=sort_max)
    outs = bp.alloc_outputs()
    bp.execute(outs, graph=True)
    torch.cuda.synchronize()
    ms_graph, _ = timed(lambda: bp.execute(outs, graph=True), args.steps, 1)
    ms_eager, _ = timed(lambda: bp.execute(outs, graph=False), args.steps, 1)
    bp.execute(outs, graph=True, persistent=True)
    torch.cuda.synchronize()
    ms_graph_p, _ = timed(lambda: bp.execute(outs, graph=True, persistent=True), args.steps, 1)
    plans = []
    for b, (dA, dB) in enumerate(pairs):
        if sort_max is not None:
            ctx.set_options(sort_max=sort_max[b])
        plans.append(ctx.plan(dA, dB))
    ctx.set_options(sort_max=0)
    single_outs = [p.alloc_output() for p in plans]

    def per_call_exec():
        for p, C in zip(plans, single_outs):
            p.execute(C)
    ms_pexec, _ = timed(per_call_exec, args.steps, 1)
    for p in plans:
        p.destroy()
    log(f"[bench] numeric only: graph {ms_graph:.2f} ms, eager {ms_eager:.2f} ms, "
        f"graph with persistent stages {ms_graph_p:.2f} ms, per-call {ms_pexec:.2f} ms")

    # sampled parity of the kept batch outputs against the oracle
    rng = np.random.default_rng(11)
    checked, worst, ok = 0, 0.0, True
    for b in range(0, count, max(1, count // 16)):
        A = pairs_host[b][0]
        rows = np.sort(rng.choice(A.nrows, size=min(64, A.nrows), replace=False)).astype(np.int64)
        ref = oracle.spgemm(A, A, rows)
        rp, col, val = outs[b].to_host()
        gl = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
        ok &= bool(np.array_equal(col[gl].astype(np.int64), ref.col) and
                   np.array_equal(np.diff(ref.rowptr), rp[rows + 1] - rp[rows]))
        err = np.abs(val[gl].astype(np.float64) - ref.ref) / np.maximum(ref.abssum, 1e-300)
        worst = max(worst, float(err.max()) if len(err) else 0.0)
        checked += len(rows)
    bp.destroy()
    parity = {"rows": checked, "structure_equal": ok, "max_err_over_abssum": worst,
              "within_rtol": bool(ok and worst <= 1e-5), "rtol": 1e-5}
    log(f"[bench] sampled parity {parity}")

    gf = lambda ms: round(2 * ip / ms / 1e6, 2)  # noqa: E731
    cfg = {"workload": f"{count} independent C = A*A, A Erdos-Renyi, n log-uniform in "
                       f"[1024, 65536], 4..32 per row, f32, int32",
           "products": count, "rows": int(sum(A.nrows for A, _ in pairs_host)),
           "intermediate_products": ip, "nnz_C": int(info["nnz_c"]),
           "categories_rows": info["rows_by_category"],
           "autotuned": tuned is not None,
           "dense_block": tuned["dense_block"] if tuned else None,
           "sort_max_histogram": ({str(k): int(v) for k, v in
                                   zip(*np.unique(sort_max, return_counts=True))} if tuned else None)}
    out = {"metric": METRIC, "value": gf(ms_b), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_b, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": cfg,
           "per_call": {"ms_per_step": round(ms_p, 3), "GFLOPs": gf(ms_p),
                        "batched_speedup": round(ms_p / ms_b, 3)},
           "numeric_only": {"graph_ms": round(ms_graph, 3), "eager_ms": round(ms_eager, 3),
                            "graph_persistent_ms": round(ms_graph_p, 3),
                            "per_call_ms": round(ms_pexec, 3), "graph_GFLOPs": gf(ms_graph),
                            "per_call_GFLOPs": gf(ms_pexec)},
           "sample_parity": parity, "src_sha": src_digest()}
    print(json.dumps(out), flush=True)


def serve_main(args, opts):
    """Serving: a Poisson stream of C = A*B requests (n log-uniform in
    [1e3, 1e6]; half R-MAT with scale round(log2 n), the operands of one
    scale shared, A and B independent; half banded with bandwidth 64 and 9
    entries per row, each request its own; f64 values, int32 indices).  The
    serial saturation rate is measured first (all requests back to back, one
    call at a time); then, at each fraction of it (--qps-fracs), the stream
    is replayed against (1) the server (admission by memory bound, batching,
    overlapped groups) and (2) one call at a time in arrival order.  Latency
    is arrival to C complete on the device.  The first served run checks
    every scale-20 request and every 8th other one against the oracle on
    sampled rows."""
    import torch

    import oracle
    import paper_2501_07056_amd as mg
    import workloads as wl

    reqs = wl.config5_requests(args.serve_count, 1.0)  # arrival times at rate 1, scaled per run
    t0 = time.time()
    host = {}

    def operand(r, which):
        if r.kind == "rmat":
            sc = int(round(math.log2(r.n)))
            key = ("rmat", sc, which)
            if key not in host:
                host[key] = wl.config5_operand("rmat", r.n, wl.seed(7000 + 2 * sc + (which == "B")))
        else:
            key = ("banded", r.rid, which)
            host[key] = wl.config5_operand("banded", r.n, r.a_seed if which == "A" else r.b_seed)
        return key

    keys = [(operand(r, "A"), operand(r, "B")) for r in reqs]
    log(f"[bench] {len(reqs)} requests, {len(host)} operands generated in {time.time() - t0:.1f} s")
    dev = {k: mg.DeviceCSR.from_host(X) for k, X in host.items()}
    torch.cuda.synchronize()
    ctx = mg.Context(0, **opts)
    ips = []
    for ka, kb in keys:
        ip, _ = ctx.batch_bound([(dev[ka], dev[kb])])
        ips.append(ip[0])
    total_flop = 2.0 * sum(ips)
    scale20 = [j for j, r in enumerate(reqs) if r.kind == "rmat" and r.n == 1 << 20]
    check_ids = set(scale20) | {j for j in range(0, len(reqs), 8)}

    def pct(v, q):
        return float(np.percentile(np.array(v), q)) if v else None

    # serial saturation: every request back to back, one call at a time
    t_start = time.perf_counter()
    last_note = 0.0
    for j in range(len(reqs)):
        if time.perf_counter() - t_start - last_note >= 2.0:
            last_note = time.perf_counter() - t_start
            log(f"[bench] saturation t={last_note:.1f} s: request {j}")
        ka, kb = keys[j]
        C = ctx.spgemm(dev[ka], dev[kb])
        torch.cuda.synchronize()
        del C
    sat_s = time.perf_counter() - t_start
    sat_rate = len(reqs) / sat_s
    log(f"[bench] serial saturation: {len(reqs)} requests in {sat_s:.2f} s = {sat_rate:.2f} req/s, "
        f"{total_flop / sat_s / 1e9:.2f} GFLOP/s")

    def sampled_check(j, srv, rid):
        """Sampled rows of a served C against the oracle (only those rows
        are copied to the host)."""
        A, B = host[keys[j][0]], host[keys[j][1]]
        rows = np.sort(np.random.default_rng(j).choice(A.nrows, min(200, A.nrows),
                                                       replace=False)).astype(np.int64)
        rp, col, val = srv.result_rows(rid, rows)
        rp = rp.astype(np.int64)
        col = col.astype(np.int64)
        val = val.astype(np.float64)
        ref = oracle.spgemm(A, B, rows)
        ok = bool(np.array_equal(col, ref.col) and
                  np.array_equal(np.diff(ref.rowptr), rp[rows + 1] - rp[rows]))
        err = np.abs(val - ref.ref) / np.maximum(ref.abssum, 1e-300)
        return ok and bool((err <= 1e-12).all())

    def served(qps, check):
        # the server's budget: most of the memory the cached blocks of the
        # one-at-a-time runs leave free
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free, _ = torch.cuda.mem_get_info()
        srv = mg.Server(0, options=opts, max_batch=args.max_batch, streams=args.streams,
                        memory_budget_bytes=int(0.9 * free))
        ids = {k: srv.register(X) for k, X in dev.items()}
        lat, qms, bsz, states, parity = {}, {}, {}, {}, {}
        outstanding = {}
        t_start = time.perf_counter()
        i = 0
        last_note, last_progress, n_done = 0.0, 0.0, 0
        while i < len(reqs) or outstanding:
            now = time.perf_counter() - t_start
            if now - last_note >= 2.0:
                log(f"[bench] served {qps:.1f}/s t={now:.1f} s: submitted {i}, finished {n_done}, "
                    f"outstanding {len(outstanding)}, reserved "
                    f"{srv.stats()['reserved_bytes'] / 1e9:.1f} GB")
                last_note = now
            if outstanding and now - last_progress > 90.0:
                st = srv.stats()
                states = {rid: srv.query(rid)["state"] for rid in list(outstanding)[:20]}
                log(f"[bench] no request finished for 90 s; stats {st}; states {states}")
                sys.stdout.flush()
                os._exit(3)
            while i < len(reqs) and reqs[i].arrival_s / qps <= now:
                ka, kb = keys[i]
                outstanding[srv.submit(ids[ka], ids[kb])] = i
                i += 1
            for rid in list(outstanding):
                if not srv.ready(rid):
                    continue
                j = outstanding.pop(rid)
                n_done += 1
                last_progress = time.perf_counter() - t_start
                info = srv.query(rid)
                states[j] = info["state"]
                if info["state"] == "failed":
                    log(f"[bench] request {j} ({reqs[j].kind}, n {reqs[j].n}) failed: {info}")
                if info["state"] == "done":
                    lat[j], qms[j], bsz[j] = info["latency_ms"], info["queue_ms"], info["batch_size"]
                    if check and j in check_ids:
                        parity[j] = sampled_check(j, srv, rid)
                srv.release(rid)
            time.sleep(0.0005)
        secs = time.perf_counter() - t_start
        st = srv.stats()
        srv.close()
        torch.cuda.synchronize()
        flop = 2.0 * sum(ips[j] for j in lat)
        log(f"[bench] served {qps:.1f}/s: {secs:.2f} s, p50 {pct(list(lat.values()), 50):.1f} ms, "
            f"p99 {pct(list(lat.values()), 99):.1f} ms, stats {st}")
        for j in sorted(lat, key=lambda j: -lat[j])[:6]:
            log(f"[bench]   slowest: request {j} {reqs[j].kind} n {reqs[j].n} arrival "
                f"{reqs[j].arrival_s / qps:.2f} s queue {qms[j]:.0f} ms latency {lat[j]:.0f} ms "
                f"group {bsz[j]}")
        return {"seconds": round(secs, 3), "req_per_s": round(len(lat) / secs, 2),
                "GFLOPs": round(flop / secs / 1e9, 2),
                "p50_ms": pct(list(lat.values()), 50), "p99_ms": pct(list(lat.values()), 99),
                "mean_queue_ms": float(np.mean(list(qms.values()))) if qms else None,
                "mean_batch": float(np.mean(list(bsz.values()))) if bsz else None,
                "completed": len(lat), "rejected": sum(v == "rejected" for v in states.values()),
                "failed": sum(v == "failed" for v in states.values()),
                "peak_reserved_GB": round(st["peak_reserved_bytes"] / 1e9, 2),
                "budget_GB": round(st["budget_bytes"] / 1e9, 2), "deferred": st["deferred"],
                "exact_probes": st["exact_probes"]}, parity

    def serial(qps):
        lat1 = {}
        t_start = time.perf_counter()
        last_note = 0.0
        for j, r in enumerate(reqs):
            if time.perf_counter() - t_start - last_note >= 2.0:
                last_note = time.perf_counter() - t_start
                log(f"[bench] serial {qps:.1f}/s t={last_note:.1f} s: request {j}")
            while time.perf_counter() - t_start < r.arrival_s / qps:
                time.sleep(0.0002)
            ka, kb = keys[j]
            try:
                C = ctx.spgemm(dev[ka], dev[kb])
                torch.cuda.synchronize()
                lat1[j] = 1e3 * (time.perf_counter() - t_start - r.arrival_s / qps)
                del C
            except mg.MagnusError as e:
                log(f"[bench] serial request {j} failed: {e}")
        secs = time.perf_counter() - t_start
        log(f"[bench] serial {qps:.1f}/s: {secs:.2f} s, p50 {pct(list(lat1.values()), 50):.1f} ms, "
            f"p99 {pct(list(lat1.values()), 99):.1f} ms")
        return {"seconds": round(secs, 3), "req_per_s": round(len(lat1) / secs, 2),
                "GFLOPs": round(2.0 * sum(ips[j] for j in lat1) / secs / 1e9, 2),
                "p50_ms": pct(list(lat1.values()), 50), "p99_ms": pct(list(lat1.values()), 99),
                "completed": len(lat1)}

    fracs = [float(x) for x in args.qps_fracs.split(",")] if args.qps <= 0 else [None]
    runs, parity = [], {}
    for k, f in enumerate(fracs):
        qps = args.qps if f is None else f * sat_rate
        sv, par = served(qps, check=(k == 0))
        parity.update(par)
        runs.append({"fraction_of_saturation": f, "qps": round(qps, 3), "served": sv,
                     "serial_fifo": serial(qps)})
    head = runs[-1]
    bad = sorted(j for j, ok in parity.items() if not ok)
    out = {"metric": METRIC, "value": head["served"]["GFLOPs"], "unit": "GFLOP/s",
           "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * head["served"]["seconds"], 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"{len(reqs)} Poisson requests, C = A*B, n log-uniform in "
                                  "[1e3, 1e6], half R-MAT (scale round(log2 n), operands shared "
                                  "per scale), half banded (w 64, 9 per row), f64, int32; served "
                                  "at fractions of the serial saturation rate",
                      "requests": len(reqs), "operands": len(host),
                      "scale20_requests": len(scale20),
                      "intermediate_products": int(sum(ips)), "max_batch": args.max_batch,
                      "streams": args.streams},
           "serial_saturation": {"seconds": round(sat_s, 3), "req_per_s": round(sat_rate, 3),
                                 "GFLOPs": round(total_flop / sat_s / 1e9, 2)},
           "runs": runs,
           "sample_parity": {"requests": len(parity), "scale20_checked": sum(j in parity for j in scale20),
                             "all_within_rtol": not bad, "failed_requests": bad[:20], "rtol": 1e-12,
                             "rows_per_request": 200},
           "src_sha": src_digest()}
    print(json.dumps(out), flush=True)


def micro_main(args, opts):
    """Building blocks on one stream of products (the microbenchmarks of
    Section 4.1, Figs. 5-6): L products with columns uniform in [0, m) and
    f32 values, cut into m / 2^s chunks by histogram, prefix sum and reorder,
    then each chunk counted and summed; every stage is event-timed.  The
    reference is the streaming time of the paper: a plain copy of the
    stream's bytes (columns and values read and written once) with the
    library's copy kernel."""
    import torch

    import paper_2501_07056_amd as mg
    ctx = mg.Context(0, **opts)
    g = torch.Generator(device="cuda")
    g.manual_seed(2501070560)
    rows = []
    for lg_l in (22, 24, 26):
        L = 1 << lg_l
        vals = torch.rand(L, generator=g, device="cuda", dtype=torch.float32) * 2 - 1
        src = torch.zeros(2 * L, dtype=torch.float32, device="cuda")
        dst = torch.zeros_like(src)
        for _ in range(2):
            ctx.stream_copy(dst, src)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(3):
            ctx.stream_copy(dst, src)
        torch.cuda.synchronize()
        ck = ctx.profile_read()[0]
        ctx.profile(False)
        t_stream = ck["ms"] / ck["launches"]
        del src, dst
        for lg_m in (16, 20, 24, 26):
            m = 1 << lg_m
            cols = torch.randint(0, m, (L,), generator=g, device="cuda", dtype=torch.int32)
            for s in (10, 12, 14):
                if (m >> s) > 8191 or (m >> s) < 1:
                    continue
                best = None
                for _ in range(3):
                    _, _, t = ctx.stream_chunks(cols, vals, m, s)
                    tot = (t["histogram_ms"] + t["scan_ms"] + t["reorder_ms"] + t["group_ms"] +
                           t["count_ms"] + t["accumulate_ms"])
                    if best is None or tot < best[0]:
                        best = (tot, t)
                tot, t = best
                gb = L * 8 / 1e9  # the stream: 32-bit column and f32 value
                row = {"L": L, "m": m, "chunk_shift": s, "chunks": t["chunks"],
                       "products_per_chunk": L / t["chunks"], "dense_chunks": t["dense_chunks"],
                       "sort_groups": t["sort_groups"], "total_ms": round(tot, 3),
                       "streaming_ms": round(t_stream, 3),
                       "multiple_of_streaming": round(tot / t_stream, 2),
                       "histogram_GBps": round(L * 4 / 1e9 / (t["histogram_ms"] / 1e3), 1),
                       "reorder_GBps": round(L * (8 + 6) / 1e9 / (t["reorder_ms"] / 1e3), 1),
                       "count_GBps": round(L * 2 / 1e9 / (t["count_ms"] / 1e3), 1),
                       "accumulate_GBps": round(L * 6 / 1e9 / (t["accumulate_ms"] / 1e3), 1),
                       "stage_ms": {k: round(t[k], 3) for k in ("histogram_ms", "scan_ms",
                                                                  "reorder_ms", "group_ms",
                                                                  "count_ms", "accumulate_ms")}}
                rows.append(row)
                log(f"[bench] L=2^{lg_l} m=2^{lg_m} chunks={t['chunks']}: {tot:.2f} ms "
                    f"= {tot / t_stream:.2f}x streaming ({gb:.2f} GB stream)")
            del cols
    # accumulators against the products per chunk (Fig. 4): 4096 chunks of
    # 2^13 columns, every chunk dense (dense_min = 1) or sorted wherever it
    # holds at most 1024 products (dense_min = 1025)
    acc = []
    m = 1 << 25
    for lg_l in (19, 20, 21, 22):
        L = 1 << lg_l
        cols = torch.randint(0, m, (L,), generator=g, device="cuda", dtype=torch.int32)
        vals = torch.rand(L, generator=g, device="cuda", dtype=torch.float32)
        for dmin, kind in ((1, "dense"), (1025, "sort")):
            best = None
            for _ in range(3):
                _, _, t = ctx.stream_chunks(cols, vals, m, 13, dmin)
                tt = t["count_ms"] + t["accumulate_ms"]
                if best is None or tt < best[0]:
                    best = (tt, t)
            tt, t = best
            acc.append({"products_per_chunk": L / 4096, "accumulator": kind,
                        "dense_chunks": t["dense_chunks"], "sort_groups": t["sort_groups"],
                        "count_ms": round(t["count_ms"], 4),
                        "accumulate_ms": round(t["accumulate_ms"], 4),
                        "Gproducts_per_s": round(L / (t["accumulate_ms"] / 1e3) / 1e9, 1)})
            log(f"[bench] {L // 4096} products per chunk, {kind}: count {t['count_ms']:.3f} ms, "
                f"sum {t['accumulate_ms']:.3f} ms")
        del cols, vals
    ctx.close()
    best = min(rows, key=lambda r: r["multiple_of_streaming"])
    out = {"metric": "building blocks on one stream: time as a multiple of the streaming time",
           "value": best["multiple_of_streaming"], "unit": "x streaming", "n_gpus": 1,
           "higher_is_better": False, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "one stream of L products, columns uniform in [0, m), "
                                  "chunks of 2^s columns", "options": opts},
           "sweep": rows, "accumulators": acc, "src_sha": src_digest()}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20",
                    help="rmat<scale> | er<log n> | cfg1 | mer<log m_C> (massive uniform random, "
                         "Section 4.3) | batch | serve | micro (building blocks, Section 4.1)")
    ap.add_argument("--mer-d", type=int, default=1024,
                    help="entries per row of A and of B for --workload mer<log m_C>")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--option", action="append", default=[],
                    help="library option name=value (repeatable)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run the plain copy kernel on this many bytes (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                       "COPY_WRITE_DIR"),
                    help="turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE CSVs into profiles/traffic_<workload>.md")
    ap.add_argument("--copy-bytes", type=int, default=1 << 32)
    ap.add_argument("--pmc-names", metavar="JSON",
                    help="with --pmc-summary: the bench line of the profiled run; only the "
                         "library kernels it reports are summarised")
    ap.add_argument("--trace-summary", metavar="STATS_DIR",
                    help="turn a rocprofv3 --kernel-trace --stats CSV into profiles/kernels_<workload>.md")
    ap.add_argument("--trace-command", default="")
    ap.add_argument("--sq-summary", nargs="+", metavar="PMC_DIR",
                    help="turn the rocprofv3 --pmc runs of SQ_PASSES into "
                         "profiles/counters_<workload>.md")
    ap.add_argument("--batch-count", type=int, default=512,
                    help="products of the batch workload (--workload batch)")
    ap.add_argument("--no-tune", action="store_true", help="batch workload: library defaults")
    ap.add_argument("--serve-count", type=int, default=2000, help="requests of --workload serve")
    ap.add_argument("--qps", type=float, default=0.0,
                    help="arrival rate of --workload serve (0: fractions of the measured serial "
                         "saturation rate, --qps-fracs)")
    ap.add_argument("--qps-fracs", default="0.5,0.8,0.95",
                    help="fractions of the serial saturation rate for --workload serve")
    ap.add_argument("--max-batch", type=int, default=32)
    ap.add_argument("--streams", type=int, default=2)
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2501_07056_amd", "tuned",
                                                         "batch_tuning.json"))
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.trace_summary:
        trace_summary(args)
        return
    if args.sq_summary:
        sq_summary(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(this build measures a single MI355X)", file=sys.stderr)
        sys.exit(2)

    opts = {}
    for o in args.option:
        k, v = o.split("=", 1)
        opts[k] = int(v) if v.lstrip("-").isdigit() else v
    if args.workload == "batch":
        batch_main(args, opts)
        return
    if args.workload == "serve":
        serve_main(args, opts)
        return
    if args.workload == "micro":
        micro_main(args, opts)
        return

    import numpy as np
    import torch

    import paper_2501_07056_amd as mg

    t0 = time.time()
    A, B, cfg = workload(args.workload, args.mer_d)
    log(f"[bench] {cfg['workload']}: generated in {time.time() - t0:.1f} s, nnz(A)={A.nnz}")
    dA = mg.DeviceCSR.from_host(A)
    dB = dA if B is A else mg.DeviceCSR.from_host(B)
    ctx = mg.Context(0, **opts)
    torch.cuda.synchronize()
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            ctx.stream_copy(dst, src)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        ctx.stream_copy(dst, src)
        torch.cuda.synchronize()
        k = ctx.profile_read()[0]
        log(f"[bench] copy {args.copy_probe} bytes: {k['bytes'] / k['ms'] / 1e6:.1f} GB/s (events)")
        return

    def step():
        p = ctx.plan(dA, dB)
        C = p.execute(rowptr_dtype=torch.int64)
        info = p.info.as_dict()
        p.destroy()
        return C, info

    for i in range(args.warmup):
        C, info = step()
        del C
        torch.cuda.synchronize()
        log(f"[bench] warmup {i} done")

    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        C, info = step()
        if i + 1 < args.steps:
            del C
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile(False)
    kstats = ctx.profile_read()
    ms = 1e3 * elapsed / args.steps
    ip = int(info["ip_total"])
    nnz_c = int(info["nnz_c"])
    gflops = 2.0 * ip / (ms / 1e3) / 1e9
    log(f"[bench] {args.steps} steps: {ms:.2f} ms/step, {gflops:.1f} GFLOP/s")

    # dominant kernel and its roofline (algorithmic bytes / event time)
    kstats.sort(key=lambda k: -k["ms"])
    dom = kstats[0]
    ach = (dom["bytes"] / dom["launches"]) / ((dom["ms"] / dom["launches"]) / 1e3) / 1e9
    traffic, tnote = stored_traffic(dom["name"], args.workload)
    roof = {"bound": "hbm", "kernel": dom["name"], "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": dom["bytes"] / dom["launches"],
            "ms_per_launch": dom["ms"] / dom["launches"], "launches": dom["launches"]}
    vid = ideal_volume(A, B, ip, nnz_c)
    ideal = {"bytes": vid, "frac_of_peak": round(vid / (ms / 1e3) / (HBM_PEAK_GBS * 1e9), 4),
             "t_ideal_ms": vid / (HBM_PEAK_GBS * 1e9) * 1e3}
    # the paper's bound divides by a measured streaming bandwidth: time a
    # plain copy of 2 GiB with the library's copy kernel and events
    src = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        ctx.stream_copy(dst, src)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(3):
        ctx.stream_copy(dst, src)
    torch.cuda.synchronize()
    ck = ctx.profile_read()[0]
    ctx.profile(False)
    del src, dst
    copy_gbs = ck["bytes"] / ck["ms"] / 1e6
    # the whole step against the paper's ideal volume, beside the dominant
    # kernel's own figure
    roof["step_ideal_volume_frac"] = ideal["frac_of_peak"]
    ideal.update({"copy_GBps": round(copy_gbs, 1),
                  "t_ideal_copy_ms": vid / (copy_gbs * 1e9) * 1e3,
                  "multiple_of_ideal_at_copy_bw": round(ms / (vid / (copy_gbs * 1e9) * 1e3), 3)})
    log(f"[bench] ideal volume {vid / 1e9:.2f} GB: {ideal['multiple_of_ideal_at_copy_bw']}x the "
        f"bound at the measured copy rate {copy_gbs:.0f} GB/s")
    kernels = [{"name": k["name"], "ms_per_step": round(k["ms"] / args.steps, 3),
                "GBps": round(k["bytes"] / max(k["ms"], 1e-9) / 1e6, 1)} for k in kstats]

    cpu = None
    parity = None
    if not args.no_cpu:
        ipr, _ = ctx.row_ip(dA, dB)
        ipr = ipr.cpu().numpy()
        cpu, rows, ref = cpu_baseline(A, B, ipr, args.cpu_seconds)
        cpu["config1_oracle"] = config1_oracle_times()
        # the sampled rows of the last timed C against the oracle
        rp = C.rowptr.cpu().numpy()
        idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
        it = torch.from_numpy(idx).to(C.col.device)
        gcol = C.col[it].cpu().numpy().astype(np.int64)
        gval = C.val[it].cpu().numpy().astype(np.float64)
        ok_struct = bool(np.array_equal(np.diff(ref.rowptr), rp[rows + 1] - rp[rows]) and
                         np.array_equal(gcol, ref.col))
        rtol = 1e-12 if A.val.dtype == np.float64 else 1e-5
        err = np.abs(gval - ref.ref) / np.maximum(ref.abssum, 1e-300)
        parity = {"rows": int(len(rows)), "entries": int(len(gcol)), "structure_equal": ok_struct,
                  "max_err_over_abssum": float(err.max()) if len(err) else 0.0,
                  "within_rtol": bool(ok_struct and (err <= rtol).all()), "rtol": rtol,
                  # every value equal to the oracle's input-precision sum taken in
                  # the order of Eq. 1 (what the deterministic option guarantees)
                  "bits_equal_stored_order_sum": bool(ok_struct and np.array_equal(gval, ref.val))}
        log(f"[bench] cpu oracle {cpu['value']:.3f} GFLOP/s on {cpu['cores']} cores; "
            f"sample parity {parity['within_rtol']}")

    dtype = "f64" if A.val.dtype == np.float64 else "f32"
    cfg.update({"nnz_A": int(A.nnz), "intermediate_products": ip, "nnz_C": nnz_c,
                "categories_rows": info["rows_by_category"], "chunk_shift": info["chunk_shift"],
                "batches": info["n_batches"], "options": opts})
    out = {"metric": METRIC, "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": cfg, "roofline": roof, "ideal_volume": ideal,
           "kernels": kernels, "cpu_baseline": cpu, "sample_parity": parity,
           "src_sha": src_digest()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
