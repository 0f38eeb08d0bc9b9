"""Benchmark: encode + CP-ALS of the skewed 4-mode tensor on one MI355X.

Workload (synthetic, seeded, drawn on the GPU): 2,000,000 x 100,000 x 50,000 x
24, 150M distinct nonzeros, labels Zipf(1.3) on modes 0-2 and uniform on mode
3, values lognormal(0,1), rank 64, 10 CP-ALS iterations.  Before the timed
region the autotuner picks the bit layout and the per-mode plan (tile,
strategy) by measured all-mode MTTKRP time against the ALTO layout.  One step
= one whole solve from the COO tensor resident in HBM: GPU encoding with the
tuned layout (bit deposit + radix sort), the per-mode plans, then 10 CP-ALS
iterations (all-mode MTTKRP, FP64 Gram/Cholesky/solve, FP64 fit).

Printed metric: MTTKRP Gnnz/s per mode over the whole step
(nnz * modes * iterations / step time).  Extra fields: the MTTKRP calls alone
(HIP events around every call), the roofline of the MTTKRP call with measured
stream rates and a cache-aware bound, the sampled-row error of every mode
against the FP64 oracle, the ratings tensor's MTTKRP, and the oracle timed on
the host (one thread, and a process pool over the host cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
def pmc_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"mttkrp_{workload}_hbm_traffic.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest() -> str:
    """Digest of the sources of every kernel one MTTKRP call runs (main kernel,
    record sort, record reduction, plan); stored HBM counters are valid only for it."""
    h = hashlib.sha256()
    for f in ("mttkrp_seg.hip", "mttkrp_table.hip", "encode.hip", "plan.cpp", "tile_common.h"):
        with open(os.path.join(ROOT, "paper_2509_00280_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(t, rank: int, mode: int) -> int:
    """Compulsory HBM bytes of one mode-n MTTKRP: the key/value stream once (12 B per
    nonzero with 64-bit keys, 20 B with 128-bit keys), every factor row that some
    nonzero touches read once, and the output written once.  ``t`` holds its
    coordinates as a torch tensor (device) or a numpy array (host)."""
    kw = 8 if sum((int(d) - 1).bit_length() for d in t.dims) <= 64 else 16
    b = t.nnz * (kw + 4)
    for k, d in enumerate(t.dims):
        if k == mode:
            b += int(d) * rank * 4
            continue
        c = t.coords[k]
        if hasattr(c, "is_cuda"):
            import torch
            seen = torch.zeros(int(d), dtype=torch.bool, device=c.device)
            seen[c.long()] = True
            used = int(seen.sum().item())
        else:
            used = int(np.count_nonzero(np.bincount(c, minlength=d)))
        b += used * rank * 4
    return b


def host_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_POOL_DATA = {}


def _pool_job(job):
    import oracle
    mode, lo, hi = job
    d = _POOL_DATA
    oracle.mttkrp(np.ascontiguousarray(d["coords"][:, lo:hi]), np.ascontiguousarray(d["vals"][lo:hi]), d["dims"],
                  d["factors"], mode)
    return hi - lo


def cpu_baseline(t, factors, budget_s: float = 20.0):
    """The FP64 oracle MTTKRP (as it stands) on a bounded sample of the tensor: one
    thread, then a process pool over the host cores (modes x nonzero chunks)."""
    import multiprocessing as mp
    import oracle
    # about 10-30 s of single-thread FP64 work: a prefix of the tensor
    n = min(t.nnz, 100_000_000 if factors[0].shape[1] <= 32 else 20_000_000)
    c = np.ascontiguousarray(t.coords[:, :n])
    v = np.ascontiguousarray(t.vals[:n])
    done = 0
    t0 = time.perf_counter()
    modes = 0
    for mode in range(t.nmodes):
        oracle.mttkrp(c, v, t.dims, factors, mode)
        modes += 1
        done += n
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(ncores, 16))
    out = {"value": round(done / el / 1e9, 6), "unit": "Gnnz/s per mode", "cores": 1, "kind": "oracle",
           "sample": f"first {n} of {t.nnz} nonzeros (input order), FP64 oracle MTTKRP, {modes} mode(s), "
                     f"{el:.1f} s on 1 thread",
           "host": {"model": host_model(), "cores_visible": ncores}}
    # the same sample, every mode, split into nonzero chunks over a process pool
    _POOL_DATA.update(coords=c, vals=v, dims=t.dims, factors=factors)
    chunk = (n + workers - 1) // workers
    jobs = [(m, lo, min(n, lo + chunk)) for m in range(t.nmodes) for lo in range(0, n, chunk)]
    try:
        ctx = mp.get_context("fork")
        t1 = time.perf_counter()
        with ctx.Pool(workers) as pool:
            tot = sum(pool.map(_pool_job, jobs, chunksize=1))
        elp = time.perf_counter() - t1
        out["pool"] = {"value": round(tot / elp / 1e9, 6), "unit": "Gnnz/s per mode", "cores": workers,
                       "sample": f"the same {n} nonzeros x {t.nmodes} modes in {len(jobs)} jobs, {elp:.1f} s wall"}
    except Exception as e:  # the pool is context; the single-thread figure stands alone
        out["pool"] = {"error": str(e)[:200]}
    finally:
        _POOL_DATA.clear()
    return out


def stream_rates() -> dict:
    """Measured streaming rates on the GPU (context for the roofline): a 1 GiB
    device copy (HBM read + write), and repeated reads of a 128 MiB buffer
    (Infinity-Cache resident) and of a 2 MiB buffer (L2 resident) through
    stride-0 views summed by torch."""
    import torch
    dev = torch.device("cuda:0")
    x = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    res = {"hbm_copy_gbs": round(2 * 4 * x.numel() * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)}
    del x, y
    for name, mib, rep in (("mall_read_gbs", 128, 8), ("l2_read_gbs", 2, 512)):
        z = torch.ones(mib << 18, dtype=torch.float32, device=dev)
        view = z.expand(rep, -1)
        view.sum()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            view.sum()
        e1.record()
        e1.synchronize()
        res[name] = round(5 * rep * z.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    return res


def sampled_errors(th, Fh, outs, nrows: int = 64, seed: int = 0, nnz_budget: int = 8_000_000) -> dict:
    """Max row error (|X|,|C| row scale) of full-size GPU outputs against the FP64
    oracle on sampled rows: the row with the most nonzeros, then rows of hotness
    rank 1, 3, 10, ..., 1000 and random rows while their nonzeros stay within a
    budget (the oracle runs on exactly the nonzeros of the sampled rows)."""
    import oracle
    rng = np.random.default_rng(seed)
    res = {}
    for n, out in enumerate(outs):
        cnt = np.bincount(th.coords[n], minlength=th.dims[n])
        nz = np.nonzero(cnt)[0]
        order = np.argsort(cnt)[::-1]
        rows, total = [int(order[0])], 0
        cand = [int(order[k]) for k in (1, 3, 10, 30, 100, 300, 1000) if k < nz.size]
        cand += [int(r) for r in rng.choice(nz, size=min(nrows, nz.size), replace=False)]
        for r in cand:
            if r in rows or total + cnt[r] > nnz_budget or len(rows) >= nrows:
                continue
            rows.append(r)
            total += int(cnt[r])
        rows = np.array(sorted(rows), dtype=np.int64)
        lut = np.zeros(th.dims[n], dtype=bool)
        lut[rows] = True
        m = lut[th.coords[n]]
        c = np.ascontiguousarray(th.coords[:, m])
        v = np.ascontiguousarray(th.vals[m])
        ref = oracle.mttkrp(c, v, th.dims, Fh, n)[rows]
        sc = oracle.mttkrp(c, np.abs(v), th.dims, [np.abs(f) for f in Fh], n)[rows]
        err, bad = oracle.row_error(out[rows], ref, sc)
        res[str(n)] = {"max_row_err": float(f"{err:.3e}"), "rows": int(rows.size), "nnz_checked": int(m.sum()),
                       "hottest_row_nnz": int(cnt[order[0]]), "nonzero_empty_rows": bad}
    return res


COUNTER_PASSES = (
    "SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_LDS SQ_INSTS_SALU",
    "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_LDS SQ_WAIT_ANY "
    "SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY",
    "TA_TA_BUSY_sum TA_BUFFER_READ_WAVEFRONTS_sum TD_TD_BUSY_sum TD_LOAD_WAVEFRONT_sum GRBM_GUI_ACTIVE",
)


def profile_cmds(workload: str) -> dict:
    bench = (f"python -u bench.py --workload {workload} --tuned profiles/tuned_layout_{workload}.json "
             f"--no-cpu-baseline --no-check --no-extra")
    cmds = {
        "kt": f"rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof/kt -o kt -- {bench} --steps 2 --warmup 1",
        "cf": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof/cf -o cf -- python -u bench.py --copy-calibration",
        "cw": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof/cw -o cw -- python -u bench.py --copy-calibration",
        "bf": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof/bf -o bf -- {bench} --steps 1 --warmup 0",
        "bw": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof/bw -o bw -- {bench} --steps 1 --warmup 0",
    }
    for i, c in enumerate(COUNTER_PASSES):
        cmds[f"p{i}"] = (f"rocprofv3 --pmc {c} --kernel-include-regex k_mttkrp_seg --output-format csv "
                         f"-d gpurun_out/prof/p{i} -o p{i} -- {bench} --steps 1 --warmup 0")
    return cmds


WORKLOAD_TITLE = {
    "ratings": "the ratings benchmark (480000 x 18000 x 2000, 100M nonzeros, rank 32)",
    "skewed4d": "the skewed 4-mode benchmark (2000000 x 100000 x 50000 x 24, 150M nonzeros, rank 64)",
}
CALL_FIRST = ("k_mttkrp_seg", "k_mttkrp_table", "k_mttkrp<")
CALL_LAST = ("k_reduce_records", "k_reduce_priv")


def _kname(full: str) -> str:
    import re
    m = re.search(r"(k_\w+(?:<[^()]*>)?)\(", full)
    return m.group(1) if m else full.split("(")[0][-60:]


def _read_csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _call_windows(rows, key):
    """Group dispatches (sorted by id) into MTTKRP calls: from a main MTTKRP kernel
    through the next record/partial reduction.  Returns per call [sum, names, per-kernel sums]."""
    rows = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
    calls, cur = [], None
    for r in rows:
        n = _kname(r["Kernel_Name"])
        if n.startswith(CALL_FIRST):
            cur = [0.0, [], {}]
        if cur is not None:
            v = key(r)
            cur[0] += v
            cur[1].append(n)
            short = n.split("<")[0]
            cur[2][short] = cur[2].get(short, 0.0) + v
            if n.startswith(CALL_LAST):
                calls.append(cur)
                cur = None
    return calls


def _per_dispatch(path):
    """Counter rows summed per (dispatch, counter) -> {dispatch: {counter: value}}."""
    out = {}
    for r in _read_csv(path):
        d = out.setdefault(int(r["Dispatch_Id"]), {"kernel": _kname(r["Kernel_Name"])})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def summarize_profiles(d: str, workload: str = "skewed4d"):
    """Write the committed summaries from rocprofv3 CSV output under d."""
    cmds = profile_cmds(workload)
    title = WORKLOAD_TITLE[workload]
    lines = [f"# Kernel trace of {title}",
             f"# command: cd /tmp && export TMPDIR=/tmp; cd <repo>; {cmds['kt']}",
             "# columns: calls, average us, total ms, percent of GPU time, kernel", ""]
    st = _read_csv(os.path.join(d, "kt", "kt_kernel_stats.csv"))
    for r in sorted(st, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} {float(r['TotalDurationNs']) / 1e6:9.2f} "
                     f"{float(r['Percentage']):6.2f}  {_kname(r['Name'])}")
    tr = _read_csv(os.path.join(d, "kt", "kt_kernel_trace.csv"))
    calls = _call_windows(tr, lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    if calls:
        per_k = {}
        for c in calls:
            for k, v in c[2].items():
                per_k[k] = per_k.get(k, 0.0) + v
        lines += ["", f"MTTKRP calls: {len(calls)}; kernel time per call (all kernels of the call) "
                      f"avg {sum(c[0] for c in calls) / len(calls):.1f} us",
                  "per kernel, avg us per call: " + ", ".join(f"{k} {v / len(calls):.1f}" for k, v in per_k.items()),
                  "kernels of one call: " + " ".join(calls[-1][1])]
    with open(os.path.join(ROOT, "profiles", f"mttkrp_{workload}_kernels.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def copy_factor(sub):
        rows = [r for r in _read_csv(os.path.join(d, sub, sub + "_counter_collection.csv"))
                if "copyBuffer" in r["Kernel_Name"] or "elementwise" in r["Kernel_Name"].lower()]
        big = [float(r["Counter_Value"]) for r in rows if float(r["Counter_Value"]) > 1e5]
        kib = sum(big) / len(big)
        return (1 << 30) / (kib * 1024.0), kib

    ff, fk = copy_factor("cf")
    wf, wk = copy_factor("cw")
    cf_ = _call_windows(_read_csv(os.path.join(d, "bf", "bf_counter_collection.csv")), lambda r: float(r["Counter_Value"]))
    cw_ = _call_windows(_read_csv(os.path.join(d, "bw", "bw_counter_collection.csv")), lambda r: float(r["Counter_Value"]))
    fetch = sum(c[0] for c in cf_) / len(cf_) * 1024 * ff
    write = sum(c[0] for c in cw_) / len(cw_) * 1024 * wf
    from paper_2509_00280_amd import synth
    nnz = synth._CONFIGS[workload][2]
    split = []
    for name, cl, fac in (("FETCH", cf_, ff), ("WRITE", cw_, wf)):
        per_k = {}
        for c in cl:
            for k, v in c[2].items():
                per_k[k] = per_k.get(k, 0.0) + v
        split.append(f"{name.lower()}_bytes_per_nnz_by_kernel: " +
                     ", ".join(f"{k} {v / len(cl) * 1024 * fac / nnz:.2f}" for k, v in per_k.items()))
    out = [f"# HBM traffic of one mode-n MTTKRP call (all of its kernels) in {title}",
           f"# commands (each its own run): cd /tmp && export TMPDIR=/tmp; cd <repo>;",
           f"#   {cmds['cf']}", f"#   {cmds['cw']}", f"#   {cmds['bf']}", f"#   {cmds['bw']}",
           f"# calibration: a 1 GiB device copy reads FETCH_SIZE {fk:.0f} KiB and WRITE_SIZE {wk:.0f} KiB per dispatch,",
           f"# so FETCH_SIZE KiB x {ff:.3f} and WRITE_SIZE KiB x {wf:.3f} give bytes",
           f"# calls averaged: {len(cf_)} (FETCH run), {len(cw_)} (WRITE run)",
           f"source_digest: {source_digest()}",
           f"nnz: {nnz}",
           f"fetch_bytes_per_launch: {fetch:.0f}",
           f"write_bytes_per_launch: {write:.0f}",
           f"hbm_bytes_per_launch: {fetch + write:.0f}",
           f"hbm_bytes_per_nnz: {(fetch + write) / nnz:.2f}"] + split
    with open(pmc_file(workload), "w") as f:
        f.write("\n".join(out) + "\n")
    # counters of the main kernel (each pass its own run)
    cl = [f"# Counters of the main MTTKRP kernel in {title}",
          "# commands (each its own run): cd /tmp && export TMPDIR=/tmp; cd <repo>;"]
    cl += [f"#   {cmds[f'p{i}']}" for i in range(len(COUNTER_PASSES))]
    cl.append("# values are per dispatch, averaged over the dispatches of the run; busy and conflict")
    cl.append("# percentages are relative to the kernel's GPU cycles (GRBM_GUI_ACTIVE x CUs per XCD)")
    agg = {}
    for i in range(len(COUNTER_PASSES)):
        path = os.path.join(d, f"p{i}", f"p{i}_counter_collection.csv")
        if not os.path.exists(path):
            continue
        disp = _per_dispatch(path)
        for dd in disp.values():
            for k, v in dd.items():
                if k != "kernel":
                    agg.setdefault(k, []).append(v)
    avg = {k: sum(v) / len(v) for k, v in agg.items()}
    for k in sorted(avg):
        cl.append(f"{k}: {avg[k]:.4g}")
    if "GRBM_GUI_ACTIVE" in avg:
        cu_cycles = avg["GRBM_GUI_ACTIVE"] / 8 * 256  # per-XCD cycles x 256 CUs
        for k in ("TA_TA_BUSY_sum", "TD_TD_BUSY_sum", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS"):
            if k in avg:
                cl.append(f"{k} per CU-cycle: {avg[k] / cu_cycles:.3f}")
        if "SQ_LDS_BANK_CONFLICT" in avg and "SQ_ACTIVE_INST_LDS" in avg:
            cl.append(f"LDS bank-conflict cycles / LDS active cycles: "
                      f"{avg['SQ_LDS_BANK_CONFLICT'] / avg['SQ_ACTIVE_INST_LDS']:.3f}")
    with open(os.path.join(ROOT, "profiles", f"mttkrp_{workload}_counters.txt"), "w") as f:
        f.write("\n".join(cl) + "\n")
    print("\n".join(lines + [""] + out + [""] + cl))


def summarize_f64(d: str, fetch_factor: float = 2.0, write_factor: float = 1.0):
    """profiles/mttkrp_f64_table3_traffic.txt from the FETCH_SIZE and WRITE_SIZE runs of
    ``bench.py --workload f64 --f64-reps 1`` under d (calibration factors of a plain
    1 GiB device copy on the same GPU, as in the skewed tensor's traffic summary)."""
    out = json.load(open(os.path.join(d, "bench.json")))
    items = out["tensors"]
    res = {}
    for c, fac in (("FETCH_SIZE", fetch_factor), ("WRITE_SIZE", write_factor)):
        calls = _call_windows(_read_csv(os.path.join(d, c, "p_counter_collection.csv")),
                              lambda r: float(r["Counter_Value"]))
        pos = 0
        for it in items:
            n = 2 * len(it["dims"])  # one warm-up call and one timed call per mode
            sel = calls[pos:pos + n]
            pos += n
            res.setdefault(it["tensor"], {})[c] = sum(x[0] for x in sel) / len(sel) * 1024 * fac
    lines = ["# FP64 MTTKRP (FP64 values and factors, rank 16: the paper's precision) on synthetic stand-ins",
             "# with the Table I shapes of the three tensors of Table III, measured HBM bytes per nonzero and mode",
             "# beside Table III's memory volumes per nonzero and mode (GB / (nnz x 3), CPU, ReLATE / ALTO).",
             "# commands (each its own run): cd /tmp && export TMPDIR=/tmp; cd <repo>;",
             "#   python -u bench.py --workload f64",
             "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/f64/FETCH_SIZE -o p -- "
             "python -u bench.py --workload f64 --f64-reps 1",
             "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/f64/WRITE_SIZE -o p -- "
             "python -u bench.py --workload f64 --f64-reps 1",
             f"# byte factors: FETCH_SIZE KiB x {fetch_factor}, WRITE_SIZE KiB x {write_factor} (1 GiB copy calibration)",
             f"# source_digest: {source_digest()}", "",
             f"{'tensor':8s} {'nnz':>10s} {'Gnnz/s/mode':>11s} {'alg B/nnz':>9s} {'meas B/nnz':>10s} "
             f"{'Table III ReLATE / ALTO B/nnz':>30s}"]
    for it in items:
        r = res[it["tensor"]]
        meas = (r["FETCH_SIZE"] + r["WRITE_SIZE"]) / it["nnz"]
        g = np.mean([m["gnnz_per_s"] for m in it["per_mode"].values()])
        t3 = it["paper_table3_bytes_per_nnz_mode_relate_alto"]
        lines.append(f"{it['tensor']:8s} {it['nnz']:10d} {g:11.2f} {it['algorithmic_bytes_per_nnz_mode']:9.2f} "
                     f"{meas:10.2f} {t3[0]:>17.1f} / {t3[1]:<10.1f}")
    with open(os.path.join(ROOT, "profiles", "mttkrp_f64_table3_traffic.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _upload(t):
    import torch
    c = torch.from_numpy(np.ascontiguousarray(t.coords).view(np.int32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(t.vals)).cuda()
    return c, v


def bench_layouts(args):
    """The layout search with the paper's reward (Section III-C): for every
    tensor, original and label-shuffled (Section IV-A), the all-mode MTTKRP time
    of the ALTO layout and of the best layout the search finds (each mode at its
    best plan), and their ratio, the speedup over ALTO.  Tensors: the ratings and
    skewed 4-mode workloads, and synthetic stand-ins with the shapes of Table I
    (nonzeros capped at --layout-nnz-cap, rank 16 as in the paper)."""
    import torch
    from paper_2509_00280_amd import spt, synth
    items = []
    for name in args.layout_tensors:
        for shuffle in (False, True):
            t0 = time.time()
            if name in ("ratings", "skewed4d"):
                t, F, rank, _ = synth.config_device(name, shuffle=shuffle)
            else:
                full = synth.TABLE1[name][1]
                t, F, rank = synth.table1_config(name, nnz=min(full, args.layout_nnz_cap), device="cuda",
                                                 shuffle=shuffle)
            torch.cuda.synchronize()
            gen_s = time.time() - t0
            h = spt.encode(t.dims, t.coords, t.vals)
            info = h.info()
            t1 = time.time()
            res = spt.autotune(h, F, budget_ms=args.tune_budget_ms, random_samples=args.tune_samples, seed=17)
            rec = {"tensor": name, "shuffled": shuffle, "dims": list(t.dims), "nnz": t.nnz, "rank": rank,
                   "key_bits": info["lp"], "alto_ms": round(res["alto_ms"], 4), "best_ms": round(res["best_ms"], 4),
                   "speedup_vs_alto": round(res["alto_ms"] / res["best_ms"], 4),
                   "candidates": res["candidates"], "random_samples": res["random_samples"],
                   "layout_changed": h.info()["layout"] != info["layout"],
                   "alto_gnnz_per_s_per_mode": round(t.nnz * t.nmodes / (res["alto_ms"] * 1e-3) / 1e9, 2),
                   "search_s": round(time.time() - t1, 1), "generate_s": round(gen_s, 1)}
            log(json.dumps(rec))
            items.append(rec)
            h.free()
            del t, F, h
            torch.cuda.empty_cache()
    sp = [r["speedup_vs_alto"] for r in items]
    geo = float(np.exp(np.mean(np.log(sp)))) if sp else None
    out = {"metric": "all-mode MTTKRP speedup of the searched layout over ALTO", "value": round(geo, 4),
           "unit": "x (geomean)", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded, drawn on the GPU)",
           "config": {"workload": "layout search: ratings, skewed 4-mode and Table I-shaped tensors, original and "
                                  "label-shuffled", "tune_budget_ms": args.tune_budget_ms,
                      "tune_samples": args.tune_samples, "nnz_cap": args.layout_nnz_cap},
           "tensors": items}
    print(json.dumps(out), flush=True)


def bench_agent(args):
    """The learned layout search (Algorithm 1: masked double DQN, reward model,
    elastic stopping) with our MTTKRP as its environment, on shuffled Table
    I-shaped stand-ins and the shuffled ratings tensor: the speedup over ALTO of
    the best layout it measures, beside the measured search (ALTO, uniform
    samples, hill climb) given the same wall time, both judged by the same
    reward (all-mode MTTKRP under the default plan, median of 3)."""
    import torch
    from paper_2509_00280_amd import agent, spt, synth
    items = []
    for name in args.agent_tensors:
        t0 = time.time()
        if name in ("ratings", "skewed4d"):
            t, F, rank, _ = synth.config_device(name, nnz=args.agent_nnz_cap, shuffle=True)
        else:
            full = synth.TABLE1[name][1]
            t, F, rank = synth.table1_config(name, nnz=min(full, args.agent_nnz_cap), device="cuda", shuffle=True)
        torch.cuda.synchronize()
        gen_s = time.time() - t0
        reward, alto, alto_ms, lbits = agent.gpu_environment(t.dims, t.coords, t.vals, F)
        t1 = time.time()
        res = agent.relate_search(reward, lbits, episodes=args.agent_episodes, seed=23,
                                  max_evaluations=args.agent_evals,
                                  log=lambda m, n=name: log(f"agent {n}: {m}"))
        agent_s = time.time() - t1
        # the measured search with the same wall time, judged by the same reward
        h = spt.encode(t.dims, t.coords, t.vals)
        t2 = time.time()
        spt.autotune(h, F, budget_ms=agent_s * 1e3, random_samples=args.tune_samples, seed=23)
        climb_s = time.time() - t2
        climb_layout = list(h.info()["layout"])
        h.free()
        climb = reward(climb_layout)
        rec = {"tensor": name, "shuffled": True, "dims": list(t.dims), "nnz": t.nnz, "rank": rank,
               "key_bits": int(sum(lbits)), "alto_ms": round(alto_ms, 4),
               "agent_speedup_vs_alto": round(res.best_reward, 4), "agent_episodes": res.episodes,
               "agent_measured": res.evaluations, "agent_cache_hits": res.cache_hits,
               "agent_imagined": res.imagined, "reward_model_trusted_at": res.model_trusted_at,
               "stopped_early": res.stopped_early, "agent_s": round(agent_s, 1),
               "climb_speedup_vs_alto": round(climb, 4), "climb_s": round(climb_s, 1),
               "generate_s": round(gen_s, 1)}
        log(json.dumps(rec))
        items.append(rec)
        del t, F
        torch.cuda.empty_cache()
    geo = lambda k: round(float(np.exp(np.mean(np.log([r[k] for r in items])))), 4) if items else None
    out = {"metric": "speedup over ALTO of the layout found by the learned search (geomean)",
           "value": geo("agent_speedup_vs_alto"), "unit": "x", "n_gpus": 1, "higher_is_better": True,
           "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded, drawn on the GPU)",
           "config": {"workload": "learned layout search (masked double DQN, Algorithm 1) on shuffled tensors",
                      "episodes_max": args.agent_episodes, "measurements_max": args.agent_evals,
                      "nnz_cap": args.agent_nnz_cap},
           "measured_search_geomean": geo("climb_speedup_vs_alto"), "tensors": items}
    print(json.dumps(out), flush=True)


# Table III of the paper: memory volume of one all-mode MTTKRP iteration per
# nonzero and mode (GB / (nnz x 3), FP64, CPU; the unit is the survey's reading)
TABLE3_BYTES_PER_NNZ_MODE = {"deli-3d": (125.8, 222.3), "patents": (16.4, 16.3), "reddit": (31.1, 50.8)}


def bench_f64(args):
    """FP64 MTTKRP (the paper's precision: FP64 values and factors, rank 16) on
    synthetic stand-ins with the Table I shapes whose memory volumes Table III
    prints, next to those volumes (ReLATE / ALTO on the paper's CPU)."""
    import torch
    from paper_2509_00280_amd import spt, synth
    items = []
    for name in args.f64_tensors:
        full = synth.TABLE1[name][1]
        t, F32, rank = synth.table1_config(name, nnz=min(full, args.layout_nnz_cap), device="cuda")
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1234)
        vals64 = torch.rand(t.nnz, generator=gen, device="cuda", dtype=torch.float64)
        F = [f.to(torch.float64) for f in F32]
        h = spt.encode(t.dims, t.coords, t.vals)
        spt.attach_f64(h, vals64)
        h.prepare(rank)
        outs = [torch.empty((d, rank), dtype=torch.float64, device="cuda") for d in t.dims]
        for n in range(t.nmodes):
            spt.mttkrp_f64(h, F, n, out=outs[n])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        per = {}
        tot = 0.0
        for n in range(t.nmodes):
            e0.record()
            for _ in range(args.f64_reps):
                spt.mttkrp_f64(h, F, n, out=outs[n])
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1) / args.f64_reps
            tot += ms
            per[str(n)] = {"ms": round(ms, 4), "gnnz_per_s": round(t.nnz / (ms * 1e-3) / 1e9, 3)}
        # compulsory bytes of an FP64 call: 8 B key + 8 B value per nonzero, touched factor rows and the output
        kw = 8 if sum((int(d) - 1).bit_length() for d in t.dims) <= 64 else 16
        alg = []
        for n in range(t.nmodes):
            b = t.nnz * (kw + 8) + int(t.dims[n]) * rank * 8
            for k, d in enumerate(t.dims):
                if k != n:
                    seen = torch.zeros(int(d), dtype=torch.bool, device="cuda")
                    seen[t.coords[k].long()] = True
                    b += int(seen.sum().item()) * rank * 8
            alg.append(b)
        rec = {"tensor": name, "dims": list(t.dims), "nnz": t.nnz, "rank": rank, "per_mode": per,
               "all_mode_ms": round(tot, 4),
               "algorithmic_bytes_per_nnz_mode": round(sum(alg) / len(alg) / t.nnz, 2),
               "paper_table3_bytes_per_nnz_mode_relate_alto": TABLE3_BYTES_PER_NNZ_MODE.get(name)}
        log(json.dumps(rec))
        items.append(rec)
        h.free()
        del t, F, F32, outs, vals64, h
        torch.cuda.empty_cache()
    out = {"metric": "FP64 MTTKRP Gnnz/s per mode", "unit": "Gnnz/s", "n_gpus": 1, "higher_is_better": True,
           "value": round(float(np.mean([np.mean([m["gnnz_per_s"] for m in r["per_mode"].values()]) for r in items])), 3),
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded, drawn on the GPU)",
           "config": {"workload": "FP64 MTTKRP on Table I-shaped stand-ins " + ", ".join(args.f64_tensors),
                      "nnz_cap": args.layout_nnz_cap},
           "tensors": items}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """256 independent tensors (3 or 4 modes, 1e4..5e6 nonzeros, Zipf(1.2)
    labels, ranks 16/32): lock-step batched CP-ALS against the plain
    per-tensor GPU CP-ALS, same iterations, same inputs; the batched run is
    timed at the default batch tile and again after the batch autotuner."""
    import torch
    from paper_2509_00280_amd import spt, synth
    t0 = time.time()
    members = synth.batch_config(seed=4, count=args.batch_count)
    log(f"generated {len(members)} tensors, {sum(t.nnz for t, _, _ in members)} nonzeros in {time.time() - t0:.1f} s")
    hs = []
    torch.cuda.synchronize()
    te = time.perf_counter()
    for t, F, R in members:
        c, v = _upload(t)
        hs.append(spt.encode(t.dims, c, v))
    torch.cuda.synchronize()
    t_enc = time.perf_counter() - te
    iters = args.batch_iters
    F0 = [[torch.from_numpy(f).cuda() for f in F] for _, F, _ in members]

    def fresh():
        return [[f.clone() for f in fl] for fl in F0]

    # warm-up of both paths (plans, pools) on the first tensors
    spt.cp_als_batched(hs[:4], fresh()[:4], 1)
    for h, fl in zip(hs[:4], fresh()[:4]):
        spt.cp_als(h, fl, 1)
    torch.cuda.synchronize()
    Fs = fresh()
    ts = time.perf_counter()
    fits_s = [spt.cp_als(h, fl, iters)[1] for h, fl in zip(hs, Fs)]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - ts
    def batched():
        Fb = fresh()
        tb = time.perf_counter()
        _, fits_b, _ = spt.cp_als_batched(hs, Fb, iters)
        torch.cuda.synchronize()
        return time.perf_counter() - tb, fits_b

    t_batch_default, _ = batched()  # the default batch tile (2048 nonzeros)
    # the batch autotuner (outside the timed regions): member layouts when
    # --batch-layout-ms > 0, then the batch tile by timing the all-mode batched MTTKRP
    tt = time.perf_counter()
    tune = spt.autotune_batched(hs, F0, layout_budget_ms=args.batch_layout_ms, random_samples=2, seed=4)
    t_tune = time.perf_counter() - tt
    log(f"batch tune in {t_tune:.1f} s: {tune}")
    spt.cp_als_batched(hs[:4], fresh()[:4], 1)  # re-plans (if any) outside the timed region
    t_batch, fits_b = batched()
    dfit = max(abs(a - b) for a, b in zip(fits_s, fits_b))
    n = len(members)
    out = {"metric": "CP-ALS solves/s (batched vs per-tensor)", "value": round(n / t_batch, 3), "unit": "solves/s",
           "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32 MTTKRP, f64 solve",
           "data": "synthetic",
           "config": {"workload": f"{n} independent tensors, 3 or 4 modes, 1e4..5e6 nonzeros (log-uniform), "
                                  f"Zipf(1.2) labels, ranks 16/32, {iters} CP-ALS iterations each",
                      "total_nnz": int(sum(t.nnz for t, _, _ in members)), "iters": iters},
           "batched_s": round(t_batch, 4), "per_tensor_s": round(t_single, 4),
           "per_tensor_solves_per_s": round(n / t_single, 3), "speedup": round(t_single / t_batch, 3),
           "encode_s": round(t_enc, 4), "max_abs_fit_diff": dfit,
           "batch_tune": {"best_tile": tune["best_tile"],
                          "all_mode_batched_mttkrp_ms": {str(k): round(v, 4) for k, v in tune["ms"].items()},
                          "layouts_tuned": tune["layouts_tuned"], "layout_speedup": round(tune["layout_speedup"], 4),
                          "tune_s": round(t_tune, 2), "batched_s_default_tile": round(t_batch_default, 4)}}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Continuous batching (the serving configuration): Poisson arrivals of CP-ALS
    requests drawn like the batched workload (3 or 4 modes, 1e4..5e6 nonzeros,
    Zipf(1.2), ranks 16/32/48/64, <= 50 iterations or |dfit| < 1e-4).  After
    --serve-warmup requests, --serve-count requests are served saturated (all
    submitted at once) and open-loop at each --serve-loads fraction of the
    saturated rate; p50/p99 of done - arrive, queueing split, errors.  The plain
    per-tensor GPU CP-ALS runs the first --serve-plain requests for comparison,
    with the largest |served fit - plain fit| over them."""
    import threading
    import torch
    from paper_2509_00280_amd import spt, synth
    t0 = time.time()
    total = args.serve_warmup + args.serve_count
    reqs = synth.serving_requests(seed=5, count=total)
    uniq = min(args.serve_unique, total)
    mats = []
    for i in range(uniq):
        mats.append(synth.materialize_device(reqs[i]))
    torch.cuda.synchronize()
    pick = [mats[i % uniq] for i in range(total)]
    log(f"drew {uniq} distinct requests ({sum(t.nnz for t, _, _ in mats)} nonzeros) for {total} arrivals "
        f"in {time.time() - t0:.1f} s")
    iters, tol = 50, 1e-4
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.5)
    warm, meas = pick[:args.serve_warmup], pick[args.serve_warmup:]

    def run_saturated(batch):
        srv = spt.Server(budget, args.serve_slots)
        ts = time.perf_counter()
        tickets = [srv.submit(t.dims, t.coords, t.vals, F, iters, tol) for t, F, R in batch]
        res = [srv.wait(k, want_factors=False)[0] for k in tickets]
        el = time.perf_counter() - ts
        srv.close()
        return res, el

    run_saturated(warm)  # warm-up requests (pools, plans, kernels)
    res_sat, t_sat = run_saturated(meas)
    sat = len(meas) / t_sat
    bad = sum(r["status"] != 0 for r in res_sat)
    log(f"saturated: {sat:.1f} solves/s over {len(meas)} requests, {bad} errors")
    # plain per-tensor GPU CP-ALS (encode + solve, one request after another) on a prefix
    nplain = min(args.serve_plain, len(meas))
    torch.cuda.synchronize()
    tp = time.perf_counter()
    plain_fit = []
    for t, F, R in meas[:nplain]:
        c = torch.from_numpy(np.ascontiguousarray(t.coords).view(np.int32)).cuda()
        v = torch.from_numpy(np.ascontiguousarray(t.vals)).cuda()
        h = spt.encode(t.dims, c, v)
        plain_fit.append(spt.cp_als(h, [torch.from_numpy(f).cuda() for f in F], iters, tol=tol)[1])
        h.free()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - tp
    dfit = max(abs(a["fit"] - b) for a, b in zip(res_sat[:nplain], plain_fit))
    # open loop: Poisson arrivals at `load` x the saturated rate
    lat = {}
    for load in args.serve_loads:
        rate = load * sat
        arrive = np.cumsum(np.random.default_rng(55).exponential(1.0 / rate, size=len(meas)))
        srv = spt.Server(budget, args.serve_slots)
        tks = [None] * len(meas)

        def submitter():
            base = srv.now()
            for i, (t, F, R) in enumerate(meas):
                d = base + arrive[i] - srv.now()
                if d > 0:
                    time.sleep(d)
                tks[i] = srv.submit(t.dims, t.coords, t.vals, F, iters, tol)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        rs = [srv.wait(k, want_factors=False)[0] for k in tks]
        srv.close()
        d = np.array([r["t_done"] - r["t_arrive"] for r in rs])
        q = np.array([r["t_admit"] - r["t_arrive"] for r in rs])
        span = max(r["t_done"] for r in rs) - min(r["t_arrive"] for r in rs)
        lat[str(load)] = {"p50_s": round(float(np.percentile(d, 50)), 4), "p99_s": round(float(np.percentile(d, 99)), 4),
                          "queue_p50_s": round(float(np.percentile(q, 50)), 4),
                          "queue_p99_s": round(float(np.percentile(q, 99)), 4),
                          "service_p50_s": round(float(np.percentile(d - q, 50)), 4),
                          "solves_per_s": round(len(rs) / span, 3), "errors": int(sum(r["status"] != 0 for r in rs))}
        log(f"load {load}: {lat[str(load)]}")
    out = {"metric": "served CP-ALS solves/s and latency", "value": round(sat, 3), "unit": "solves/s",
           "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32 MTTKRP, f64 solve",
           "data": "synthetic (seeded; tensors drawn on the GPU)",
           "config": {"workload": f"{args.serve_count} requests after {args.serve_warmup} warm-up requests "
                                  f"({uniq} distinct tensors cycled), 3 or 4 modes, 1e4..5e6 nonzeros "
                                  f"(log-uniform), Zipf(1.2), ranks 16/32/48/64, <= {iters} iterations or "
                                  f"|dfit| < {tol}",
                      "hbm_budget_bytes": budget, "slots": args.serve_slots},
           "saturated_solves_per_s": round(sat, 3),
           "plain_per_tensor_solves_per_s": round(nplain / t_plain, 3),
           "plain_measured_on": nplain,
           "speedup_vs_plain": round(sat / (nplain / t_plain), 3),
           "max_abs_fit_served_vs_plain": float(f"{dfit:.3e}"),
           "errors": bad, "open_loop": lat}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nnz", type=float, default=None, help="scale the tensor down (debug only; not the benchmark)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("skewed4d", "ratings", "batch", "serve", "layouts", "f64", "agent"),
                    default="skewed4d",
                    help="skewed4d: the headline, the 4-mode rank-64 tensor whose factors exceed the Infinity "
                         "Cache; ratings: the 3-mode rank-32 tensor; batch: batched vs per-tensor CP-ALS; "
                         "serve: continuous-batching server latency")
    ap.add_argument("--tune-budget-ms", type=float, default=30000.0,
                    help="wall-time budget of the layout and plan search before the timed region (0: ALTO)")
    ap.add_argument("--tune-samples", type=int, default=4, help="uniform samples of the layout space in the search")
    ap.add_argument("--tuned", default=None, metavar="JSON",
                    help="use a recorded search result (layout and plan) instead of searching")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle check")
    ap.add_argument("--layout-tensors", nargs="*", default=None,
                    help="layouts workload: tensors to search (default: ratings, skewed4d and every Table I shape)")
    ap.add_argument("--layout-nnz-cap", type=int, default=150_000_000)
    ap.add_argument("--f64-tensors", nargs="*", default=["deli-3d", "patents", "reddit"])
    ap.add_argument("--f64-reps", type=int, default=5)
    ap.add_argument("--no-extra", action="store_true", help="skip the ratings MTTKRP line")
    ap.add_argument("--torch-allocator", action="store_true",
                    help="route the library's device memory through PyTorch's caching allocator")
    ap.add_argument("--agent-tensors", nargs="+", default=["reddit", "deli-3d", "ratings"])
    ap.add_argument("--agent-episodes", type=int, default=400, help="E_max of the learned search")
    ap.add_argument("--agent-evals", type=int, default=150, help="real measurements at most per tensor")
    ap.add_argument("--agent-nnz-cap", type=int, default=20_000_000)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-iters", type=int, default=10)
    ap.add_argument("--batch-layout-ms", type=float, default=0.0,
                    help="layout search budget per member in the batch autotuner (0: tile only)")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-unique", type=int, default=250, help="distinct request tensors drawn (then cycled)")
    ap.add_argument("--serve-plain", type=int, default=300, help="requests run through the plain per-tensor path")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-loads", type=float, nargs="*", default=[0.5, 0.8, 1.0])
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None,
                    help="write the profiles/ summaries from rocprofv3 CSV output under DIR (no GPU)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_profiles:
        if args.workload == "f64":
            summarize_f64(args.summarize_profiles)
        else:
            summarize_profiles(args.summarize_profiles, args.workload)
        return
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; sharding across GPUs is not implemented; "
                                   "--gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "agent":
        bench_agent(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "f64":
        bench_f64(args)
        return
    if args.workload == "layouts":
        from paper_2509_00280_amd import synth
        if args.layout_tensors is None:
            args.layout_tensors = ["ratings", "skewed4d"] + list(synth.TABLE1)
        if args.tune_budget_ms == 30000.0:
            args.tune_budget_ms = 8000.0
        bench_layouts(args)
        return

    bench_tensor(args)


def mttkrp_line(spt, t, F, rank, reps: int = 10, layout=None, plan=None) -> dict:
    """All-mode MTTKRP of one device tensor: per-mode call time (HIP events),
    Gnnz/s, algorithmic bytes and the call's HBM-roofline fraction."""
    import torch
    h = spt.encode(t.dims, t.coords, t.vals, layout=layout)
    if plan is not None:
        h.set_plan(tile=plan["tile"], strategy=plan["strategy"], row_cache=plan["row_cache"])
    h.prepare(rank)
    outs = [torch.empty((d, rank), device="cuda") for d in t.dims]
    for n in range(t.nmodes):
        spt.mttkrp(h, F, n, out=outs[n])
    torch.cuda.synchronize()
    per_mode = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for n in range(t.nmodes):
        e0.record()
        for _ in range(reps):
            spt.mttkrp(h, F, n, out=outs[n])
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        alg = algorithmic_bytes(t, rank, n)
        per_mode[str(n)] = {"ms": round(ms, 4), "gnnz_per_s": round(t.nnz / (ms * 1e-3) / 1e9, 3),
                            "algorithmic_bytes": alg, "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    h.free()
    return {"per_mode": per_mode, "outs": outs}


def bench_tensor(args):
    import torch
    from paper_2509_00280_amd import spt, synth

    if args.torch_allocator:
        spt.use_torch_allocator(True)
    t0 = time.time()
    t, F0, rank, iters = synth.config_device(args.workload, nnz=None if args.nnz is None else int(args.nnz))
    torch.cuda.synchronize()
    log(f"generated {t.nnz} nonzeros on the GPU in {time.time() - t0:.1f} s")
    dev = torch.device("cuda:0")
    nm = t.nmodes
    Fw = [torch.empty_like(f) for f in F0]
    lam = torch.empty(rank, dtype=torch.float64, device=dev)

    # the autotuner picks the layout and per-mode plan (outside the timed region)
    tune = None
    layout, plan = None, None
    if args.tuned:
        with open(args.tuned) as f:
            tune = json.load(f)
        layout, plan = tune["layout"], dict(tune["plan"])
        plan["tile"] = plan["tile"] + [4096] * (8 - nm)
        plan["strategy"] = plan["strategy"] + [4] * (8 - nm)
        tune["from_file"] = os.path.relpath(args.tuned, ROOT)
    elif args.tune_budget_ms > 0:
        h = spt.encode(t.dims, t.coords, t.vals)
        t1 = time.time()
        tune = spt.autotune(h, F0, budget_ms=args.tune_budget_ms, random_samples=args.tune_samples, seed=7)
        layout, plan = h.info()["layout"], h.get_plan()
        tune.update(search_s=round(time.time() - t1, 2), layout=layout,
                    plan={"tile": plan["tile"][:nm], "strategy": plan["strategy"][:nm], "row_cache": plan["row_cache"]},
                    speedup_vs_alto=round(tune["alto_ms"] / tune["best_ms"], 4))
        h.free()
        log(f"autotune: {tune}")
        os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
        with open(os.path.join(ROOT, "gpurun_out", f"tuned_{args.workload}.json"), "w") as f:
            json.dump(tune, f)

    def step():
        for a, b in zip(Fw, F0):
            a.copy_(b)
        h = spt.encode(t.dims, t.coords, t.vals, layout=layout)
        if plan is not None:
            h.set_plan(tile=plan["tile"], strategy=plan["strategy"], row_cache=plan["row_cache"])
        _, fit, its = spt.cp_als(h, Fw, iters, lam=lam)
        h.free()
        return fit, its

    for i in range(args.warmup):
        fit, its = step()
        log(f"warmup {i}: fit {fit:.6f} iters {its}")
    torch.cuda.synchronize()
    spt.profile_reset()
    t_start = time.perf_counter()
    for i in range(args.steps):
        fit, its = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t_start
    prof = spt.profile_read()
    spt.profile_reset(False)
    ms_step = el * 1e3 / args.steps
    value = t.nnz * nm * iters / (ms_step * 1e-3) / 1e9
    log(f"{args.steps} steps in {el:.3f} s: {ms_step:.2f} ms/step, fit {fit:.6f}")

    # MTTKRP calls alone (HIP events on the library's stream around every call)
    per_mode = {}
    for m in range(nm):
        cnt = prof["mttkrp_launches"][m]
        ms = prof["mttkrp_ms"][m] / max(cnt, 1)
        per_mode[str(m)] = {"ms": round(ms, 4), "gnnz_per_s": round(t.nnz / (ms * 1e-3) / 1e9, 3)}
    mk_ms = sum(prof["mttkrp_ms"]) / max(sum(prof["mttkrp_launches"]), 1)
    alg = [algorithmic_bytes(t, rank, m) for m in range(nm)]
    alg_avg = sum(alg) / nm
    achieved = alg_avg / (mk_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(pmc_file(args.workload)):
        pmc = {}
        with open(pmc_file(args.workload)) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    pmc[k.strip()] = v.strip()
        if pmc.get("source_digest") == source_digest() and pmc.get("nnz") == str(t.nnz):
            traffic = float(pmc["hbm_bytes_per_launch"])
    rates = stream_rates()
    # every factor-row read of a call (no reuse) must at least cross the fastest
    # on-chip path, LDS: 128 B per clock per CU x 256 CUs x 2.4 GHz
    gather_bytes = t.nnz * (nm - 1) * 4 * rank
    lds_peak_gbs = 128 * 256 * 2.4
    bound_ms = max(alg_avg / (HBM_PEAK_GBS * 1e9), gather_bytes / (lds_peak_gbs * 1e9)) * 1e3
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "one mode-n MTTKRP call (k_mttkrp_segd, k_fill_zero, k_reduce_records)",
                "algorithmic_bytes_per_launch": int(alg_avg),
                "algorithmic_bytes_per_nnz": round(alg_avg / t.nnz, 2),
                "measured_bytes_per_nnz": None if traffic is None else round(traffic / t.nnz, 2),
                "avg_launch_ms": round(mk_ms, 4),
                "measured_rates": rates,
                "frac_of_measured_hbm_copy": round(achieved / rates["hbm_copy_gbs"], 4),
                "cache_aware_bound": {"ms": round(bound_ms, 4), "frac": round(bound_ms / mk_ms, 4),
                                      "gather_bytes_per_launch": int(gather_bytes),
                                      "rule": "max(compulsory bytes / 8 TB/s HBM, factor-row gather bytes without "
                                              "reuse / 78.6 TB/s LDS peak); frac = bound / measured call time"}}
    shape = "x".join(map(str, t.dims))
    if args.workload == "ratings":
        desc = (f"ratings-shaped 3-mode tensor {shape}, {t.nnz} nonzeros, Zipf(1.1)/Zipf(1.1)/uniform labels, "
                f"values in 1..5, rank {rank}, ")
    else:
        desc = (f"skewed 4-mode tensor {shape}, {t.nnz} nonzeros, Zipf(1.3) x3 / uniform labels, "
                f"lognormal values, rank {rank}, ")
    out = {
        "metric": "MTTKRP Gnnz/s per mode", "value": round(value, 3), "unit": "Gnnz/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded, drawn on the GPU)",
        "config": {"workload": desc + f"autotuned layout and plan, GPU encode + {iters} CP-ALS iterations per step",
                   "nnz": t.nnz, "rank": rank, "iters": iters, "parallelism": "single GPU"},
        "mttkrp_per_mode": per_mode,
        "solves_per_s": round(1e3 / ms_step, 4),
        "fit": round(fit, 6),
        "dtype_solve": "f64",
        "autotune": tune,
        "roofline": roofline,
    }
    # full-size MTTKRP of every mode (GPU outputs; compared with the oracle in
    # the cpu_baseline leg below)
    th = t.to_host()
    Fh = [f.cpu().numpy() for f in F0]
    checks = []  # (where, host tensor, host factors, host outputs)
    if not args.no_check:
        line = mttkrp_line(spt, t, F0, rank, reps=3, layout=layout, plan=plan)
        checks.append((out, th, Fh, [o.cpu().numpy() for o in line["outs"]]))
        del line
    if args.workload != "ratings" and not args.no_extra:
        tr, Fr, rr, _ = synth.config_device("ratings")
        r = mttkrp_line(spt, tr, Fr, rr)
        extra = {"workload": "ratings-shaped 3-mode tensor 480000x18000x2000, 100M nonzeros, rank 32, ALTO layout",
                 "mttkrp_per_mode": r["per_mode"]}
        if not args.no_check:
            checks.append((extra, tr.to_host(), [f.cpu().numpy() for f in Fr], [o.cpu().numpy() for o in r["outs"]]))
        out["ratings"] = extra
        del r, tr, Fr
    if not args.no_cpu_baseline:
        # the cpu_baseline leg: the oracle timed on a bounded sample of the
        # workload, and the oracle's rows for sampled output rows of every mode
        # against the GPU outputs above
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(th, Fh)
        for where, h_t, h_f, h_outs in checks:
            where["error_vs_oracle"] = sampled_errors(h_t, h_f, h_outs)
            where["error_vs_oracle"]["metric"] = ("max_i |gpu - oracle|_inf / |MTTKRP(|X|,|C|)_i|_inf over sampled "
                                                  "rows (the hottest, a few by hotness rank, random), FP64 oracle")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
