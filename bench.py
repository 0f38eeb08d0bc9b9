"""Benchmark: encode + CP-ALS of the 3-mode ratings-shaped tensor on one MI355X.

Workload (synthetic, seeded): 480,000 x 18,000 x 2,000, 100M distinct nonzeros,
mode-0/1 labels Zipf(1.1), mode-2 uniform, values uniform on {1..5}, rank 32,
20 CP-ALS iterations.  One step = one whole solve from the COO tensor resident
in HBM: GPU encoding (bit deposit + radix sort) followed by 20 CP-ALS
iterations (all-mode MTTKRP, FP64 Gram/Cholesky/solve, FP64 fit).

Printed metric: MTTKRP Gnnz/s per mode over the whole step
(nnz * modes * iterations / step time).  Extra fields: the MTTKRP kernels alone
(HIP events around every launch), the roofline of the MTTKRP kernel, solves/s,
and the FP64 oracle timed on a bounded sample on the host.
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
PMC_FILE = os.path.join(ROOT, "profiles", "mttkrp_ratings_hbm_traffic.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2509_00280_amd", "csrc", "mttkrp.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(t, rank: int, mode: int) -> int:
    """Compulsory HBM bytes of one mode-n MTTKRP: the key/value stream once (12 B per
    nonzero with 64-bit keys), every factor row that some nonzero touches read once,
    and the output written once."""
    kw = 8 if sum((int(d) - 1).bit_length() for d in t.dims) <= 64 else 16
    b = t.nnz * (kw + 4)
    for k, d in enumerate(t.dims):
        used = int(np.count_nonzero(np.bincount(t.coords[k], minlength=d)))
        if k == mode:
            b += int(d) * rank * 4
        else:
            b += used * rank * 4
    return b


def cpu_baseline(t, factors, budget_s: float = 20.0):
    """The FP64 oracle MTTKRP (single thread, as it stands) on a bounded sample."""
    import oracle
    n = min(t.nnz, 40_000_000)
    sample = slice(0, n)
    c = np.ascontiguousarray(t.coords[:, sample])
    v = np.ascontiguousarray(t.vals[sample])
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
    return {"value": round(done / el / 1e9, 6), "unit": "Gnnz/s per mode", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {t.nnz} nonzeros (input order), FP64 oracle MTTKRP, {modes} mode(s), "
                      f"{el:.1f} s on 1 thread of {os.cpu_count()} host cores"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nnz", type=float, default=None, help="scale the tensor down (debug only; not the benchmark)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
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
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2509_00280_amd import spt, synth

    t0 = time.time()
    t, F, rank, iters = synth.config("ratings", nnz=None if args.nnz is None else int(args.nnz))
    log(f"generated {t.nnz} nonzeros in {time.time() - t0:.1f} s")
    dev = torch.device("cuda:0")
    coords = torch.from_numpy(t.coords.view(np.int32)).to(dev)
    vals = torch.from_numpy(t.vals).to(dev)
    F0 = [torch.from_numpy(f).to(dev) for f in F]
    Fw = [torch.empty_like(f) for f in F0]
    lam = torch.empty(rank, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    nm = t.nmodes

    def step():
        for a, b in zip(Fw, F0):
            a.copy_(b)
        h = spt.encode(t.dims, coords, vals)
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
    ms_step = el * 1e3 / args.steps
    value = t.nnz * nm * iters / (ms_step * 1e-3) / 1e9
    log(f"{args.steps} steps in {el:.3f} s: {ms_step:.2f} ms/step, fit {fit:.6f}")

    # MTTKRP kernels alone (HIP events on the library's stream around every launch)
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
    if os.path.exists(PMC_FILE):
        pmc = {}
        with open(PMC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    pmc[k.strip()] = v.strip()
        if pmc.get("source_digest") == source_digest() and pmc.get("nnz") == str(t.nnz):
            traffic = float(pmc["hbm_bytes_per_launch"])
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "mttkrp", "algorithmic_bytes_per_launch": int(alg_avg),
                "avg_launch_ms": round(mk_ms, 4)}
    out = {
        "metric": "MTTKRP Gnnz/s per mode", "value": round(value, 3), "unit": "Gnnz/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ratings-shaped 3-mode tensor {'x'.join(map(str, t.dims))}, {t.nnz} nonzeros, "
                               f"Zipf(1.1)/Zipf(1.1)/uniform labels, values in 1..5, rank {rank}, "
                               f"GPU encode + {iters} CP-ALS iterations per step",
                   "nnz": t.nnz, "rank": rank, "iters": iters, "parallelism": "single GPU"},
        "mttkrp_per_mode": per_mode,
        "solves_per_s": round(1e3 / ms_step, 4),
        "fit": round(fit, 6),
        "dtype_solve": "f64",
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(t, F)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
