#!/usr/bin/env python3
"""Benchmark of the SPED hot path on one MI355X.

Workload: stochastic block model, 10^6 nodes in 100 equal blocks, mean degree
20 with 5% of edges between blocks, symmetric normalised Laplacian (float32
values, int32 columns, int64 row pointers), a 32-column float32 block and the
degree-16 limit polynomial M = (I - L/16)^16.

One step = one pass of the whole hot path over the resident block Q:
  1. W = M Q exactly: 16 fused sparse-times-block launches;
  2. the walk estimate of M Q, 8 importance-sampled walks per row;
  3. Cholesky QR2 of W (float64 Gram on the matrix cores, 32x32 Cholesky);
  4. Rayleigh-Ritz on L with residuals (one more sparse product, Gram,
     Jacobi, two rotations); Q <- Ritz vectors.
`value` is the p(L)V bandwidth: algorithmic bytes of one exact application
divided by its time, measured with events around step 1 inside every timed
step.  The roofline object prices one sparse step launch; `cpu_baseline` times
the float64 oracle on the host's cores (column slices on up to 16 threads,
median of 3) on full applications of the same workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                  [--no-solve]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "p(L)·V GB/s (% HBM peak); time to bottom-k at 1e-6, SPED vs plain L"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmm_sbm1m_k32_traffic.json")
SPMM_SRC = os.path.join(ROOT, "paper_2207_14589_amd", "csrc", "spmm.hip")


def spmm_step_bytes(n, nnz, k, horner=False, b_val=4, b_u=4):
    """Compulsory bytes of one fused step: row pointers, column ids and values
    once, the block read once and written once (Horner also reads X once),
    plus the diagonal."""
    return 8 * (n + 1) + nnz * (4 + b_val) + 4 * n + n * k * (2 * b_u + (b_u if horner else 0))


def kernel_source_hash():
    with open(SPMM_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(per_launch_alg):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


COPY_BYTES = 512 * 1024 * 1024


def traffic_probe(args):
    """Workload for the counter runs: 3 plain copies of COPY_BYTES (the
    calibration kernel), then 2 exact applications (32 fused-step launches)."""
    import numpy as np
    import torch

    from paper_2207_14589_amd import sped, synth

    n, s, d, _ = synth.sbm_from_degrees(1_000_000, 100, 19.0, 1.0, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    Q = torch.from_numpy(synth.gaussian_block(n, 32, 2).astype(np.float32)).cuda()
    W = torch.empty_like(Q)
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        sped.stream_copy(a, b)
    p = sped.transform("limit", 16)
    for _ in range(2):
        sped.apply_poly(L, p, Q, out=W)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "done", "n": L.n, "nnz": L.nnz}), flush=True)


def write_traffic(fetch_db, write_db):
    """Turn two rocprofv3 --pmc databases (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) into HBM bytes per fused-step launch, each counter scaled by what
    it reads for the plain copy kernel of known size."""
    import sqlite3

    def per_kernel(db, counter):
        c = sqlite3.connect(db)
        rows = c.execute("select name, avg(counter_value), count(*) from pmc_events where counter_name = ? "
                         "group by name", (counter,)).fetchall()
        out = {}
        for name, v, cnt in rows:
            if "copy_kernel" in name:
                out["copy"] = v
            elif "spmm_light" in name:
                out["spmm"] = v
        return out

    f = per_kernel(fetch_db, "FETCH_SIZE")
    w = per_kernel(write_db, "WRITE_SIZE")
    f_scale = COPY_BYTES / f["copy"]
    w_scale = COPY_BYTES / w["copy"]
    fetch = f["spmm"] * f_scale
    write = w["spmm"] * w_scale
    out = {"kernel": "spmm_light (fused sparse step), SBM n=1e6, k=32, float32",
           "kernel_sha": kernel_source_hash(),
           "copy_bytes": COPY_BYTES,
           "copy_fetch_kib": f["copy"], "copy_write_kib": w["copy"],
           "fetch_scale": f_scale, "write_scale": w_scale,
           "spmm_fetch_kib": f["spmm"], "spmm_write_kib": w["spmm"],
           "hbm_fetch_bytes_per_launch": fetch, "hbm_write_bytes_per_launch": write,
           "hbm_bytes_per_launch": fetch + write}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def mfma_summary(db):
    """Per-kernel MFMA use from a rocprofv3 --pmc database holding
    SQ_VALU_MFMA_BUSY_CYCLES, SQ_INSTS_VALU_MFMA_MOPS_F64/_F32 and
    GRBM_GUI_ACTIVE: the SQ counters arrive once per shader engine and are
    summed per dispatch; busy % = busy cycles / (GUI-active cycles x 1024
    SIMDs); flops = MOPS x 512."""
    import collections
    import sqlite3

    con = sqlite3.connect(db)
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    meta = {}
    for did, name, cn, v, d in con.execute(
            "select dispatch_id, name, counter_name, counter_value, duration from pmc_events"):
        per[did][cn].append(v)
        meta[did] = (name, d)
    agg = collections.defaultdict(list)
    for did, cs in per.items():
        name, d = meta[did]
        nm = name.replace("sped::(anonymous namespace)::", "").replace("void ", "")
        nm = nm[:nm.index("(")] if "(" in nm else nm
        agg[nm].append((sum(cs.get("SQ_VALU_MFMA_BUSY_CYCLES", [0])), max(cs.get("GRBM_GUI_ACTIVE", [1])),
                        512 * sum(cs.get("SQ_INSTS_VALU_MFMA_MOPS_F64", [0])),
                        512 * sum(cs.get("SQ_INSTS_VALU_MFMA_MOPS_F32", [0])), d))
    print("| kernel | dispatches | MFMA busy (% of SIMD-cycles) | FP64 MFMA flop / dispatch | "
          "FP32 MFMA flop / dispatch | avg duration us | achieved MFMA TFLOP/s |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for nm, recs in sorted(agg.items(), key=lambda kv: -sum(r[2] + r[3] for r in kv[1])):
        m = len(recs)
        flops = sum(r[2] + r[3] for r in recs) / m
        if flops == 0:
            continue
        util = 100.0 * sum(r[0] for r in recs) / sum(r[1] * 1024 for r in recs)
        dur = sum(r[4] for r in recs) / m
        print(f"| `{nm}` | {m} | {util:.2f} | {sum(r[2] for r in recs) / m:.3e} | "
              f"{sum(r[3] for r in recs) / m:.3e} | {dur / 1e3:.1f} | {flops / dur / 1e3:.2f} |")


def locality_sweep():
    """Per-launch time of the fused step on SBMs of 1e6 nodes and mean degree
    20 whose block size sets how local each row's neighbourhood is, plus a
    plain copy of the same compulsory byte count."""
    import numpy as np
    import torch

    from paper_2207_14589_amd import sped, synth

    n = 1_000_000
    X = torch.from_numpy(synth.gaussian_block(n, 32, 2).astype(np.float32)).cuda()
    Y = torch.empty_like(X)
    p = sped.transform("limit", 16)
    for bs in (125, 1000, 10000, 100000, 1000000):
        if bs < n:
            _, s, d, _ = synth.sbm_from_degrees(n, n // bs, 19.0, 1.0, seed=1)
        else:
            _, s, d, _ = synth.sbm_sparse([n], 20.0 / (n - 1), 0.0, seed=1)
        L = sped.Laplacian(n, s, d, kind="sym")
        for _ in range(2):
            sped.apply_poly(L, p, X, out=Y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            sped.apply_poly(L, p, X, out=Y)
        e1.record()
        torch.cuda.synchronize()
        print(json.dumps({"block": bs, "nnz": L.nnz, "step_us": round(e0.elapsed_time(e1) * 100 / 16, 2)}),
              flush=True)
        del L
    nbytes = spmm_step_bytes(n, 20_000_000, 32) // 16 * 16
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        sped.stream_copy(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(20):
        sped.stream_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1000 / 20
    print(json.dumps({"copy_bytes_each_way": nbytes, "copy_us": round(us, 2),
                      "copy_GBps_read_plus_write": round(2 * nbytes / us / 1e3, 1)}), flush=True)


def sstep_sweep():
    """The degree-16 limit chain on 10^6-node SBMs (mean degree 20, k = 32
    float32) whose block size is 125, 1,000 or 10,000 rows and whose mean
    degree between blocks is 1 (5% of edges), 0.1 or 0: 16 single fused steps
    against 8 launches of two steps each on
    LDS-resident row blocks (sped_apply_poly_blocked, block_rows = the block
    size, capped at 1,000), same algorithmic bytes (16 single steps)."""
    import numpy as np
    import torch

    from paper_2207_14589_amd import sped, synth

    n, ell = 1_000_000, 16
    X = torch.from_numpy(synth.gaussian_block(n, 32, 2).astype(np.float32)).cuda()
    Y = torch.empty_like(X)
    p = sped.transform("limit", ell)

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = []
    for bs, d_out in ((125, 1.0), (125, 0.1), (125, 0.0), (1000, 1.0), (1000, 0.1), (10000, 1.0)):
        _, s, d, _ = synth.sbm_from_degrees(n, n // bs, 20.0 - d_out, d_out, seed=1)
        L = sped.Laplacian(n, s, d, kind="sym", walk_records=False)
        B = min(bs, 1000)
        single = timed(lambda: sped.apply_poly(L, p, X, out=Y))
        ref = Y.clone()
        fused = timed(lambda: sped.apply_poly_blocked(L, p, X, B, out=Y))
        alg = ell * spmm_step_bytes(L.n, L.nnz, 32)
        row = {"block": bs, "cross_degree": d_out, "block_rows": B, "nnz": L.nnz, "single_steps_ms": round(single, 4),
               "two_step_launches_ms": round(fused, 4), "speedup": round(single / fused, 3),
               "single_GBps": round(alg / single / 1e6, 1), "two_step_GBps": round(alg / fused / 1e6, 1),
               "rel_diff": float((Y - ref).norm() / ref.norm())}
        print(json.dumps(row), flush=True)
        out.append(row)
        del L
    return out


def _host_info():
    """Host cores, CPU model and RAM, read from the OS."""
    import os

    model, mem_gb = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model,
            "ram_GiB": mem_gb}


def cpu_baseline_leg(n, s, d, X, ell, alg_bytes, runs=3):
    """The oracle's (I - L/l)^l V, unchanged, on the host's cores: the block's
    columns are independent, so W threads each run the oracle on a slice of
    columns (scipy's sparse products release the interpreter lock) and the
    slices are joined; the result equals the one-thread call exactly.  Median
    of `runs` full applications."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    from oracle import laplacian as olap
    from oracle import poly as opoly

    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    Xd = X.astype(np.float64)
    k = Xd.shape[1]
    # the machine's CPU share for one GPU is 16 threads
    workers = max(1, min(16, len(os.sched_getaffinity(0)), k))
    slices = [np.ascontiguousarray(Xd[:, c]) for c in np.array_split(np.arange(k), workers)]
    times = []
    with ThreadPoolExecutor(workers) as ex:
        for _ in range(runs):
            t0 = time.perf_counter()
            parts = list(ex.map(lambda V: opoly.apply_limit_product(ref.L, ell, V), slices))
            np.concatenate(parts, axis=1)
            times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    return {"value": round(ell * alg_bytes / med / 1e9, 4), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "seconds_median": round(med, 3), "seconds_each": [round(t, 3) for t in times],
            "host": _host_info(),
            "sample": f"median of {runs} full degree-{ell} applications (I - L/{ell})^{ell} V on the same "
                      f"{n}-node graph, {k} columns in {workers} column slices on {workers} threads, "
                      f"float64 scipy CSR products"}


def time_to_tolerance(sped, synth, torch, np):
    """SPED (limit, l = 8) against the plain operator 2I - L, same solver,
    cadence and precision: 2,000-node SBM with 10 blocks, bottom 10.  Also
    degree-8 coefficients tuned by gradient descent through PolyApply on
    another 2,000-node SBM of the same family (seed 5; the tuning time is
    reported beside the solves), with the largest difference of its Ritz
    values from plain L's (the same bottom-10 subspace, not another invariant
    one)."""
    from paper_2207_14589_amd import tune

    k, guard, ell = 10, 4, 8
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=5)
    Lp = sped.Laplacian(n, s, d, kind="sym")
    Vt = torch.from_numpy(synth.gaussian_block(n, k + guard, 7).astype(np.float32)).cuda()
    tune.tune_coefficients(Lp, k, ell, Vt, steps=2, unroll=3)  # warm the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, hist = tune.tune_coefficients(Lp, k, ell, Vt, steps=60, unroll=3)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    del Lp, Vt
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    V0 = torch.from_numpy(synth.gaussian_block(n, k + guard, 2).astype(np.float32)).cuda()
    out = {"workload": "SBM n=2000, 10 blocks, p_in=0.05, p_out=0.0005, k=10 (+4 guard), tol 1e-6",
           "tuning": {"graph": "SBM n=2000 of the same family (seed 5)", "degree": ell, "seconds": round(tune_s, 3),
                      "steps": len(hist), "loss_first": hist[0], "loss_best": min(hist)}}
    evals = {}
    for name, p, polish in (("sped_limit8", sped.transform("limit", ell), 0), ("plain", None, 0),
                            ("sped_tuned8", sped.monomial(theta, shift=1.0, scale=1.0), 2)):
        sped.bottomk(L, k, p, V0=V0, guard=guard, tol=1e-6, max_iters=5000, polish=polish)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=1e-6, max_iters=5000, polish=polish)
        dt = time.perf_counter() - t0
        evals[name] = np.asarray(r.evals, dtype=np.float64)
        out[name] = {"seconds": round(dt, 5), "iters": r.stats["iters"], "spmm": r.stats["spmm_count"],
                     "polish_iters": r.stats["polish_iters"], "converged": bool(r.converged),
                     "bound": r.stats["bound"]}
    out["sped_tuned8"]["evals_max_abs_diff_vs_plain"] = float(np.abs(evals["sped_tuned8"] - evals["plain"]).max())
    out["speedup_sped_vs_plain"] = round(out["plain"]["seconds"] / out["sped_limit8"]["seconds"], 3)
    out["speedup_tuned_vs_plain"] = round(out["plain"]["seconds"] / out["sped_tuned8"]["seconds"], 3)
    return out


def gather_probe(sped, torch):
    """The chip's rate for the sparse step's load pattern (sped_gather_probe):
    128-byte rows, 8 lanes x 16 bytes per row, 8 rows per instruction, from
    tables that fit L1, one XCD's L2, or neither; scattered rows against 1 KB
    contiguous reads.  Rates in TB/s and in 128-byte lines per clock per CU
    (256 CUs at 2.4 GHz)."""
    blocks, iters = 2048, 4096
    out_buf = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    res = []
    for rows in (128, 16384, 262144):
        table = torch.zeros(rows, 32, dtype=torch.float32, device="cuda")
        for scattered in (True, False):
            sped.gather_probe(table, iters, scattered, blocks, out_buf)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            sped.gather_probe(table, iters, scattered, blocks, out_buf)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            nbytes = blocks * 256 * iters * 16
            res.append({"table_kb": rows * 128 // 1024, "pattern": "scattered rows" if scattered else "contiguous 1 KB",
                        "ms": round(ms, 3), "TBps": round(nbytes / (ms * 1e-3) / 1e12, 2),
                        "lines_per_clk_per_cu": round(nbytes / 128 / (ms * 1e-3 * 2.4e9) / 256, 3)})
        del table
    return res


def time_to_tolerance_powerlaw200k(sped, synth, torch, np):
    """A power-law graph with planted communities at solver scale: Chung-Lu
    n = 2e5 (exponent 2.1, mean degree 16, 64 communities, 95% of draws
    inside), largest component, symmetric normalised L; bottom 64 (+8 guard)
    with bf16 storage and the float32 refinement, to the 1e-5 bound (the
    float32 floor of this graph, bottom gap 0.09, is near 2e-6); plain L
    against the degree-16 limit polynomial and degree-12 coefficients tuned
    by gradient descent through PolyApply on a 2e4-node graph of the same
    family (tuning time reported), same solver and cadence."""
    from paper_2207_14589_amd import tune

    k, guard, ell = 64, 8, 12
    n, s, d, _ = synth.chung_lu(20_000, 2.1, 16.0, 64, 0.95, seed=5)
    Lp = sped.Laplacian(n, s, d, kind="sym", lcc=True)
    Vt = torch.from_numpy(synth.gaussian_block(Lp.n, k + guard, 7).astype(np.float32)).cuda()
    tune.tune_coefficients(Lp, k, ell, Vt, steps=2, unroll=3)  # warm the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, hist = tune.tune_coefficients(Lp, k, ell, Vt, steps=60, unroll=3)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    del Lp, Vt
    n, s, d, _ = synth.chung_lu(200_000, 2.1, 16.0, 64, 0.95, seed=3)
    L = sped.Laplacian(n, s, d, kind="sym", lcc=True, walk_records=False)
    V0 = synth.gaussian_block_device(L.n, 72, seed=2)
    out = {"workload": "Chung-Lu n=2e5, exponent 2.1, mean degree 16, 64 communities; largest component; "
                       "k=64 (+8 guard), bf16 storage + float32 refinement, tol 1e-5 and 1e-6 "
                       "(the polynomial runs end with plain iterations once their float32 floor stalls them)",
           "n_lcc": L.n, "nnz": L.nnz,
           "tuning": {"graph": "Chung-Lu n=2e4 of the same family (largest component)", "degree": ell,
                      "seconds": round(tune_s, 3), "steps": len(hist), "loss_first": hist[0],
                      "loss_best": min(hist)}}
    for tol in (1e-5, 1e-6):
        for name, p in (("plain", None), ("sped_limit16", sped.transform("limit", 16)),
                        ("sped_tuned12", sped.monomial(theta, shift=1.0, scale=1.0))):
            kw = dict(guard=8, tol=tol, max_iters=3000, storage="bf16", polish=2 if p is not None else 0)
            sped.bottomk(L, 64, p, V0=V0, **kw)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sped.bottomk(L, 64, p, V0=V0, **kw)
            dt = time.perf_counter() - t0
            out[f"{name}_{tol:g}"] = {"seconds": round(dt, 4), "iters": r.stats["iters"],
                                      "bf16_iters": r.stats["coarse_iters"], "polish_iters": r.stats["polish_iters"],
                                      "spmm": r.stats["spmm_count"], "converged": bool(r.converged),
                                      "bound": r.stats["bound"]}
        out[f"speedup_sped_vs_plain_{tol:g}"] = round(out[f"plain_{tol:g}"]["seconds"] /
                                                      out[f"sped_limit16_{tol:g}"]["seconds"], 3)
        out[f"speedup_tuned_vs_plain_{tol:g}"] = round(out[f"plain_{tol:g}"]["seconds"] /
                                                       out[f"sped_tuned12_{tol:g}"]["seconds"], 3)
    return out


def polyapply_sbm500k(sped, synth, torch, np):
    """The learnable-coefficient workload: 500k-node SBM (50 blocks, mean
    degree 24, 5% cross), k = 50, degree 12, float32.  Times PolyApply's
    forward (Horner: 12 fused steps that also re-read X) and backward (dX by
    the same Horner chain on dY; dtheta by 12 recomputed powers with the fused
    float64 inner product), each with its algorithmic bytes."""
    from paper_2207_14589_amd.autograd import poly_apply

    n, s, d, _ = synth.sbm_from_degrees(500_000, 50, 22.8, 1.2, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym", walk_records=False)
    k, ell = 50, 12
    g = torch.Generator(device="cpu").manual_seed(5)
    theta = (torch.randn(ell + 1, generator=g, dtype=torch.float64) * 0.3).requires_grad_(True)
    X = synth.gaussian_block_device(L.n, k, seed=6).requires_grad_(True)
    dY = synth.gaussian_block_device(L.n, k, seed=7)

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    Y = poly_apply(theta, X, L, 1.0, 1.0)
    fwd_ms = timed(lambda: poly_apply(theta, X, L, 1.0, 1.0))
    bwd_ms = timed(lambda: torch.autograd.grad(Y, (theta, X), dY, retain_graph=True))
    idx = 8 * (L.n + 1) + L.nnz * 8 + 4 * L.n
    horner = ell * (idx + L.n * k * 12)                          # U in, O out, X re-read
    fwd_bytes = horner
    bwd_bytes = horner + ell * (idx + L.n * k * 12) + L.n * k * 8  # dX chain; powers with dY dot; first dot
    return {"workload": "SBM n=5e5, 50 blocks, mean degree 24, 5% cross; k=50, degree 12, float32",
            "forward_ms": round(fwd_ms, 4), "forward_GBps": round(fwd_bytes / (fwd_ms * 1e-3) / 1e9, 1),
            "backward_ms": round(bwd_ms, 4), "backward_GBps": round(bwd_bytes / (bwd_ms * 1e-3) / 1e9, 1)}


def time_to_tolerance_combinatorial(sped, synth, torch, np):
    """The combinatorial Laplacian, whose spectrum reaches 2 d_max: plain
    iteration on lambda_bound I - L contracts the unwanted directions by only
    1 - gap / lambda_bound per step, while (I - L/l)^l with 2l > lambda_bound
    (the smallest multiple of 16 that satisfies it) contracts them by about
    e^{-gap}.  Same solver, cadence and float32 precision; tolerances 1e-5
    and 1e-6 on the residual bound (the plain operator's float32 floor,
    lambda_bound / gap times the rounding, lies near 1e-6 here; the polynomial
    runs may hand over to plain iterations when they stall); 2,000-node and
    500k-node SBMs."""
    out = {}
    cases = (("sbm2000", lambda: synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1), 10, 4, 5000),
             ("sbm500k", lambda: synth.sbm_from_degrees(500_000, 50, 22.8, 1.2, seed=1), 50, 6, 3000))
    for tag, gen, k, guard, cap in cases:
        n, s, d, _ = gen()
        L = sped.Laplacian(n, s, d, kind="combinatorial")
        ell = 16 * int(np.ceil((L.lambda_bound / 2 + 1) / 16))
        V0 = torch.from_numpy(synth.gaussian_block(n, k + guard, 2).astype(np.float32)).cuda()
        row = {"n": L.n, "k": k, "guard": guard, "lambda_bound": L.lambda_bound, "ell": ell}
        for tol in (1e-5, 1e-6):
            for name, p in (("plain", None), (f"sped_limit{ell}", sped.transform("limit", ell, L.lambda_bound))):
                kw = dict(guard=guard, tol=tol, max_iters=cap, polish=2 if p is not None else 0)
                if tol == 1e-5:
                    sped.bottomk(L, k, p, V0=V0, **kw)  # warm
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = sped.bottomk(L, k, p, V0=V0, **kw)
                dt = time.perf_counter() - t0
                row[f"{name}_{tol:g}"] = {"seconds": round(dt, 5), "iters": r.stats["iters"],
                                          "polish_iters": r.stats["polish_iters"], "spmm": r.stats["spmm_count"],
                                          "converged": bool(r.converged), "bound": r.stats["bound"]}
            row[f"speedup_sped_vs_plain_{tol:g}"] = round(row[f"plain_{tol:g}"]["seconds"] /
                                                          row[f"sped_limit{ell}_{tol:g}"]["seconds"], 3)
        out[tag] = row
        del L, V0
        torch.cuda.empty_cache()
    return out


def time_to_tolerance_sbm500k(sped, synth, torch, np, tol=1e-6):
    """500k-node SBM (50 blocks, mean degree 24, 5% cross), bottom 50 (+6
    guard) to the 1e-6 bound with the same solver, cadence and precision for:
    the plain operator 2I - L, the degree-12 limit polynomial, and degree-12
    coefficients tuned by gradient descent through PolyApply.  The polynomial
    runs hand over to plain iterations once their float32 floor stalls them
    (polish_checks = 2).  The coefficients are tuned once on a 25k-node graph
    of the same family (same blocks count and degrees, so the same spectrum
    shape) and that time is reported beside the solves."""
    from paper_2207_14589_amd import tune

    k, guard, ell = 50, 6, 12
    n, s, d, _ = synth.sbm_from_degrees(25_000, 50, 22.8, 1.2, seed=5)
    Lp = sped.Laplacian(n, s, d, kind="sym")
    Vt = torch.from_numpy(synth.gaussian_block(n, k + guard, 7).astype(np.float32)).cuda()
    tune.tune_coefficients(Lp, k, ell, Vt, steps=2, unroll=3)  # warm the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, hist = tune.tune_coefficients(Lp, k, ell, Vt, steps=60, unroll=3)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    del Lp, Vt
    n, s, d, _ = synth.sbm_from_degrees(500_000, 50, 22.8, 1.2, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    V0 = torch.from_numpy(synth.gaussian_block(n, k + guard, 2).astype(np.float32)).cuda()
    out = {"workload": f"SBM n=5e5, 50 blocks, mean degree 24, 5% cross; k=50 (+6 guard), tol {tol:g}",
           "tuning": {"graph": "SBM n=2.5e4 of the same family", "seconds": round(tune_s, 3), "steps": len(hist),
                      "loss_first": hist[0], "loss_best": min(hist), "theta": [float(x) for x in theta]}}
    ops = (("plain", None, 0), ("sped_limit12", sped.transform("limit", ell), 2),
           ("sped_tuned12", sped.monomial(theta, shift=1.0, scale=1.0), 2))
    for name, p, polish in ops:
        sped.bottomk(L, k, p, V0=V0, guard=guard, tol=tol, max_iters=4000, polish=polish)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=tol, max_iters=4000, polish=polish)
        dt = time.perf_counter() - t0
        out[name] = {"seconds": round(dt, 4), "iters": r.stats["iters"], "polish_iters": r.stats["polish_iters"],
                     "spmm": r.stats["spmm_count"], "converged": bool(r.converged), "bound": r.stats["bound"],
                     "gap_estimate": r.stats["gap_estimate"]}
    pl = out["plain"]["seconds"]
    out["speedup_limit_vs_plain"] = round(pl / out["sped_limit12"]["seconds"], 3)
    out["speedup_tuned_vs_plain"] = round(pl / out["sped_tuned12"]["seconds"], 3)
    out["speedup_tuned_vs_plain_with_tuning"] = round(pl / (out["sped_tuned12"]["seconds"] + tune_s), 3)
    return out


def mu_eg_streak_sbm2000(sped, synth, torch, np):
    """mu-EigenGame on the 2,000-node SBM (k = 10 + 4 guard players): the
    eigenvector streak (Sec. 5.2, eps = pi/8) against the dense eigenvectors
    after T iterations, for the plain operator 2I - L and the degree-8 limit
    operator, each with step 0.5 / rho(M) (rho = 2 and 1).  Every point is a
    fresh deterministic run of T iterations from the same start block."""
    from paper_2207_14589_amd import metrics

    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    rowptr, col, val, diag, _ = L.host_csr()
    Ld = np.diag(diag.astype(np.float64))
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    Ld[rows, col] -= val.astype(np.float64)
    lam, U = np.linalg.eigh(Ld)
    k, guard = 10, 4
    Uref = torch.from_numpy(U[:, :k].astype(np.float32)).cuda()
    V0 = torch.from_numpy(synth.gaussian_block(n, k + guard, 2).astype(np.float32)).cuda()
    checkpoints = [10, 40, 160, 640, 2560, 10240]
    out = {"workload": "SBM n=2000, 10 blocks, k=10 (+4 guard players); streak eps = pi/8",
           "checkpoints": checkpoints}
    for name, p, eta in (("plain", None, 0.25), ("sped_limit8", sped.transform("limit", 8), 0.5)):
        streaks, secs = [], []
        for T in checkpoints:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=0.0, max_iters=T, check_every=T, solver="mu_eg",
                             eta=eta)
            secs.append(round(time.perf_counter() - t0, 4))
            streaks.append(metrics.eigenvector_streak(Uref, r.V))
        full = [T for T, st in zip(checkpoints, streaks) if st == k]
        out[name] = {"eta": eta, "streak": streaks, "seconds": secs, "first_full_streak_iters": full[0] if full else None}
    return out


def _dense_lap(L, np):
    rowptr, col, val, diag, _ = L.host_csr()
    n = L.n
    Ld = np.diag(diag.astype(np.float64))
    Ld[np.repeat(np.arange(n), np.diff(rowptr)), col] -= val.astype(np.float64)
    return np.linalg.eigh(Ld)


def _sin_angle(U, V, np):
    Q, _ = np.linalg.qr(V.astype(np.float64))
    return float(np.linalg.norm(Q - U @ (U.T @ Q), 2))


def rmat26_solver(sped, synth, torch, np, budget_s=20.0):
    """The R-MAT workload at its full shape: scale 26 (2^26 nodes, edge factor
    16, a, b, c = 0.57, 0.19, 0.19, seeded vertex permutation), drawn on the
    device, largest component, symmetric normalised L; bottom 64 (+8 guard)
    with bf16 iterate storage.  Each operator runs from the same start block
    for about `budget_s` seconds (an iteration cap from a one-iteration probe)
    and records its bound and largest residual at every check: the plain
    operator, the exact degree-16 limit polynomial, the same polynomial
    estimated by lazy node walks (8 per row) for the first 3/4 of the
    iterations, then exact, and degree-12 coefficients tuned through
    PolyApply on R-MAT scale 16.  Prints one progress line per stage."""
    t0 = time.perf_counter()
    n0, src, dst = synth.rmat_device(26, 16, 0.57, 0.19, 0.19, seed=1)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    print(json.dumps({"rmat26": "generated", "edges": int(src.numel()), "seconds": round(gen_s, 2)}), flush=True)
    t0 = time.perf_counter()
    L = sped.Laplacian(n0, src, dst, kind="sym", lcc=True, walk_records=False)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    del src, dst
    torch.cuda.empty_cache()
    print(json.dumps({"rmat26": "built", "n_lcc": L.n, "nnz": L.nnz, "seconds": round(build_s, 2)}), flush=True)
    k, guard = 64, 8
    V0 = synth.gaussian_block_device(L.n, k + guard, seed=2)
    out = {"workload": "R-MAT scale 26, edge factor 16 (0.57, 0.19, 0.19), device draw; largest component; "
                       "sym-normalised L; bottom 64 (+8 guard), bf16 iterate storage, checks every iteration",
           "n_lcc": L.n, "nnz": L.nnz, "max_degree": L.max_degree, "generate_s": round(gen_s, 2),
           "build_s": round(build_s, 2), "budget_s": budget_s}
    # degree-12 coefficients tuned once on R-MAT scale 16 (same parameters,
    # largest component)
    from paper_2207_14589_amd import tune
    n1, s1, d1 = synth.rmat(16, 16, 0.57, 0.19, 0.19, seed=5)
    Lp = sped.Laplacian(n1, s1, d1, kind="sym", lcc=True)
    Vt = torch.from_numpy(synth.gaussian_block(Lp.n, k + guard, 7).astype(np.float32)).cuda()
    tune.tune_coefficients(Lp, k, 12, Vt, steps=2, unroll=3)  # warm the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, hist = tune.tune_coefficients(Lp, k, 12, Vt, steps=60, unroll=3)
    torch.cuda.synchronize()
    out["tuning"] = {"graph": "R-MAT scale 16 of the same parameters (largest component)", "n_lcc": Lp.n,
                     "degree": 12, "seconds": round(time.perf_counter() - t0, 3), "loss_first": hist[0],
                     "loss_best": min(hist)}
    del Lp, Vt
    print(json.dumps({"rmat26": "tuned", **out["tuning"]}), flush=True)
    p16 = sped.transform("limit", 16)
    runs = (("plain", None, {}), ("sped_limit16_exact", p16, {}),
            ("sped_limit16_lazy_then_exact", p16, {"walks_per_row": 8, "sampler": "lazy"}),
            ("sped_tuned12_exact", sped.monomial(theta, shift=1.0, scale=1.0), {}))
    for name, p, kw in runs:
        kw = dict(kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sped.bottomk(L, k, p, V0=V0, guard=guard, tol=0.0, max_iters=1, storage="bf16",
                     **({"stochastic_iters": 1} if "sampler" in kw else {}), **kw)
        torch.cuda.synchronize()
        per = time.perf_counter() - t0
        iters = max(2, int(budget_s / per))
        if "sampler" in kw:
            kw["stochastic_iters"] = (3 * iters) // 4
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=0.0, max_iters=iters, storage="bf16",
                         coarse_tol=1e-30, trace_cap=iters + 1, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tr = r.stats["trace"]
        out[name] = {"iters": r.stats["iters"], "seconds": round(dt, 3),
                     "seconds_per_iter": round(dt / max(r.stats["iters"], 1), 4), "spmm": r.stats["spmm_count"],
                     "bound": r.stats["bound"], "gap_estimate": r.stats["gap_estimate"],
                     "max_residual": r.stats["max_residual"],
                     "trace_iter_s_bound_maxres": [[int(a), round(b, 3), c, round(d, 6)] for a, b, c, d in tr]}
        print(json.dumps({"rmat26": name, **{x: y for x, y in out[name].items() if x != "trace_iter_s_bound_maxres"}}),
              flush=True)
        del r
        torch.cuda.empty_cache()
    return out


def power_law_4m_solve(sped, synth, torch, np, tol=1e-5, max_iters=400):
    """The power-law workload solved at full size: Chung-Lu n = 4e6
    (exponent 2.1, mean degree 16, 256 communities, device draw), largest
    component; bottom 64 (+8 guard) with bf16 storage down to its floor, then
    the float32 refinement to `tol`; the plain operator against the degree-16
    limit polynomial and degree-12 coefficients tuned through PolyApply on a
    4e4-node graph of the same family (both hand over to plain iterations if
    their float32 floor stalls them), same solver and cadence, from one start
    block; the tuned run again on the label-propagation numbering of the same
    graph (the start block's rows permuted alike, the ordered build timed
    apart)."""
    from paper_2207_14589_amd import tune

    # degree-12 coefficients tuned once on a 4e4-node graph of the same family
    n, s, d, _ = synth.chung_lu(40_000, 2.1, 16.0, 256, 0.95, seed=5)
    Lp = sped.Laplacian(n, s, d, kind="sym", lcc=True)
    Vt = torch.from_numpy(synth.gaussian_block(Lp.n, 72, 7).astype(np.float32)).cuda()
    tune.tune_coefficients(Lp, 64, 12, Vt, steps=2, unroll=3)  # warm the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, hist = tune.tune_coefficients(Lp, 64, 12, Vt, steps=60, unroll=3)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    del Lp, Vt
    n0, src, dst = synth.chung_lu_device(4_000_000, 2.1, 16.0, 256, 0.95, seed=1)
    L = sped.Laplacian(n0, src, dst, kind="sym", lcc=True, walk_records=False)
    torch.cuda.empty_cache()
    V0 = synth.gaussian_block_device(L.n, 72, seed=2)
    out = {"workload": f"Chung-Lu n=4e6 (device draw), exponent 2.1, mean degree 16, 256 communities; largest "
                       f"component; k=64 (+8 guard), bf16 storage + float32 refinement, tol {tol:g}",
           "n_lcc": L.n, "nnz": L.nnz, "max_iters": max_iters,
           "tuning": {"graph": "Chung-Lu n=4e4 of the same family (largest component)", "degree": 12,
                      "seconds": round(tune_s, 3), "loss_first": hist[0], "loss_best": min(hist)}}
    for name, p in (("plain", None), ("sped_limit16", sped.transform("limit", 16)),
                    ("sped_tuned12", sped.monomial(theta, shift=1.0, scale=1.0))):
        kw = dict(guard=8, tol=tol, max_iters=max_iters, storage="bf16", polish=2 if p is not None else 0,
                  trace_cap=max_iters + 1)
        sped.bottomk(L, 64, p, V0=V0, guard=8, tol=0.0, max_iters=1, storage="bf16")  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sped.bottomk(L, 64, p, V0=V0, **kw)
        dt = time.perf_counter() - t0
        tr = r.stats["trace"]
        out[name] = {"seconds": round(dt, 3), "iters": r.stats["iters"], "bf16_iters": r.stats["coarse_iters"],
                     "polish_iters": r.stats["polish_iters"], "spmm": r.stats["spmm_count"],
                     "converged": bool(r.converged), "bound": r.stats["bound"],
                     "gap_estimate": r.stats["gap_estimate"],
                     "trace_every_10th": [[int(a), round(b, 3), c, round(d, 7)] for a, b, c, d in tr[::10]]}
        print(json.dumps({"power_law_4m": name, **{x: y for x, y in out[name].items() if x != "trace_every_10th"}}),
              flush=True)
    out["speedup_sped_vs_plain"] = round(out["plain"]["seconds"] / out["sped_limit16"]["seconds"], 3)
    # the tuned run on the label-propagation numbering: row j of the ordered
    # Laplacian is original node old_of_new[j], which is row where[...] of L
    where = torch.full((n0,), -1, dtype=torch.int64, device=V0.device)
    where[L.old_of_new.long()] = torch.arange(L.n, device=V0.device)
    del L
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Lo = sped.Laplacian(n0, src, dst, kind="sym", lcc=True, walk_records=False, order="label_propagation")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    del src, dst
    V0o = V0[where[Lo.old_of_new.long()]].contiguous()
    p = sped.monomial(theta, shift=1.0, scale=1.0)
    sped.bottomk(Lo, 64, p, V0=V0o, guard=8, tol=0.0, max_iters=1, storage="bf16")  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sped.bottomk(Lo, 64, p, V0=V0o, guard=8, tol=tol, max_iters=max_iters, storage="bf16", polish=2,
                     trace_cap=max_iters + 1)
    dt = time.perf_counter() - t0
    tr = r.stats["trace"]
    out["sped_tuned12_label_propagation_ids"] = {
        "ordered_build_s": round(build_s, 3), "seconds": round(dt, 3), "iters": r.stats["iters"],
        "bf16_iters": r.stats["coarse_iters"], "polish_iters": r.stats["polish_iters"], "spmm": r.stats["spmm_count"],
        "converged": bool(r.converged), "bound": r.stats["bound"], "gap_estimate": r.stats["gap_estimate"],
        "trace_every_10th": [[int(a), round(b, 3), c, round(d, 7)] for a, b, c, d in tr[::10]]}
    print(json.dumps({"power_law_4m": "sped_tuned12_label_propagation_ids",
                      **{x: y for x, y in out["sped_tuned12_label_propagation_ids"].items()
                         if x != "trace_every_10th"}}), flush=True)
    return out


def rmat26_step(sped, synth, torch, np, reps=5):
    """One fused step (L X) on the R-MAT scale-26 largest component at the
    solver's widths: 72 float32 columns (64 + 8 guard; a 288-byte row touches
    three 128-byte lines), 72 bf16 columns (two lines) and 64 bf16 columns
    (one line).  Reports the row and entry counts of the three row bins and,
    per width, the step time, its algorithmic bytes and the 128-byte lines its
    neighbour-row gathers touch (nnz x lines per row)."""
    n0, src, dst = synth.rmat_device(26, 16, 0.57, 0.19, 0.19, seed=1)
    L = sped.Laplacian(n0, src, dst, kind="sym", lcc=True, walk_records=False)
    del src, dst
    torch.cuda.empty_cache()
    rp = L.rowptr[: L.n + 1]
    deg = rp[1:] - rp[:-1]
    bins = [deg <= 128, (deg > 128) & (deg <= 8192), deg > 8192]
    out = {"workload": "R-MAT scale 26, edge factor 16 (0.57, 0.19, 0.19), device draw; largest component; "
                       "sym-normalised L; one fused step L X",
           "n_lcc": L.n, "nnz": L.nnz, "max_degree": L.max_degree,
           "bin_rows": [int(b.sum()) for b in bins], "bin_entries": [int(deg[b].sum()) for b in bins]}
    del deg, bins, rp
    one = sped.monomial([0.0, 1.0])
    for k, dt, lines in ((72, torch.float32, 3), (72, torch.bfloat16, 2), (64, torch.bfloat16, 1)):
        X = synth.gaussian_block_device(L.n, k, seed=2, dtype=dt)
        Y = torch.empty_like(X)
        sped.apply_poly(L, one, X, out=Y)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            sped.apply_poly(L, one, X, out=Y)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        eb = X.element_size()
        alg = 8 * (L.n + 1) + L.nnz * 8 + 4 * L.n + L.n * k * 2 * eb
        line_bytes = L.nnz * lines * 128
        out[f"k{k}_{str(dt).split('.')[-1]}"] = {
            "step_ms": round(ms, 3), "alg_GB": round(alg / 1e9, 2), "alg_GBps": round(alg / ms / 1e6, 1),
            "gather_lines_GB": round(line_bytes / 1e9, 1), "gather_lines_TBps": round(line_bytes / ms / 1e9, 2)}
        print(json.dumps({"rmat26_step": f"k{k}", **out[f"k{k}_{str(dt).split('.')[-1]}"]}), flush=True)
        del X, Y
        torch.cuda.empty_cache()
    return out


def _cpu_baseline_threaded(apply, X, runs):
    """Median seconds of `apply` over column slices of X on up to 16 host
    threads (scipy's sparse products release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    k = X.shape[1]
    workers = max(1, min(16, len(os.sched_getaffinity(0)), k))
    slices = [np.ascontiguousarray(X[:, c]) for c in np.array_split(np.arange(k), workers)]
    times = []
    with ThreadPoolExecutor(workers) as ex:
        for _ in range(runs):
            t0 = time.perf_counter()
            np.concatenate(list(ex.map(apply, slices)), axis=1)
            times.append(time.perf_counter() - t0)
            print(f"[oracle] run {len(times)}: {times[-1]:.3f} s", file=sys.stderr, flush=True)
    return float(np.median(times)), [round(t, 3) for t in times], workers


def cpu_baseline_workloads_leg(sped, synth, torch, np, runs=3):
    """cpu_baseline leg for the power-law and PolyApply workloads: the
    float64 oracle, unchanged, timed as a reported baseline on the host's
    cores (column slices on threads, median of
    `runs`), beside the GPU's time for the same operation:
    power-law: Chung-Lu n = 4e6, largest component, the degree-16 limit
      product (I - L/16)^16 V on 64 columns (GPU: bf16 in and out, float32
      between factors, as the solver's bf16 phase);
    SBM 500k: the degree-12 polynomial sum_i theta_i (L - I)^i X on 50
      columns by explicit powers (GPU: PolyApply's forward, float32)."""
    from oracle import laplacian as olap
    from oracle import poly as opoly
    from paper_2207_14589_amd.autograd import poly_apply

    def gpu_ms(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = {"host": _host_info()}
    # the 2,000-node SBM: the oracle's plain and SPED (limit, l = 8) subspace
    # iterations to the 1e-6 bound, one thread, against dense eigh
    from oracle import solver as osol
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    _, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = synth.gaussian_block(n, 14, 2).astype(np.float32).astype(np.float64)
    c1 = {"workload": "SBM n=2000, 10 blocks, p_in=0.05, p_out=0.0005, k=10 (+4 guard), tol 1e-6, float64, 1 thread"}
    for name, app in (("plain", lambda V: ref.lambda_bound * V - ref.L @ V),
                      ("sped_limit8", lambda V: opoly.apply_limit_product(ref.L, 8, V))):
        t0 = time.perf_counter()
        r = osol.subspace_iteration(ref.L, app, 10, V0, max_iters=5000, tol=1e-6, guard=4)
        c1[name] = {"seconds": round(time.perf_counter() - t0, 3), "iters": r.iters, "converged": r.converged,
                    "angle_vs_eigh": osol.max_principal_angle(U, r.Q)}
    out["sbm2000_solve"] = c1
    n0, src, dst = synth.chung_lu_device(4_000_000, 2.1, 16.0, 256, 0.95, seed=1)
    src_h, dst_h = src.cpu().numpy(), dst.cpu().numpy()
    L = sped.Laplacian(n0, src, dst, kind="sym", lcc=True, walk_records=False)
    del src, dst
    X = synth.gaussian_block_device(L.n, 64, seed=2, dtype=torch.bfloat16)
    Y = torch.empty_like(X)
    p = sped.transform("limit", 16)
    g = gpu_ms(lambda: sped.apply_poly(L, p, X, out=Y))
    Xh = X.float().cpu().numpy().astype(np.float64)
    n_lcc, nnz = L.n, L.nnz
    del L, X, Y
    torch.cuda.empty_cache()
    ref = olap.laplacian(n0, src_h, dst_h, kind=olap.SYM_NORMALIZED, lcc=True)
    print("[oracle] power-law Laplacian built", file=sys.stderr, flush=True)
    med, each, workers = _cpu_baseline_threaded(lambda V: opoly.apply_limit_product(ref.L, 16, V), Xh, runs)
    out["power_law_4m_limit16_k64"] = {"n_lcc": n_lcc, "nnz": nnz, "oracle_s_median": round(med, 3),
                                       "oracle_s_each": each, "oracle_cores": workers,
                                       "gpu_ms_bf16": round(g, 3), "gpu_over_oracle": round(med * 1e3 / g, 1)}
    del ref, Xh
    n, s, d, _ = synth.sbm_from_degrees(500_000, 50, 22.8, 1.2, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym", walk_records=False)
    gen = torch.Generator(device="cpu").manual_seed(5)
    theta = torch.randn(13, generator=gen, dtype=torch.float64) * 0.3
    X = synth.gaussian_block_device(L.n, 50, seed=6)
    g = gpu_ms(lambda: poly_apply(theta, X, L, 1.0, 1.0))
    Xh = X.cpu().numpy().astype(np.float64)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    pol = opoly.Poly(theta.numpy(), 1.0, 1.0)
    med, each, workers = _cpu_baseline_threaded(lambda V: opoly.apply_terms(ref.L, pol, V), Xh, runs)
    out["sbm500k_degree12_k50"] = {"n": L.n, "nnz": L.nnz, "oracle_s_median": round(med, 3), "oracle_s_each": each,
                                   "oracle_cores": workers, "gpu_ms_f32": round(g, 3),
                                   "gpu_over_oracle": round(med * 1e3 / g, 1)}
    del L, X
    torch.cuda.empty_cache()
    return out


def cpu_baseline_rmat_leg(sped, synth, torch, np, scale=22, runs=3):
    """cpu_baseline leg for the R-MAT workload: the oracle, unchanged, timed
    as a reported baseline.  Scale 26 does not fit the float64
    oracle, so its one sparse step L X (64 columns) is timed on the scale-22
    largest component (same generator and parameters), on the host's cores
    (column slices on threads, median of `runs`), beside the GPU's step on the
    same graph; the scale-26 figure is extrapolated by the ratio of stored
    entries (the step's work is proportional to nnz x k), with scale 26 built
    on the GPU in the same run to read its nnz and time its step."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    from oracle import laplacian as olap

    k = 64
    one = sped.monomial([0.0, 1.0])

    def gpu_step(L):
        X = synth.gaussian_block_device(L.n, k, seed=2, dtype=torch.float32)
        Y = torch.empty_like(X)
        sped.apply_poly(L, one, X, out=Y)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            sped.apply_poly(L, one, X, out=Y)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return X, float(np.median(ts))

    n, src, dst = synth.rmat_device(scale, 16, 0.57, 0.19, 0.19, seed=1)
    src_h, dst_h = src.cpu().numpy(), dst.cpu().numpy()
    L = sped.Laplacian(n, src, dst, kind="sym", lcc=True, walk_records=False)
    del src, dst
    X, g_ms = gpu_step(L)
    Xh = X.cpu().numpy().astype(np.float64)
    del X
    ref = olap.laplacian(n, src_h, dst_h, kind=olap.SYM_NORMALIZED, lcc=True)
    print(f"[rmat-oracle] scale {scale} built: oracle and GPU", file=sys.stderr, flush=True)
    workers = max(1, min(16, len(os.sched_getaffinity(0)), k))
    slices = [np.ascontiguousarray(Xh[:, c]) for c in np.array_split(np.arange(k), workers)]
    times = []
    with ThreadPoolExecutor(workers) as ex:
        for _ in range(runs):
            t0 = time.perf_counter()
            parts = list(ex.map(lambda V: ref.L @ V, slices))
            np.concatenate(parts, axis=1)
            times.append(time.perf_counter() - t0)
            print(f"[rmat-oracle] oracle step {len(times)}: {times[-1]:.3f} s", file=sys.stderr, flush=True)
    o_s = float(np.median(times))
    out = {"workload": f"R-MAT scale {scale} and 26, edge factor 16 (0.57, 0.19, 0.19), device draw; largest "
                       f"component; sym-normalised L; one sparse step L X, k={k}",
           f"scale{scale}": {"n_lcc": L.n, "nnz": L.nnz, "oracle_step_s_median": round(o_s, 3),
                             "oracle_step_s_each": [round(t, 3) for t in times], "oracle_cores": workers,
                             "gpu_step_ms_f32": round(g_ms, 3), "gpu_over_oracle": round(o_s * 1e3 / g_ms, 1)},
           "host": _host_info()}
    del L, ref, Xh, slices
    torch.cuda.empty_cache()
    n26, src, dst = synth.rmat_device(26, 16, 0.57, 0.19, 0.19, seed=1)
    L = sped.Laplacian(n26, src, dst, kind="sym", lcc=True, walk_records=False)
    del src, dst
    torch.cuda.empty_cache()
    X, g26 = gpu_step(L)
    ratio = L.nnz / out[f"scale{scale}"]["nnz"]
    out["scale26"] = {"n_lcc": L.n, "nnz": L.nnz, "gpu_step_ms_f32": round(g26, 3),
                      "oracle_step_s_extrapolated": round(o_s * ratio, 1), "nnz_ratio": round(ratio, 2),
                      "gpu_over_oracle_extrapolated": round(o_s * ratio * 1e3 / g26, 1),
                      "basis": f"scale-{scale} oracle median x stored-entry ratio (work ~ nnz x k)"}
    del X, L
    torch.cuda.empty_cache()
    return out


def reorder_leg(sped, synth, torch, np, graph="powerlaw4m", reps=10):
    """Node orders for gather locality (sped_laplacian_csr_ordered), timed
    apart from the solve: the build with each order against the plain build,
    the order alone on the built Laplacian, and one fused step L X per block
    width on each numbering.  powerlaw4m: the 4e6-node Chung-Lu workload
    (largest component); rmat26: R-MAT scale 26 (largest component)."""
    if graph == "rmat26":
        n0, src, dst = synth.rmat_device(26, 16, 0.57, 0.19, 0.19, seed=1)
        widths = ((64, torch.bfloat16, 1), (72, torch.bfloat16, 2), (72, torch.float32, 3))
        reps = 3
        desc = "R-MAT scale 26, edge factor 16 (0.57, 0.19, 0.19), device draw; largest component"
    else:
        n0, src, dst = synth.chung_lu_device(4_000_000, 2.1, 16.0, 256, 0.95, seed=1)
        widths = ((64, torch.bfloat16, 1), (64, torch.float32, 2))
        desc = ("Chung-Lu n=4e6 (device draw), exponent 2.1, mean degree 16, 256 communities; largest "
                "component")
    out = {"workload": desc + "; sym-normalised L; one fused step L X per width", "reps": reps}
    one = sped.monomial([0.0, 1.0])
    for order in (None, "degree", "cuthill_mckee", "label_propagation"):
        # built twice: the first build's time includes mapping fresh device
        # memory for its workspace, the second reuses the allocator's blocks
        rec = {}
        for key in ("build_first_s", "build_s"):
            L = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L = sped.Laplacian(n0, src, dst, kind="sym", lcc=True, walk_records=False, order=order)
            torch.cuda.synchronize()
            rec[key] = round(time.perf_counter() - t0, 3)
        if order is None:
            out["n_lcc"], out["nnz"] = L.n, L.nnz
            for method in ("degree", "cuthill_mckee", "label_propagation"):
                sped.locality_order(L, method)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sped.locality_order(L, method)
                torch.cuda.synchronize()
                rec[f"order_only_{method}_s"] = round(time.perf_counter() - t0, 3)
        for k, dt, lines in widths:
            X = synth.gaussian_block_device(L.n, k, seed=2, dtype=dt)
            Y = torch.empty_like(X)
            sped.apply_poly(L, one, X, out=Y)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                sped.apply_poly(L, one, X, out=Y)
                b.record()
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            ms = float(np.median(ts))
            alg = 8 * (L.n + 1) + L.nnz * 8 + 4 * L.n + L.n * k * 2 * X.element_size()
            rec[f"k{k}_{str(dt).split('.')[-1]}"] = {"step_ms": round(ms, 3), "alg_GBps": round(alg / ms / 1e6, 1)}
            del X, Y
        name = order or "given_ids"
        out[name] = rec
        print(json.dumps({"reorder": graph, "order": name, **rec}), flush=True)
        del L
    return out


def paper_experiments(sped, synth, torch, np):
    """Qualitative reproductions of the paper's own synthetic experiments on
    the GPU solvers (combinatorial Laplacian, as there).
    cliques: n nodes in c cliques joined by 0-25 random short-circuit edges per
      clique pair (Sec. 5, cliques); subspace iteration to 1e-6 (cap 200) with
      plain L reversed and the limit operator of degree 11/51/151/251 (App. A,
      series accuracy): success means the bottom-c subspace was reached.
    mdp_3room: the 3-room grid world, s = 2, h = 10 (Sec. 5, proto-value
      functions), bottom 3 (the room modes; +2 guard): the paper's subspace
      error 1 - ||U*^T Q||_F^2 / k against the dense eigenvectors after T
      iterations of subspace iteration, block Oja and mu-EigenGame (step
      0.5 / rho(M) for the last two), and the mu-EG eigenvector streak, for
      the identity and the degree-251 limit and Taylor forms of -e^{-L}.  The
      solver's own residual bound is not used here: at degree 251 float32
      rounding leaves high-frequency noise whose residual overstates the angle
      by about lambda_max / gap.
    link_prediction: 1000 nodes in 5 cliques with 20% of edges removed and
      completed by common-neighbour scores (Sec. 5, link prediction); plain vs
      degree-251 limit, iterations to 1e-6 and the k-means ARI against the
      cliques."""
    from paper_2207_14589_amd import metrics

    def solve(L, k, p, V0, U, guard, max_iters, tol=1e-6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            r = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=tol, max_iters=max_iters)
        except RuntimeError as e:
            return {"reached_bottom": False, "error": str(e).split(": ")[-1]}
        sec = time.perf_counter() - t0
        ang = _sin_angle(U, r.V.cpu().numpy(), np)
        return {"reached_bottom": bool(r.converged and ang < 10 * tol), "iters": r.stats["iters"],
                "seconds": round(sec, 4), "sin_angle_to_bottom": ang}

    out = {"cliques": []}
    for n, c in ((1000, 5), (2000, 5), (2000, 4)):
        N, s, d, _ = synth.cliques_short_circuit(n, c, seed=1)
        L = sped.Laplacian(N, s, d, kind="combinatorial")
        lam, U = _dense_lap(L, np)
        V0 = torch.from_numpy(synth.gaussian_block(N, c + 2, 2).astype(np.float32)).cuda()
        rec = {"n": N, "c": c, "lambda_max": float(lam[-1]), "plain": solve(L, c, None, V0, U[:, :c], 2, 200)}
        for ell in (11, 51, 151, 251):
            rec[f"limit{ell}"] = dict(solve(L, c, sped.transform("limit", ell), V0, U[:, :c], 2, 200),
                                      two_l_above_lambda_max=bool(2 * ell > lam[-1]))
        out["cliques"].append(rec)

    N, s, d = synth.three_room_grid(2, 10)
    L = sped.Laplacian(N, s, d, kind="combinatorial")
    lam, U = _dense_lap(L, np)
    k, guard = 3, 2
    V0 = torch.from_numpy(synth.gaussian_block(N, k + guard, 2).astype(np.float32)).cuda()
    Uk = U[:, :k]
    Uref = torch.from_numpy(Uk.astype(np.float32)).cuda()
    checkpoints = [10, 40, 160, 640, 2560, 10240]
    mdp = {"n": N, "k": k, "lambda_max": float(lam[-1]), "checkpoints": checkpoints,
           "target_subspace_error": 1e-8}

    def subspace_error(V):
        Q, _ = np.linalg.qr(V.astype(np.float64))
        return float(max(0.0, 1.0 - np.linalg.norm(Uk.T @ Q) ** 2 / k))

    for name, p, rho in (("identity", None, L.lambda_bound),
                         ("limit251", sped.transform("limit", 251), 1.0),
                         ("taylor_exp251", sped.transform("taylor_exp", 251), 1.0)):
        rec = {}
        for solver, eta in (("subspace", 1.0), ("oja", 0.5 / rho), ("mu_eg", 0.5 / rho)):
            errs, streaks = [], []
            done = False
            for T in checkpoints:  # later checkpoints are skipped once the target is met
                if done:
                    errs.append(None)
                    if solver == "mu_eg":
                        streaks.append(None)
                    continue
                r = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=0.0, max_iters=T, check_every=T, solver=solver,
                                 eta=eta)
                errs.append(subspace_error(r.V.cpu().numpy()))
                if solver == "mu_eg":
                    streaks.append(metrics.eigenvector_streak(Uref, r.V))
                done = errs[-1] < 1e-8 and (solver != "mu_eg" or streaks[-1] == k)
            hit = [T for T, e in zip(checkpoints, errs) if e is not None and e < 1e-8]
            rec[solver] = {"eta": eta if solver != "subspace" else None, "subspace_error": errs,
                           "first_checkpoint_below_target": hit[0] if hit else None}
            if solver == "mu_eg":
                rec[solver]["streak"] = streaks
        mdp[name] = rec
    out["mdp_3room"] = mdp

    # link prediction: 1000 nodes in 5 cliques, 20% of edges removed and filled
    # back with common-neighbour weights; SPED on the weighted graph
    from sklearn.metrics import adjusted_rand_score

    N, s, d, w, labels = synth.link_prediction_cliques(1000, 5, seed=1)
    L = sped.Laplacian(N, s, d, w, kind="combinatorial")
    lam, U = _dense_lap(L, np)
    c = 5
    V0 = torch.from_numpy(synth.gaussian_block(N, c + 2, 2).astype(np.float32)).cuda()
    lp = {"n": N, "c": c, "edges": int(s.shape[0]), "weighted_edges": int((w < 1).sum()),
          "lambda_max": float(lam[-1])}
    for name, p in (("plain", None), ("limit251", sped.transform("limit", 251))):
        rec = solve(L, c, p, V0, U[:, :c], 2, 2000)
        if "iters" in rec:
            r = sped.bottomk(L, c, p, V0=V0, guard=2, tol=1e-6, max_iters=2000)
            lab, _, _, _ = sped.cluster_embed(r.V, c, row_normalize=False, seed=1)
            rec["ari_vs_cliques"] = float(adjusted_rand_score(labels, lab.cpu().numpy()))
        lp[name] = rec
    out["link_prediction"] = lp
    return out


def estimator_comparison(sped, torch, L, p, coeffs, Q, X, ell, walks, stream):
    """The unbiased estimates of (I - L/l)^l V at the same walks per row: the
    importance edge-chain walk (Sec. 4.3), the lazy node walk (bounded
    weights, one row gather per walk) and the edge walk with its first m
    terms exact (m sparse steps, walks of length l - m), as relative
    Frobenius error against the exact product, on the solver's current
    iterate Q (near the bottom eigenvectors) and on the Gaussian block X; and
    their times."""
    out = {"walks_per_row": walks}
    for name, V in (("on_iterate", Q), ("on_gaussian", torch.from_numpy(X).cuda())):
        exact = sped.apply_poly(L, p, V)
        edge = sped.apply_poly_stochastic(L, coeffs, V, walks=walks, seed=7)
        lazy = sped.apply_limit_lazy(L, ell, V, walks, seed=7)
        nrm = float(exact.norm())
        out[name] = {"rel_err_edge_walk": float((edge - exact).norm()) / nrm,
                     "rel_err_lazy_walk": float((lazy - exact).norm()) / nrm}
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    Y = torch.empty_like(Q)
    for i, (a, b) in enumerate(evs):
        a.record(stream)
        sped.apply_limit_lazy(L, ell, Q, walks, seed=11, counter=i, out=Y)
        b.record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in evs)[len(evs) // 2]
    out["lazy_walk_ms"] = round(ms, 4)
    out["lazy_walks_per_s"] = round(L.n * walks / (ms * 1e-3), 1)
    # exact low-order terms, sampled tail: error and time against the number of exact terms
    hyb = {}
    G = torch.from_numpy(X).cuda()
    for m in (0, 1, 2, 3, 4):
        row = {}
        for name, V in (("on_iterate", Q), ("on_gaussian", G)):
            exact = sped.apply_poly(L, p, V)
            est = sped.apply_poly_hybrid(L, coeffs, V, m, walks=walks, seed=7)
            row["rel_err_" + name] = float((est - exact).norm()) / float(exact.norm())
        for i, (a, b) in enumerate(evs):
            a.record(stream)
            sped.apply_poly_hybrid(L, coeffs, Q, m, walks=walks, seed=11, counter=i, out=Y)
            b.record(stream)
        torch.cuda.synchronize()
        row["ms"] = round(sorted(a.elapsed_time(b) for a, b in evs)[len(evs) // 2], 4)
        hyb[f"exact_terms_{m}"] = row
    out["exact_low_sampled_tail"] = hyb
    # the solver driven by random estimates only: where each estimator's noise
    # leaves the iterate (bottom 28 + 4 guard, 30 iterations from one start)
    V0 = torch.from_numpy(X).cuda()
    floor = {}
    for name, kw in (("edge_walk", {"exact_terms": 0}), ("exact_terms_2", {"exact_terms": 2}),
                     ("lazy_walk", {"sampler": "lazy"})):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sped.bottomk(L, 28, p, V0=V0, guard=4, tol=0.0, max_iters=30, stochastic_iters=30, walks_per_row=walks,
                         **kw)
        floor[name] = {"max_residual": r.stats["max_residual"], "bound": r.stats["bound"],
                       "seconds": round(time.perf_counter() - t0, 4)}
    out["solver_noise_floor_30_random_iterations"] = floor
    return out


def stream_apply_leg(sped, torch, np, L, n, s, d, Q):
    """L Q from the bench graph's edge list held in pinned host memory and
    streamed in batches (the edge-minibatch path: the graph not resident),
    against the resident sparse step's L Q.  Host->device bytes are 8 per edge
    (two int32 endpoints, no weights), so the rate includes the PCIe copies."""
    sh = torch.from_numpy(np.ascontiguousarray(s)).to(torch.int32).pin_memory()
    dh = torch.from_numpy(np.ascontiguousarray(d)).to(torch.int32).pin_memory()
    m = sh.numel()
    batch = 1 << 22
    _, scale = sped.stream_node_scales(n, sh, dh, kind="sym", batch=batch)   # first call: one-time costs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        _, scale = sped.stream_node_scales(n, sh, dh, kind="sym", batch=batch)
    torch.cuda.synchronize()
    scales_ms = (time.perf_counter() - t0) * 1e3 / 3
    Y = torch.empty(n, Q.shape[1], dtype=torch.float32, device=Q.device)
    sped.stream_laplacian_apply(n, sh, dh, Q, scale=scale, out=Y, batch=batch)
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        sped.stream_laplacian_apply(n, sh, dh, Q, scale=scale, out=Y, batch=batch)
    ms = (time.perf_counter() - t0) * 1e3 / reps
    Yc = sped.apply_poly(L, sped.monomial([0.0, 1.0]), Q)
    torch.cuda.synchronize()
    rel = float((Y - Yc).abs().max() / Yc.abs().max())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sped.apply_poly(L, sped.monomial([0.0, 1.0]), Q, out=Yc)
    e1.record()
    torch.cuda.synchronize()
    resident_ms = e0.elapsed_time(e1) / reps
    # minibatch Oja steps with the degree-8 limit polynomial, one batch of 2^21
    # edges per factor (8 batches per step), on a copy of Q
    V = Q.clone()
    sped.minibatch_oja(n, sh, dh, V, scale=scale, degree=8, batch=1 << 21, eta=0.5, iters=1)
    torch.cuda.synchronize()
    steps = 3
    t0 = time.perf_counter()
    sped.minibatch_oja(n, sh, dh, V, scale=scale, degree=8, batch=1 << 21, eta=0.5, iters=steps)
    oja_ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"workload": "same SBM edge list (int32 pairs, pinned host memory), L Q with k=32, batches of 2^22 edges",
            "edges": m, "node_scales_ms": round(scales_ms, 3),
            "node_scales_host_to_device_GBps": round(8 * m / (scales_ms * 1e-3) / 1e9, 2), "apply_ms": round(ms, 3),
            "minibatch_oja_limit8_ms_per_step": round(oja_ms, 3),
            "minibatch_oja_edge_samples_per_s": round(8 * (1 << 21) / (oja_ms * 1e-3), 1),
            "edges_per_s": round(m / (ms * 1e-3), 1), "host_to_device_GBps": round(8 * m / (ms * 1e-3) / 1e9, 2),
            "resident_sparse_step_ms": round(resident_ms, 4), "max_rel_diff_vs_resident": rel}


def copy_rate_leg(sped, torch, np, reps=10):
    """The achievable HBM rate on this machine: the library's plain copy kernel
    over 512 MiB (read + write bytes / time, median of `reps` launches)."""
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    sped.stream_copy(a, b)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sped.stream_copy(a, b)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * COPY_BYTES / (float(np.median(ts)) * 1e-3) / 1e9


def ordered_chain_leg(sped, torch, np, n, s, d, Q, ell, per_launch, reps=10):
    """The headline's exact chain on the same SBM numbered by label
    propagation (the optional order, built and timed apart; `value` stays on
    the generator's ids).  The operator is the same with its rows permuted;
    the generator already numbers each block contiguously, so what changes is
    the order inside each found community (decreasing degree)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Lo = sped.Laplacian(n, s, d, kind="sym", walk_records=False, order="label_propagation")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    p = sped.transform("limit", ell)
    W2 = torch.empty_like(Q)
    sped.apply_poly(Lo, p, Q, out=W2)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sped.apply_poly(Lo, p, Q, out=W2)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    del Lo, W2
    return {"ordered_build_s": round(build_s, 3), "exact_pLV_ms_median": round(ms, 4),
            "pLV_GBps": round(ell * per_launch / (ms * 1e-3) / 1e9, 1),
            "avg_launch_us": round(ms * 1e3 / ell, 2)}


def power_law_bf16(sped, synth, torch, np):
    """The power-law workload at its full shape: a 4e6-node Chung-Lu graph
    (exponent 2.1, mean degree 16, 256 planted communities, 95% of draws
    inside the community), drawn on the device, largest component only, the
    symmetric normalised L; a 64-column bf16 block.  Times the degree-16
    limit application (bf16 in and out, float32 intermediates, as the
    solver's bf16 phase uses it) and one all-bf16 fused step, with the
    algorithmic bytes of each, on the generator's ids and again on the
    label-propagation numbering (the ordered build timed apart)."""
    n0, src, dst = synth.chung_lu_device(4_000_000, 2.1, 16.0, 256, 0.95, seed=1)
    L = sped.Laplacian(n0, src, dst, kind="sym", lcc=True, walk_records=False)
    k, ell = 64, 16
    X = synth.gaussian_block_device(L.n, k, seed=2, dtype=torch.bfloat16)
    Y = torch.empty_like(X)
    p = sped.transform("limit", ell)
    one = sped.monomial([0.0, 1.0])

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    chain_ms = timed(lambda: sped.apply_poly(L, p, X, out=Y), 5)
    step_ms = timed(lambda: sped.apply_poly(L, one, X, out=Y), 20)
    idx = 8 * (L.n + 1) + L.nnz * 8 + 4 * L.n
    step_bytes = idx + L.n * k * (2 + 2)                      # bf16 U in, bf16 O out
    chain_bytes = ell * idx + L.n * k * (2 + 4 + (ell - 2) * 8 + 4 + 2)  # bf16 X, f32 between, bf16 Y
    out = {"workload": "Chung-Lu n=4e6 (device draw), exponent 2.1, mean degree 16, 256 communities; "
                       "largest component; sym-normalised L; k=64 bf16",
           "n_lcc": L.n, "nnz": L.nnz, "max_degree": L.max_degree, "medium_rows": L.n_medium,
           "heavy_rows": L.n_heavy, "xcd_rows": L.xcd_rows,
           "chain_ms": round(chain_ms, 4), "chain_GBps": round(chain_bytes / (chain_ms * 1e-3) / 1e9, 1),
           "bf16_step_us": round(step_ms * 1e3, 2), "bf16_step_GBps": round(step_bytes / (step_ms * 1e-3) / 1e9, 1)}
    # the same graph numbered by label propagation (same operator, rows permuted)
    del L, X, Y
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = sped.Laplacian(n0, src, dst, kind="sym", lcc=True, walk_records=False, order="label_propagation")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    del src, dst
    X = synth.gaussian_block_device(L.n, k, seed=2, dtype=torch.bfloat16)
    Y = torch.empty_like(X)
    chain_ms = timed(lambda: sped.apply_poly(L, p, X, out=Y), 5)
    step_ms = timed(lambda: sped.apply_poly(L, one, X, out=Y), 20)
    out["label_propagation_ids"] = {
        "ordered_build_s": round(build_s, 3),
        "chain_ms": round(chain_ms, 4), "chain_GBps": round(chain_bytes / (chain_ms * 1e-3) / 1e9, 1),
        "bf16_step_us": round(step_ms * 1e3, 2), "bf16_step_GBps": round(step_bytes / (step_ms * 1e-3) / 1e9, 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--mfma-summary", metavar="PMC_DB",
                    help="print per-kernel MFMA use from a rocprofv3 --pmc database")
    ap.add_argument("--tolerance-only", action="store_true",
                    help="run only the time-to-tolerance comparisons (profiling the solver)")
    ap.add_argument("--chain-only", action="store_true", help="time only the exact p(L)V chain (profiling)")
    ap.add_argument("--power-law-only", action="store_true",
                    help="run only the power-law bf16 workload (profiling the SpMM bins)")
    ap.add_argument("--stream-only", action="store_true",
                    help="run only the streamed edge-batch L Q on the bench graph (profiling that path)")
    ap.add_argument("--gather-probe", action="store_true",
                    help="measure the chip's rate for the sparse step's row-load pattern")
    ap.add_argument("--rmat26", action="store_true",
                    help="run only the R-MAT scale-26 solver iterations (minutes; not part of the default run)")
    ap.add_argument("--power-law-solve", action="store_true",
                    help="solve the 4e6-node power-law workload to 1e-5, plain against SPED (minutes)")
    ap.add_argument("--rmat26-step", action="store_true",
                    help="time one fused step on the R-MAT scale-26 graph at 72/64 columns (profiling the bins)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run the copy-calibrated workload for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="summarise the two counter databases into the committed traffic file")
    ap.add_argument("--sstep-sweep", action="store_true",
                    help="time the chain as single steps and as two-step launches on LDS row blocks")
    ap.add_argument("--cpu-baseline-workloads", action="store_true",
                    help="cpu_baseline legs: time the oracle on the power-law and PolyApply workloads beside the GPU")
    ap.add_argument("--cpu-baseline-rmat", action="store_true",
                    help="cpu_baseline leg: time the oracle's sparse step on R-MAT scale 22, extrapolated to scale 26")
    ap.add_argument("--reorder", choices=["powerlaw4m", "rmat26"],
                    help="build with each node order and time one fused step per block width on each")
    ap.add_argument("--locality-sweep", action="store_true",
                    help="time the fused step against neighbourhood locality, and a plain copy")
    args = ap.parse_args()
    if args.locality_sweep:
        locality_sweep()
        return
    if args.sstep_sweep:
        print(json.dumps({"sstep_sweep": sstep_sweep()}), flush=True)
        return
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.mfma_summary:
        mfma_summary(args.mfma_summary)
        return
    if args.traffic_probe:
        traffic_probe(args)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(collectives and sharding are out of scope); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2207_14589_amd import sped, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.tolerance_only:
        out = {"time_to_tolerance": time_to_tolerance(sped, synth, torch, np),
               "time_to_tolerance_sbm500k": time_to_tolerance_sbm500k(sped, synth, torch, np),
               "time_to_tolerance_combinatorial": time_to_tolerance_combinatorial(sped, synth, torch, np),
               "mu_eg_streak": mu_eg_streak_sbm2000(sped, synth, torch, np),
               "paper_experiments": paper_experiments(sped, synth, torch, np)}
        print(json.dumps(out), flush=True)
        return
    if args.gather_probe:
        print(json.dumps({"gather_probe": gather_probe(sped, torch)}), flush=True)
        return
    if args.rmat26:
        print(json.dumps({"rmat26_solver": rmat26_solver(sped, synth, torch, np)}), flush=True)
        return
    if args.power_law_solve:
        print(json.dumps({"power_law_4m_solve": power_law_4m_solve(sped, synth, torch, np)}), flush=True)
        return
    if args.rmat26_step:
        print(json.dumps({"rmat26_step": rmat26_step(sped, synth, torch, np)}), flush=True)
        return
    if args.cpu_baseline_workloads:
        print(json.dumps({"cpu_baseline_workloads": cpu_baseline_workloads_leg(sped, synth, torch, np)}), flush=True)
        return
    if args.cpu_baseline_rmat:
        print(json.dumps({"cpu_baseline_rmat": cpu_baseline_rmat_leg(sped, synth, torch, np)}), flush=True)
        return
    if args.reorder:
        print(json.dumps({"reorder": reorder_leg(sped, synth, torch, np, args.reorder)}), flush=True)
        return
    if args.power_law_only:
        print(json.dumps({"power_law_bf16_k64": power_law_bf16(sped, synth, torch, np)}), flush=True)
        return
    if args.stream_only:
        n, s, d, _ = synth.sbm_from_degrees(1_000_000, 100, 19.0, 1.0, seed=1)
        L = sped.Laplacian(n, s, d, kind="sym", walk_records=False)
        Q = torch.from_numpy(synth.gaussian_block(n, 32, 2).astype(np.float32)).cuda()
        print(json.dumps({"stream_apply": stream_apply_leg(sped, torch, np, L, n, s, d, Q)}), flush=True)
        return
    k, ell, walks = 32, 16, 8
    t0 = time.perf_counter()
    n, s, d, _ = synth.sbm_from_degrees(1_000_000, 100, 19.0, 1.0, seed=1)
    gen_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = sped.Laplacian(n, s, d, kind="sym")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    X = synth.gaussian_block(n, k, 2).astype(np.float32)
    Q = torch.from_numpy(X).cuda()
    sped.orthonormalize(Q, passes=2)
    W = torch.empty_like(Q)
    S = torch.empty_like(Q)
    p = sped.transform("limit", ell)
    coeffs = p.monomial()
    stream = torch.cuda.current_stream()

    def step(i, ev):
        nonlocal Q, W
        ev[0].record(stream)
        sped.apply_poly(L, p, Q, out=W)
        ev[1].record(stream)
        if args.chain_only:
            return
        sped.apply_poly_stochastic(L, coeffs, Q, walks=walks, seed=3, counter=i, out=S)
        ev[2].record(stream)
        sped.orthonormalize(W, passes=2)
        ev[3].record(stream)
        sped.rayleigh_ritz(L, W)
        ev[4].record(stream)
        Q, W = W, Q

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    for i in range(args.warmup):
        step(i, mk())
    torch.cuda.synchronize()
    evs = [mk() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    chain_all = [e[0].elapsed_time(e[1]) for e in evs]
    chain_ms = np.mean(chain_all)
    parts = {"exact_pLV_ms": round(float(chain_ms), 4),
             "exact_pLV_ms_median": round(float(np.median(chain_all)), 4),
             "exact_pLV_ms_min": round(float(np.min(chain_all)), 4)}
    if not args.chain_only:
        parts["walk_estimate_ms"] = round(float(np.mean([e[1].elapsed_time(e[2]) for e in evs])), 4)
        parts["cholqr2_ms"] = round(float(np.mean([e[2].elapsed_time(e[3]) for e in evs])), 4)
        parts["rayleigh_ritz_ms"] = round(float(np.mean([e[3].elapsed_time(e[4]) for e in evs])), 4)
    per_launch = spmm_step_bytes(L.n, L.nnz, k)
    copy_GBps = copy_rate_leg(sped, torch, np)
    app_bytes = ell * per_launch
    value = app_bytes / (chain_ms * 1e-3) / 1e9
    launch_s = chain_ms * 1e-3 / ell
    achieved = per_launch / launch_s / 1e9
    traffic = measured_traffic(per_launch)
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "SBM n=1e6, 100 blocks, mean degree 20, 5% cross edges; sym-normalised L; "
                               f"k={k} float32 block; limit polynomial degree {ell}; {walks} walks/row",
                   "n": L.n, "nnz": L.nnz, "k": k, "degree": ell, "walks_per_row": walks,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "spmm_light (fused sparse step)",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "alg_bytes_per_launch": per_launch, "avg_launch_us": round(launch_s * 1e6, 3),
                     # the rate a plain 512 MiB copy reaches on this machine, beside the spec peak
                     "copy_GBps": round(copy_GBps, 1), "frac_of_copy": round(achieved / copy_GBps, 4)},
        "step_breakdown": parts,
        "pLV_per_s": round(1e3 / chain_ms, 2),
        # one timed step is one solver iteration (exact product, walk estimate,
        # CholQR2, Rayleigh-Ritz)
        "solver_iters_per_s": None if args.chain_only else round(1e3 / ms_per_step, 2),
        "walk_steps_per_s": (round(L.n * walks * ell / (parts["walk_estimate_ms"] * 1e-3), 1)
                             if "walk_estimate_ms" in parts else None),
        # bytes a walk-step touches: one 32-byte entry record and one X row
        # (each node's row is gathered once, when the walk leaves it)
        "walk_touched_GBps": (round(L.n * walks * ell * (32 + 4 * k) / (parts["walk_estimate_ms"] * 1e-3) / 1e9, 1)
                              if "walk_estimate_ms" in parts else None),
        "setup": {"graph_gen_s": round(gen_s, 3), "laplacian_build_s": round(build_s, 3)},
    }
    if not args.chain_only:
        line["estimators"] = estimator_comparison(sped, torch, L, p, coeffs, Q, X, ell, walks, stream)
        line["stream_apply"] = stream_apply_leg(sped, torch, np, L, n, s, d, Q)
        line["label_propagation_ids"] = ordered_chain_leg(sped, torch, np, n, s, d, Q, ell, per_launch)
    if not args.chain_only and not args.no_solve:
        del L, Q, W, S
        torch.cuda.empty_cache()
        line["power_law_bf16_k64"] = power_law_bf16(sped, synth, torch, np)
    if not args.no_solve and not args.chain_only:
        line["time_to_tolerance"] = time_to_tolerance(sped, synth, torch, np)
        line["time_to_tolerance_sbm500k"] = time_to_tolerance_sbm500k(sped, synth, torch, np)
        line["time_to_tolerance_combinatorial"] = time_to_tolerance_combinatorial(sped, synth, torch, np)
        line["polyapply_sbm500k"] = polyapply_sbm500k(sped, synth, torch, np)
        line["time_to_tolerance_powerlaw200k"] = time_to_tolerance_powerlaw200k(sped, synth, torch, np)
        line["mu_eg_streak"] = mu_eg_streak_sbm2000(sped, synth, torch, np)
        line["paper_experiments"] = paper_experiments(sped, synth, torch, np)
    if not args.no_cpu_baseline and not args.chain_only:
        line["cpu_baseline"] = cpu_baseline_leg(n, s, d, X, ell, per_launch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
