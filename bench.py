"""Benchmark: randomized CP-ALS sweeps/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload zipf3xl]

A step is one ALS sweep (every mode solved once: pseudo-inverse, draws,
merge, sampled MTTKRP, solve, renormalisation, Gram, sampler rebuild) over
the resident synthetic tensor.  The default workload is the largest
single-GPU configuration: the 3-way power-law tensor 8,000,000 x 8,000,000 x
200,000 with 1.5 billion nonzeros (Zipf(1.05) indices, lognormal FP32
values), R = 100, J = 262,144 draws per mode solve, STS-CP, mixed precision
(FP32 MTTKRP, split-BF16 MFMA factor Grams, FP64 sampler and row solve),
generated on the GPU.  Other workloads: zipf3 (100,000 x 80,000 x
60,000, 50M nonzeros, R = 32), zipf4 (4-way, 200M nonzeros, R = 64,
CP-ARLS-LEV), planted (200 x 150 x 100, R = 8).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import tensorgen as tg  # noqa: E402

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
FP64_PEAK_TFS = 78.6      # MI355X FP64 vector / matrix
N_SIMD = 256 * 4          # MI355X: 256 compute units of 4 SIMDs
N_XCD = 8                 # accelerator dies (each counts GRBM_GUI_ACTIVE)

# per workload: precision and STS leaf size when not given (0: the library
# chooses it per tree factor)
DEFAULTS = {"planted": ("fp64", 0), "zipf3": ("fp32", 0),
            "zipf4": ("mixed", 0), "zipf3xl": ("mixed", 0),
            "batch3": ("mixed", 16)}
DEVICE_GENERATED = ("zipf4", "zipf3xl", "batch3")
BATCH_RANKS = (8, 16, 32, 64, 128)   # batched restarts: ranks drawn from
BATCH_B = 64                         # these, for 64 restarts


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="zipf3xl",
                   choices=["zipf3xl", "zipf4", "zipf3", "planted",
                            "batch3"])
    p.add_argument("--autotune", action="store_true",
                   help="choose the leaf size / bucket rows (or streams) "
                        "by timing candidates first (cached)")
    p.add_argument("--nstreams", type=int, default=0,
                   help="batch3: concurrent streams (0: 4)")
    p.add_argument("--precision", default=None)
    p.add_argument("--leaf", type=int, default=0)
    p.add_argument("--compare", default=None, metavar="PRECISION",
                   help="also run the same sweeps in this precision form "
                        "(identical inputs and uniforms); report its rate "
                        "and fit (default: fp64 for the billion-nonzero "
                        "workload, none elsewhere; 'none' turns it off)"),
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-profile", action="store_true")
    p.add_argument("--reduce-counters", nargs=3,
                   metavar=("FETCH_DB", "WRITE_DB", "SOLVES"),
                   help="reduce two rocprofv3 --pmc databases to HBM bytes "
                        "per mode solve and exit")
    p.add_argument("--kernel-stats", metavar="DB",
                   help="print per-kernel totals of a rocprofv3 "
                        "--kernel-trace database as a markdown table and exit")
    p.add_argument("--counter-table", metavar="DB",
                   help="print per-dispatch averages of every counter of a "
                        "rocprofv3 --pmc database per kernel (with the "
                        "matrix-core busy fraction when SQ_VALU_MFMA_BUSY_"
                        "CYCLES and GRBM_GUI_ACTIVE are among them) and exit")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="also copy MIB MiB device to device (a plain copy "
                        "kernel of known size, to scale HBM counters)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sts_flops_per_solve(dims, j, R, J, F):
    """Algorithmic FP64 FLOPs of the STS-CP draws of one mode-j solve.

    First factor (h = 1): row masses U[i] G_{>k} U[i]^T, 2R^2 + 2R per row.
    Each later factor k, per draw: the root and one left-child mass per
    level, <(h h^T) (*) G_{>k}, G^node> at 3 FLOPs per packed entry
    (P = R(R+1)/2), then F[k] leaf rows at R + 2R^2 each.  Per draw:
    h^T G^+ h, 2R^2 + R.
    """
    P = R * (R + 1) // 2
    modes = [k for k in range(len(dims)) if k != j]
    fl = dims[modes[0]] * (2 * R * R + 2 * R)
    for k in modes[1:]:
        depth = math.ceil(math.log2(max(1, -(-dims[k] // F[k]))))
        fl += J * ((depth + 1) * 3 * P + F[k] * (2 * R * R + R))
    return fl + J * (2 * R * R + R)


def host_info():
    """Cores this process may use, CPU model, RAM and BLAS threads."""
    cores = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return cores, model, ram


def cpu_baseline(ctx, dims, nnz, idx_s, val_s, J, N, R, sampler, uni_j):
    """Time the FP64 oracle on a bounded sample of one mode-0 solve.

    Every piece runs on a sample and is scaled to the full solve: the
    sampler structures on a prefix of each factor's rows (cost linear in
    rows), a subset of the draws (each draw's cost does not depend on J),
    the scan-filter extraction and the sampled MTTKRP on a uniform subset
    of the nonzeros (idx_s, val_s), the solve and Gram at full size.
    """
    import oracle as O
    import torch
    from threadpoolctl import threadpool_info, threadpool_limits
    cores, model, ram = host_info()
    j = 0
    modes = [k for k in range(N) if k != j]
    U = [ctx.get_factor(k).cpu().numpy() for k in range(N)]
    G = [ctx.get_gram(k).cpu().numpy() for k in range(N)]
    with threadpool_limits(limits=cores):
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        ROWS = 100_000
        blk = 64  # oracle prefix-Gram block (ROWS R^2 long doubles at most)
        t_pre = 0.0
        sub = {}
        for k in modes:
            rows = min(dims[k], ROWS)
            t0 = time.perf_counter()
            if sampler == "sts":
                sub[k] = O.sts_prefix_grams(U[k][:rows], blk)
            else:
                sub[k] = O.arls_build(U[k][:rows], G[k])
            t_pre += (time.perf_counter() - t0) * dims[k] / rows
        # draws on the sampled factors: cost per draw, scaled to J
        Us = [U[k][:min(dims[k], ROWS)] if k != j else U[k] for k in range(N)]
        Js = min(J, 256 if sampler == "sts" else 8192)
        u = uni_j[:Js]
        t0 = time.perf_counter()
        if sampler == "sts":
            O.sts_sample(Us, G, j, u, block=blk,
                         prefix={k: sub[k] for k in modes})
        else:
            O.arls_sample(Us, sub, j, u)
        t_draw = (time.perf_counter() - t0) * (J / Js)
        # merge, extraction and MTTKRP for the GPU's full draw set of mode 0,
        # extraction scanning the sampled nonzeros
        gidx, gprob = ctx.sample(j, torch.from_numpy(uni_j))
        sidx = gidx.cpu().numpy().astype(np.int64)
        prob = gprob.cpu().numpy()
        t0 = time.perf_counter()
        h = np.ones((J, R))
        for q, k in enumerate(modes):
            h = h * U[k][sidx[:, q]]
        keys, rep, cnt, wts = O.dedup(sidx, prob, dims, j, J)
        t_merge = time.perf_counter() - t0
        t0 = time.perf_counter()
        ck, rows, vals, slot = O.extract(idx_s, val_s, dims, j, keys)
        M = O.sampled_mttkrp(dims[j], rows, vals, slot, wts, h[rep])
        t_ext = (time.perf_counter() - t0) * nnz / idx_s.shape[0]
        t0 = time.perf_counter()
        Uj, sig = O.solve(M, O.pinv_psd(O.gram_hadamard(G, j)))
        O.gram(Uj)
        t_solve = time.perf_counter() - t0
        rows_b = min(dims[j], ROWS)
        t0 = time.perf_counter()
        if sampler == "sts":
            O.sts_prefix_grams(Uj[:rows_b], blk)
        else:
            O.arls_build(Uj[:rows_b], O.gram(Uj))
        t_build = (time.perf_counter() - t0) * dims[j] / rows_b
    per_solve = t_pre / (N - 1) + t_draw + t_merge + t_ext + t_solve + t_build
    per_sweep = N * per_solve
    sample = (f"one mode-0 solve, extrapolated to a sweep (x{N}): sampler "
              f"structures on the first {ROWS} rows of each factor "
              f"({t_pre:.1f} s scaled by rows, counted once per solve), "
              f"{Js} of {J} draws ({t_draw * Js / J:.1f} s, scaled "
              f"x{J / Js:.0f}), merge of the GPU's {J} draws "
              f"({t_merge:.1f} s), scan-filter extraction + sampled MTTKRP "
              f"over {idx_s.shape[0]} of {nnz} nonzeros ({t_ext * idx_s.shape[0] / nnz:.1f} s, "
              f"scaled x{nnz / idx_s.shape[0]:.0f}), solve + Gram at full "
              f"size ({t_solve:.1f} s), sampler rebuild ({t_build:.1f} s "
              f"scaled); NumPy outside BLAS runs on one thread")
    return dict(value=1.0 / per_sweep, unit="sweeps/s", cores=blas,
                kind="oracle", sample=sample, host_cores=cores,
                blas_threads=blas, cpu_model=model, host_ram_gib=ram,
                seconds_per_sweep_extrapolated=per_sweep)


# kernel sets whose HBM traffic is reported, and the sources they come from
KERNEL_SETS = {"sts_draw": ("k_sts_", ["k_sts.hip"]),
               "sampled_mttkrp": ("k_bk_", ["k_mttkrp.hip"])}


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2210_05105_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_kernel_name(n):
    import re
    n = re.sub(r"^void ", "", n)
    n = re.sub(r"cpr::\(anonymous namespace\)::", "", n)
    return re.sub(r"\(.*$", "", n)


def kernel_stats(db, top=60):
    """Markdown table of per-kernel time from a rocprofv3 database."""
    import sqlite3
    from collections import defaultdict
    cur = sqlite3.connect(db).cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    name = "kernel_name" if "kernel_name" in cols else "name"
    tot, cnt = defaultdict(float), defaultdict(int)
    for n, b, e in cur.execute(f"select {name}, start, end from kernels"):
        k = short_kernel_name(n)
        tot[k] += e - b
        cnt[k] += 1
    allt = sum(tot.values())
    out = ["| kernel | calls | total ms | avg us | % |",
           "|---|---:|---:|---:|---:|"]
    for k in sorted(tot, key=lambda k: -tot[k])[:top]:
        out.append(f"| {k} | {cnt[k]} | {tot[k] / 1e6:.2f} | "
                   f"{tot[k] / cnt[k] / 1e3:.1f} | {100 * tot[k] / allt:.1f} |")
    out.append(f"\ntotal kernel time {allt / 1e6:.1f} ms over "
               f"{sum(cnt.values())} dispatches")
    return "\n".join(out)


def counter_table(db):
    """Markdown table: per kernel, the dispatch count, the average duration
    and the per-dispatch average of every counter in a rocprofv3 --pmc
    database.  With SQ_VALU_MFMA_BUSY_CYCLES (summed over the SIMDs) and
    GRBM_GUI_ACTIVE (summed over the dies) it adds the matrix cores' busy
    fraction: busy cycles / (SIMDs x active cycles of one die)."""
    import sqlite3
    from collections import defaultdict
    cur = sqlite3.connect(db).cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(counters_collection)")]
    cn = "counter_name" if "counter_name" in cols else "name"
    kn = "kernel_name" if "kernel_name" in cols else "name"
    tot = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for k, c, v, d in cur.execute(
            f"select {kn}, {cn}, value, dispatch_id from counters_collection"):
        k = short_kernel_name(k)
        tot[k][c] += v
        disp[k].add(d)
    dur = defaultdict(list)
    kc = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    if kc:
        kk = "kernel_name" if "kernel_name" in kc else "name"
        for k, b, e in cur.execute(f"select {kk}, start, end from kernels"):
            dur[short_kernel_name(k)].append((e - b) / 1e3)
    names = sorted({c for k in tot for c in tot[k]})
    mf = "SQ_VALU_MFMA_BUSY_CYCLES" in names and "GRBM_GUI_ACTIVE" in names
    head = ["kernel", "n", "avg us"] + names + (["MFMA busy"] if mf else [])
    out = ["| " + " | ".join(head) + " |",
           "|---|" + "---:|" * (len(head) - 1)]
    for k in sorted(tot, key=lambda k: -sum(dur.get(k, [0]))):
        n = len(disp[k])
        avg = {c: tot[k][c] / n for c in names}
        row = [k, str(n), f"{sum(dur[k]) / len(dur[k]):.1f}" if dur.get(k)
               else "-"] + [f"{avg[c]:.4g}" for c in names]
        if mf:
            act = avg["GRBM_GUI_ACTIVE"] / N_XCD
            row.append(f"{avg['SQ_VALU_MFMA_BUSY_CYCLES'] / (N_SIMD * act):.1%}"
                       if act > 0 else "-")
        out.append("| " + " | ".join(row) + " |")
    return "\n".join(out)


def reduce_counters(fetch_db, write_db, solves, calib_mib):
    """HBM bytes per mode solve of each kernel set, from two rocprofv3 --pmc
    databases (FETCH_SIZE, WRITE_SIZE; KiB per dispatch).  Each counter is
    scaled by the ratio of the known size of the first device-to-device
    copies of the process (--copy-calibration) to what the counter reads for
    them."""
    import sqlite3
    out = {}
    for name, db in (("fetch", fetch_db), ("write", write_db)):
        cur = sqlite3.connect(db).cursor()
        rows = list(cur.execute(
            "select kernel_name, value from counters_collection "
            "order by dispatch_id"))
        copies = [v for k, v in rows if "copyBuffer" in k][:3]
        factor = calib_mib * 1024.0 / (sum(copies) / len(copies))
        log(f"{name}: the calibration copies read {copies} KiB: "
            f"factor {factor:.4f}")
        per = {}
        for k, v in rows:
            if "copyBuffer" not in k:
                per[short_kernel_name(k)] = per.get(short_kernel_name(k), 0) + v
        for k, v in per.items():
            out.setdefault("per_kernel", {}).setdefault(k, {})[
                name + "_MiB_per_solve"] = v * factor / 1024.0 / solves
        for ks, (prefix, _) in KERNEL_SETS.items():
            kib = sum(v for k, v in rows if prefix in k)
            d = out.setdefault(ks, {})
            d[name + "_bytes_per_solve"] = kib * 1024.0 * factor / solves
            d[name + "_factor"] = factor
    for ks, (_, files) in KERNEL_SETS.items():
        out[ks]["source_digest"] = source_digest(files)
    per = out.pop("per_kernel", {})
    log("| kernel | fetch MiB/solve | write MiB/solve |")
    log("|---|---:|---:|")
    for k in sorted(per, key=lambda k: -sum(per[k].values())):
        log(f"| {k} | {per[k].get('fetch_MiB_per_solve', 0):.1f} | "
            f"{per[k].get('write_MiB_per_solve', 0):.1f} |")
    return out


def measured_traffic(workload, kernel):
    """HBM bytes per launch of a kernel set from the committed counter
    summary, or None if absent or taken on other sources."""
    try:
        with open(traffic_file(workload)) as fh:
            t = json.load(fh)[kernel]
    except (OSError, KeyError, ValueError):
        return None
    if t.get("source_digest") != source_digest(KERNEL_SETS[kernel][1]):
        return None
    return t["fetch_bytes_per_solve"] + t["write_bytes_per_solve"]


def build_inputs(a, w, dev):
    """Tensor (device COO), initial factors and uniforms of the workload."""
    import torch
    N = len(w["dims"])
    t0 = time.time()
    if a.workload in DEVICE_GENERATED:
        dims, idx_d, val_d = tg.make_tensor_device(a.workload, dev, log=log)
        base = 2210_5105 * 16 + int(w["tag"])
        if "R" not in w:
            U0 = None
        elif w.get("init") == "slice_scaled":
            U0 = tg.init_factors_slice_scaled_device(base + 11, dims, w["R"],
                                                     idx_d)
        else:
            U0 = tg.init_factors_device(base + 11, dims, w["R"], dev)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    else:
        T = tg.make_tensor(a.workload)
        dims = T.dims
        idx_d = torch.from_numpy(T.idx).to(dev)
        val_d = torch.from_numpy(T.val).to(dev)
        _, _, rinit, _ = tg.streams(w["tag"])
        U0 = [torch.from_numpy(u).to(dev) for u in
              tg.init_factors(rinit, dims, w["R"], dtype=np.float32)]
    log(f"generated {a.workload}: dims {dims} nnz {idx_d.shape[0]} in "
        f"{time.time() - t0:.1f}s")
    return dims, N, idx_d, val_d, U0


def dev_of(t):
    return t.device


def run_form(a, w, dims, N, idx_d, val_d, U0, uni, precision, leaf, timed,
             bucket_rows=0):
    """Build a context in one precision form and run warmup + timed sweeps.
    Returns (ctx, seconds of the timed sweeps, init seconds, fit, counters,
    per-phase times of the timed sweeps)."""
    import torch
    from paper_2210_05105_amd import Context
    R, J, sampler = w["R"], w["J"], w["sampler"]
    vdt = torch.float64 if precision == "fp64" else torch.float32
    torch.cuda.synchronize()
    t0 = time.time()
    ctx = Context(idx_d, val_d.to(vdt), dims, R, sampler, precision, max_J=J,
                  sts_leaf=leaf, bucket_rows=bucket_rows)
    torch.cuda.synchronize()
    t_init = time.time() - t0
    torch.cuda.empty_cache()
    free_b, total_b = torch.cuda.mem_get_info(dev_of(idx_d))
    log(f"[{precision}] cp_init (per-mode index build) {t_init:.2f}s; device "
        f"memory free {free_b / 2**30:.1f} of {total_b / 2**30:.1f} GiB")
    for k in range(N):
        ctx.set_factor(k, U0[k])
    if a.warmup:
        ctx.sweep(a.warmup, J, uni[:a.warmup])
    ctx.sync()
    ctx.counters(reset=True)
    if timed and not a.no_profile:
        ctx.profile(True, phases=["sample", "mttkrp"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sweep(a.steps, J, uni[a.warmup:a.warmup + a.steps])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.sync()
    ph_timed = ctx.profile_read() if timed and not a.no_profile else {}
    ctx.profile(False)
    cnt = ctx.counters()
    fit = ctx.fit()
    log(f"[{precision}] timed {a.steps} sweeps in {dt:.4f}s; fit {fit:.6f}; "
        f"counters {cnt}")
    return ctx, dt, t_init, fit, cnt, ph_timed


def bench_batch(a, w, dev, precision, leaf):
    """Batched restarts: 64 decompositions of one tensor with ranks drawn
    uniformly from {8, 16, 32, 64, 128}, every sweep one replay of a
    captured HIP graph.  value = restart-sweeps per second.  The plain FP64
    one-instance form is timed per rank class (one restart each, its own
    context) and summed over the 64 restarts by class counts."""
    import torch
    from paper_2210_05105_amd import Batch, Context
    J, sampler = w["J"], w["sampler"]
    rng = np.random.default_rng(2210_5105 + 5)
    ranks = [int(r) for r in rng.choice(BATCH_RANKS, size=BATCH_B)]
    w = dict(w, R=max(ranks))
    dims, N, idx_d, val_d, _ = build_inputs(a, w, dev)
    nnz = int(idx_d.shape[0])
    vdt = torch.float64 if precision == "fp64" else torch.float32
    base = 2210_5105 * 16 + int(w["tag"])
    nstreams = a.nstreams
    tuned = None
    if a.autotune:
        from paper_2210_05105_amd.autotune import tune_batch
        tuned = tune_batch(idx_d, val_d.to(vdt), dims, ranks, sampler,
                           precision, J, log=log)
        nstreams = tuned["nstreams"]
        log(f"autotune: {tuned}")
    t0 = time.time()
    bt = Batch(idx_d, val_d.to(vdt), dims, ranks, sampler, precision, J=J,
               sts_leaf=leaf, nstreams=nstreams)
    torch.cuda.synchronize()
    t_init = time.time() - t0
    log(f"batch init (shared index, {BATCH_B} restarts) {t_init:.2f}s")
    U0 = [tg.init_factors_device(base + 100 + b, dims, R, dev)
          for b, R in enumerate(ranks)]
    for b in range(BATCH_B):
        for k in range(N):
            bt.set_factor(b, k, U0[b][k])
    nsw = a.warmup + a.steps
    uni_all = tg.uniforms_device(base + 13, (nsw, BATCH_B, N, J, N - 1), dev)
    ubuf = torch.empty_like(uni_all[0])
    for t in range(a.warmup):
        ubuf.copy_(uni_all[t])
        bt.sweep(ubuf)
    bt.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(a.warmup, nsw):
        ubuf.copy_(uni_all[t])   # refill the captured buffer (a device copy)
        bt.sweep(ubuf)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bt.sync()
    fits = bt.fit()
    bt.close()
    torch.cuda.empty_cache()
    rate = BATCH_B * a.steps / dt
    log(f"batch: {a.steps} sweeps of {BATCH_B} restarts in {dt:.3f}s "
        f"({rate:.1f} restart-sweeps/s); mean fit {np.mean(fits):.5f}")
    # plain FP64 one-instance reference: one restart per rank class
    ref = {}
    if a.compare:
        vref = val_d.to(torch.float64 if a.compare == "fp64" else
                        torch.float32)
        for R in sorted(set(ranks)):
            b = ranks.index(R)
            c = Context(idx_d, vref, dims, R, sampler, a.compare, max_J=J,
                        sts_leaf=leaf)
            for k in range(N):
                c.set_factor(k, U0[b][k])
            c.sweep(a.warmup, J, uni_all[:a.warmup, b])
            c.sync()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            c.sweep(a.steps, J, uni_all[a.warmup:, b])
            torch.cuda.synchronize()
            tr = (time.perf_counter() - t1) / a.steps
            ref[R] = dict(count=ranks.count(R), s_per_sweep=tr, fit=c.fit(),
                          batch_fit=fits[b])
            c.close()
            torch.cuda.empty_cache()
            log(f"[{a.compare}] one instance R={R}: {tr * 1e3:.2f} ms/sweep, "
                f"fit {ref[R]['fit']:.5f} (batch restart {fits[b]:.5f})")
    compare = None
    if ref:
        tot = sum(v["count"] * v["s_per_sweep"] for v in ref.values())
        compare = dict(precision=a.compare, form="one instance per restart",
                       value=BATCH_B / tot,
                       per_rank={str(k): v for k, v in ref.items()},
                       max_abs_fit_difference=max(
                           abs(v["fit"] - v["batch_fit"]) for v in ref.values()))
    out = {
        "metric": "ALS sweeps/sec and sampled-MTTKRP HBM GB/s (% of peak) at fixed fit",
        "value": rate, "unit": "restart-sweeps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if precision != "fp64" else "f64", "data": "synthetic",
        "config": {"workload": "batch3", "dims": list(dims), "nnz": nnz,
                   "restarts": BATCH_B, "ranks": ranks, "J": J,
                   "sampler": sampler, "precision": precision,
                   "nstreams": nstreams or 4, "sts_leaf": leaf,
                   "parallelism": "single-gpu", "autotuned": tuned},
        "fits": fits, "init_s": t_init, "compare": compare,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.kernel_stats:
        print(kernel_stats(a.kernel_stats))
        return
    if a.counter_table:
        print(counter_table(a.counter_table))
        return
    if a.reduce_counters:
        fdb, wdb, solves = a.reduce_counters
        print(json.dumps(reduce_counters(fdb, wdb, float(solves),
                                         a.copy_calibration or 256), indent=1))
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); this "
              f"library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2210_05105_amd import load_library
    load_library()
    dev = torch.device("cuda:0")
    if a.copy_calibration:  # first copies of the process: known size
        n = a.copy_calibration * (1 << 20) // 4
        src_t = torch.ones(n, dtype=torch.float32, device=dev)
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {a.copy_calibration} MiB")
        del src_t, dst_t
    w = dict(tg.WORKLOADS[a.workload])
    prec0, leaf0 = DEFAULTS[a.workload]
    # the headline rate is quoted at fixed fit: by default the plain FP64
    # form runs the same sweeps first and its rate and fit are reported
    if a.compare is None and a.workload == "zipf3xl":
        a.compare = "fp64"
    if a.compare == "none":
        a.compare = None
    precision = a.precision or prec0
    leaf = a.leaf or leaf0
    if a.workload == "batch3":
        return bench_batch(a, w, dev, precision, leaf)
    R, J, sampler = w["R"], w["J"], w["sampler"]
    dims, N, idx_d, val_d, U0 = build_inputs(a, w, dev)
    nnz = int(idx_d.shape[0])
    tuned = None
    if a.autotune:
        from paper_2210_05105_amd.autotune import tune_context
        tuned = tune_context(idx_d, val_d.to(torch.float64 if precision ==
                                             "fp64" else torch.float32),
                             dims, R, sampler, precision, J, log=log)
        leaf = tuned["sts_leaf"] or leaf
        log(f"autotune: {tuned}")
    # a uniform sample of the nonzeros for the oracle's bounded extraction,
    # kept on the host
    S = min(nnz, 8_000_000)
    gs = torch.Generator(device=dev)
    gs.manual_seed(17)
    pick = torch.randint(nnz, (S,), device=dev, generator=gs) \
        if S < nnz else torch.arange(nnz, device=dev)
    idx_s = idx_d[pick].cpu().numpy()
    val_s = val_d[pick].double().cpu().numpy()
    del pick
    # after the timed sweeps, a short pass with events on every phase gives
    # the breakdown (events cost the stream a few microseconds each, so the
    # timed sweeps record them only around the two phases the line reports)
    extra = 0 if a.no_profile else min(a.steps, 3)
    nsw = a.warmup + a.steps + extra
    uni = tg.uniforms_device(2210_5105 * 16 + int(w["tag"]) + 13,
                             (nsw, N, J, N - 1), dev)
    compare = None
    if a.compare:
        cctx, cdt, cinit, cfit, _, _ = run_form(
            a, w, dims, N, idx_d, val_d, U0, uni, a.compare, leaf, False)
        cctx.close()
        torch.cuda.empty_cache()
        compare = dict(precision=a.compare, value=a.steps / cdt,
                       ms_per_step=cdt / a.steps * 1e3, fit=cfit)
    ctx, dt, t_init, fit, cnt, ph_timed = run_form(
        a, w, dims, N, idx_d, val_d, U0, uni, precision, leaf, True,
        tuned["bucket_rows"] if tuned else 0)
    del idx_d, val_d
    torch.cuda.empty_cache()
    ph = {}
    if extra:
        ctx.profile(True)
        ctx.sweep(extra, J, uni[a.warmup + a.steps:])
        ctx.sync()
        ph = ctx.profile_read()
        ctx.profile(False)
    sweeps_per_s = a.steps / dt
    # rows per leaf of each factor's tree (0: no tree)
    leaves = [ctx.sts_leaf(k)[0] if sampler == "sts" else 0 for k in range(N)]

    # ---- roofline of the dominant kernel and the sampled MTTKRP
    solves = max(cnt["solves"], 1)
    tb = 4 if precision != "fp64" else 8
    mtt_bytes = (16 * cnt["unique"] + cnt["nnz"] * (4 + tb) +
                 cnt["unique"] * R * tb + cnt["rows"] * R * tb) / solves
    phases = {k: dict(ms_total=v[0], launches=v[1]) for k, v in ph.items()}
    roof = None
    mttkrp = None
    sts_draw = None

    def per_launch(k):  # from the timed sweeps when they timed phase k
        src = ph_timed if ph_timed.get(k, (0, 0))[1] else ph
        return src[k][0] / max(src[k][1], 1)

    if ph:
        ms_mtt = per_launch("mttkrp")
        mtt_gbs = mtt_bytes / (ms_mtt * 1e-3) / 1e9
        mttkrp = dict(algorithmic_bytes_per_launch=mtt_bytes,
                      ms_per_launch=ms_mtt, achieved_GBs=mtt_gbs,
                      frac_of_peak=mtt_gbs / HBM_PEAK_GBS,
                      nnz_extracted_per_solve=cnt["nnz"] / solves,
                      distinct_columns_per_solve=cnt["unique"] / solves,
                      rows_out_per_solve=cnt["rows"] / solves)
        if sampler == "sts" and ph.get("sample", (0, 0))[1]:
            fl = np.mean([sts_flops_per_solve(dims, j, R, J, leaves)
                          for j in range(N)])
            ms_s = per_launch("sample")
            ach = fl / (ms_s * 1e-3) / 1e12
            sts_draw = dict(flops_per_launch=fl, ms_per_launch=ms_s,
                            achieved_TFs=ach, frac_of_fp64_peak=ach /
                            FP64_PEAK_TFS)
        dom = max(ph, key=lambda k: ph[k][0])
        ms_dom = per_launch(dom)
        if dom == "sample" and sampler == "sts":
            fl = np.mean([sts_flops_per_solve(dims, j, R, J, leaves)
                          for j in range(N)])
            ach = fl / (ms_dom * 1e-3) / 1e12
            roof = dict(kernel="sts_draw", bound="mfma", achieved=ach,
                        peak=FP64_PEAK_TFS, unit="TFLOP/s",
                        frac=ach / FP64_PEAK_TFS,
                        traffic=measured_traffic(a.workload, "sts_draw"),
                        flops_per_launch=fl, ms_per_launch=ms_dom)
        elif dom == "mttkrp":
            roof = dict(kernel="sampled_mttkrp", bound="hbm",
                        achieved=mttkrp["achieved_GBs"], peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=mttkrp["frac_of_peak"],
                        traffic=measured_traffic(a.workload,
                                                 "sampled_mttkrp"),
                        bytes_per_launch=mtt_bytes, ms_per_launch=ms_mtt)
        else:
            roof = dict(kernel=dom, bound="latency", achieved=None,
                        peak=None, unit=None, frac=None, traffic=None,
                        ms_per_launch=ms_dom)
    cpu = None
    if not a.no_cpu_baseline:
        log("timing the oracle on the host ...")
        cpu = cpu_baseline(ctx, dims, nnz, idx_s, val_s, J, N, R, sampler,
                           uni[0, 0].cpu().numpy())
        log(f"oracle: {cpu['seconds_per_sweep_extrapolated']:.1f} s/sweep")
    out = {
        "metric": "ALS sweeps/sec and sampled-MTTKRP HBM GB/s (% of peak) at fixed fit",
        "value": sweeps_per_s, "unit": "sweeps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "dims": list(dims), "nnz": nnz,
                   "R": R, "J": J, "sampler": sampler,
                   "precision": precision, "sweeps_timed": a.steps,
                   "sts_leaf": leaves, "parallelism": "single-gpu",
                   "autotuned": tuned},
        "fit": fit, "init_s": t_init,
        "compare": compare,
        "sampled_mttkrp": mttkrp, "sts_draw": sts_draw, "phases": phases,
        "phases_sweeps": extra,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
