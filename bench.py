"""Benchmark: randomized CP-ALS sweeps/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload zipf3]

A step is one ALS sweep (every mode solved once: pseudo-inverse, draws,
merge, sampled MTTKRP, solve, renormalisation, Gram, sampler rebuild) over
the resident synthetic tensor.  The default workload is the 3-way power-law
tensor 100,000 x 80,000 x 60,000 with 50M nonzeros (Zipf(1.1) indices,
lognormal FP32 values), R = 32, J = 65,536 draws per mode solve, STS-CP,
FP32 MTTKRP with FP64 Grams / sampler / solve.  Prints one JSON line.
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


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="zipf3",
                   choices=["zipf3", "planted"])
    p.add_argument("--precision", default=None)
    p.add_argument("--leaf", type=int, default=0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-profile", action="store_true")
    p.add_argument("--reduce-counters", nargs=3,
                   metavar=("FETCH_DB", "WRITE_DB", "SOLVES"),
                   help="reduce two rocprofv3 --pmc databases to HBM bytes "
                        "per mode solve and exit")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="also copy MIB MiB device to device (a plain copy "
                        "kernel of known size, to scale HBM counters)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sts_flops_per_solve(dims, j, R, J, F):
    """Algorithmic FP64 FLOPs of the STS-CP draws of one mode-j solve.

    First factor (h = 1): row masses U[i] G_{>k} U[i]^T, 2R^2 + 2R per row.
    Each later factor, per draw: the root and one left-child mass per level,
    <(h h^T) (*) G_{>k}, G^node> at 3 FLOPs per packed entry (P = R(R+1)/2),
    then F leaf rows at R + 2R^2 each.  Per draw: h^T G^+ h, 2R^2 + R.
    """
    P = R * (R + 1) // 2
    modes = [k for k in range(len(dims)) if k != j]
    fl = dims[modes[0]] * (2 * R * R + 2 * R)
    for k in modes[1:]:
        depth = math.ceil(math.log2(max(1, -(-dims[k] // F))))
        fl += J * ((depth + 1) * 3 * P + F * (2 * R * R + R))
    return fl + J * (2 * R * R + R)


def cpu_baseline(T, w, ctx, J, N, R, sampler):
    """Time the FP64 oracle on a bounded sample of one mode solve."""
    import oracle as O
    import torch
    j = 0
    U = [ctx.get_factor(k).cpu().numpy() for k in range(N)]
    G = [ctx.get_gram(k).cpu().numpy() for k in range(N)]
    rng = np.random.default_rng(123)
    Js = 512 if sampler == "sts" else J
    u = rng.random((J, N - 1))
    t0 = time.perf_counter()
    if sampler == "sts":
        pre = {k: O.sts_prefix_grams(U[k], 64) for k in range(N) if k != j}
        t_pre = time.perf_counter() - t0
        t1 = time.perf_counter()
        O.sts_sample(U, G, j, u[:Js], 64, prefix=pre)
        t_draw = (time.perf_counter() - t1) * (J / Js)
    else:
        st = {k: O.arls_build(U[k], G[k]) for k in range(N) if k != j}
        t_pre = time.perf_counter() - t0
        t1 = time.perf_counter()
        O.arls_sample(U, st, j, u)
        t_draw = time.perf_counter() - t1
    # merge, extraction (scan over all nonzeros), MTTKRP and solve for the
    # GPU's full draw set of this mode
    gidx, gprob = ctx.sample(j, torch.from_numpy(u))
    sidx, prob = gidx.cpu().numpy().astype(np.int64), gprob.cpu().numpy()
    t2 = time.perf_counter()
    h = np.ones((J, R))
    for q, k in enumerate([k for k in range(N) if k != j]):
        h = h * U[k][sidx[:, q]]
    keys, rep, cnt, wts = O.dedup(sidx, prob, T.dims, j, J)
    ck, rows, vals, slot = O.extract(T.idx, T.val, T.dims, j, keys)
    M = O.sampled_mttkrp(T.dims[j], rows, vals, slot, wts, h[rep])
    Uj, sig = O.solve(M, O.pinv_psd(O.gram_hadamard(G, j)))
    Gj = O.gram(Uj)
    t_rest = time.perf_counter() - t2
    t3 = time.perf_counter()
    if sampler == "sts":
        O.sts_prefix_grams(Uj, 64)
    else:
        O.arls_build(Uj, Gj)
    t_build = time.perf_counter() - t3
    per_solve = t_pre / (N - 1) + t_draw + t_rest + t_build
    per_sweep = N * per_solve
    sample = (f"one mode solve of mode 0 at full size: sampler structures for "
              f"the {N - 1} drawn factors ({t_pre:.1f} s, counted once per "
              f"solve), {Js} of {J} draws ({t_draw * Js / J:.1f} s, scaled "
              f"x{J // Js}), merge + scan-filter extraction over all "
              f"{T.nnz} nonzeros + sampled MTTKRP + solve ({t_rest:.1f} s), "
              f"sampler rebuild ({t_build:.1f} s); sweep = {N} x mode solve")
    return dict(value=1.0 / per_sweep, unit="sweeps/s", cores=1,
                kind="oracle", sample=sample,
                seconds_per_sweep_extrapolated=per_sweep)


# kernel sets whose HBM traffic is reported, and the sources they come from
KERNEL_SETS = {"sts_draw": ("k_sts_", ["k_sts.hip"]),
               "sampled_mttkrp": ("k_bk_", ["k_mttkrp.hip"])}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_zipf3_sts_fp32.json")


def source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2210_05105_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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
        for ks, (prefix, _) in KERNEL_SETS.items():
            kib = sum(v for k, v in rows if prefix in k)
            d = out.setdefault(ks, {})
            d[name + "_bytes_per_solve"] = kib * 1024.0 * factor / solves
            d[name + "_factor"] = factor
    for ks, (_, files) in KERNEL_SETS.items():
        out[ks]["source_digest"] = source_digest(files)
    return out


def measured_traffic(kernel):
    """HBM bytes per launch of a kernel set from the committed counter
    summary, or None if absent or taken on other sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)[kernel]
    except (OSError, KeyError, ValueError):
        return None
    if t.get("source_digest") != source_digest(KERNEL_SETS[kernel][1]):
        return None
    return t["fetch_bytes_per_solve"] + t["write_bytes_per_solve"]


def main():
    a = parse()
    if a.reduce_counters:
        fdb, wdb, solves = a.reduce_counters
        print(json.dumps(reduce_counters(fdb, wdb, float(solves),
                                         a.copy_calibration or 256), indent=1))
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the "
              f"multi-GPU layout is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2210_05105_amd import Context, load_library
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
    if a.workload == "zipf3":
        R, J, sampler = w["R"], w["J"], w["sampler"]
        precision = a.precision or "fp32"
    else:
        R, J, sampler = w["R"], w["J"], w["sampler"]
        precision = a.precision or "fp64"
    t0 = time.time()
    T = tg.make_tensor(a.workload)
    log(f"generated {a.workload}: dims {T.dims} nnz {T.nnz} in "
        f"{time.time() - t0:.1f}s")
    N = T.N
    vdt = torch.float64 if precision == "fp64" else torch.float32
    idx_d = torch.from_numpy(T.idx).to(dev)
    val_d = torch.from_numpy(T.val).to(dev, vdt)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx = Context(idx_d, val_d, T.dims, R, sampler, precision, max_J=J,
                  sts_leaf=a.leaf)
    torch.cuda.synchronize()
    t_init = time.time() - t0
    del idx_d, val_d
    log(f"cp_init (per-mode index build) {t_init:.2f}s")
    _, _, rinit, runi = tg.streams(w["tag"])
    U0 = tg.init_factors(rinit, T.dims, R,
                         dtype=np.float64 if precision == "fp64" else np.float32)
    for k in range(N):
        ctx.set_factor(k, torch.from_numpy(U0[k]))
    # after the timed sweeps, a short pass with events on every phase gives
    # the breakdown (events cost the stream a few microseconds each, so the
    # timed sweeps record them only around the two phases the line reports)
    extra = 0 if a.no_profile else min(a.steps, 5)
    uni = torch.from_numpy(
        tg.uniform_blocks(runi, a.warmup + a.steps + extra, J, N)).to(dev)
    torch.cuda.synchronize()
    per = J * N * (N - 1)
    if a.warmup:
        ctx.sweep(a.warmup, J, uni[:a.warmup])
    ctx.sync()
    ctx.counters(reset=True)
    if not a.no_profile:
        ctx.profile(True, phases=["sample", "mttkrp"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sweep(a.steps, J, uni[a.warmup:a.warmup + a.steps])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.sync()
    ph_timed = ctx.profile_read() if not a.no_profile else {}
    ctx.profile(False)
    cnt = ctx.counters()
    fit = ctx.fit()
    ph = {}
    if extra:
        ctx.profile(True)
        ctx.sweep(extra, J, uni[a.warmup + a.steps:])
        ctx.sync()
        ph = ctx.profile_read()
        ctx.profile(False)
    log(f"timed {a.steps} sweeps in {dt:.4f}s; fit {fit:.6f}; counters {cnt}")
    sweeps_per_s = a.steps / dt

    # ---- roofline of the dominant kernel and the sampled MTTKRP
    solves = max(cnt["solves"], 1)
    tb = 4 if precision != "fp64" else 8
    mtt_bytes = (16 * cnt["unique"] + cnt["nnz"] * (4 + tb) +
                 cnt["unique"] * R * tb + cnt["rows"] * R * tb) / solves
    phases = {k: dict(ms_total=v[0], launches=v[1]) for k, v in ph.items()}
    roof = None
    mttkrp = None

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
        dom = max(ph, key=lambda k: ph[k][0])
        ms_dom = per_launch(dom)
        if dom == "sample" and sampler == "sts":
            F = a.leaf or 16
            fl = np.mean([sts_flops_per_solve(T.dims, j, R, J, F)
                          for j in range(N)])
            ach = fl / (ms_dom * 1e-3) / 1e12
            roof = dict(kernel="sts_draw", bound="mfma", achieved=ach,
                        peak=FP64_PEAK_TFS, unit="TFLOP/s",
                        frac=ach / FP64_PEAK_TFS,
                        traffic=measured_traffic("sts_draw"),
                        flops_per_launch=fl, ms_per_launch=ms_dom)
        elif dom == "mttkrp":
            roof = dict(kernel="sampled_mttkrp", bound="hbm",
                        achieved=mttkrp["achieved_GBs"], peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=mttkrp["frac_of_peak"],
                        traffic=measured_traffic("sampled_mttkrp"),
                        bytes_per_launch=mtt_bytes, ms_per_launch=ms_mtt)
        else:
            roof = dict(kernel=dom, bound="latency", achieved=None,
                        peak=None, unit=None, frac=None, traffic=None,
                        ms_per_launch=ms_dom)
    cpu = None
    if not a.no_cpu_baseline:
        log("timing the oracle on the host ...")
        cpu = cpu_baseline(T, w, ctx, J, N, R, sampler)
        log(f"oracle: {cpu['seconds_per_sweep_extrapolated']:.1f} s/sweep")
    out = {
        "metric": "ALS sweeps/sec and sampled-MTTKRP HBM GB/s (% of peak) at fixed fit",
        "value": sweeps_per_s, "unit": "sweeps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "dims": list(T.dims),
                   "nnz": T.nnz, "R": R, "J": J, "sampler": sampler,
                   "precision": precision, "sweeps_timed": a.steps,
                   "sts_leaf": a.leaf or 16, "parallelism": "single-gpu"},
        "fit": fit, "init_s": t_init,
        "sampled_mttkrp": mttkrp, "phases": phases,
        "phases_sweeps": extra,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
