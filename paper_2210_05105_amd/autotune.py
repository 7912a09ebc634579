"""Autotuner for the layout and launch parameters of the hot path.

Parameters are chosen by timing whole ALS sweeps on the caller's own tensor
(random N(0,1) factors, seeded uniforms), one candidate at a time:

- ``sts_leaf``: rows per STS-CP tree leaf, the library's per-factor choice
  (0) or one F in {16, 32, 64} for every tree (tree depth and tree bytes
  against the rows each draw scans in its leaf);
- ``bucket_rows``: output rows per bucket of the sampled MTTKRP's
  row-ordered placement, B in {64, 128, 256} (placement atomics against
  split buckets to combine);
- ``nstreams``: for batched restarts, concurrent streams in {1, 2, 4, 8}.

The search is coordinate-wise (F first with the default B, then B with the
best F; streams last for batches).  A candidate the library refuses for
lack of device memory (CP_ENOMEM) is skipped.  Results are cached in a JSON file
(``CPR_TUNE_CACHE`` or ``~/.cache/cpr_autotune.json``) keyed by the device
name, tensor dimensions and nonzero count, rank(s), sampler, precision and
J.  Only the public API of the library is used; nothing here computes any
part of the method.
"""
from __future__ import annotations

import json
import os
import time

LEAVES = (0, 16, 32, 64)
BUCKETS = (64, 128, 256)
STREAMS = (1, 2, 4, 8)


def cache_path():
    return os.environ.get("CPR_TUNE_CACHE",
                          os.path.expanduser("~/.cache/cpr_autotune.json"))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def problem_key(device, dims, nnz, ranks, sampler, precision, J):
    import torch
    name = torch.cuda.get_device_name(device)
    rk = "-".join(str(r) for r in ranks)
    return (f"{name}|dims={'x'.join(str(d) for d in dims)}|nnz={nnz}|"
            f"R={rk}|{sampler}|{precision}|J={J}")


def _time_sweeps(run, sweeps):
    import torch
    run(1)  # warm up (first launches, LDS attributes)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    run(sweeps)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / sweeps


def _time_context(idx, val, dims, R, sampler, precision, J, leaf, buckets,
                  sweeps, seed):
    import torch
    from .binding import Context
    dev = idx.device
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    ctx = Context(idx, val, dims, R, sampler, precision, max_J=J,
                  sts_leaf=leaf, bucket_rows=buckets)
    try:
        for k, d in enumerate(dims):
            ctx.set_factor(k, torch.randn((d, R), dtype=torch.float64,
                                          device=dev, generator=g))
        N = len(dims)
        uni = torch.rand((sweeps + 1, N, J, N - 1), dtype=torch.float64,
                         device=dev, generator=g)
        state = {"t": 0}

        def run(n):
            t = state["t"]
            ctx.sweep(n, J, uni[t:t + n])
            state["t"] = t + n if t + n < uni.shape[0] else 0

        return _time_sweeps(run, sweeps)
    finally:
        ctx.close()
        torch.cuda.empty_cache()


def _try(fn, log):
    """A candidate's time, or None if the library refuses it for lack of
    device memory (CP_ENOMEM: every context keeps a reserve free)."""
    from .binding import CprError
    try:
        return fn()
    except CprError as e:
        if e.name != "CP_ENOMEM":
            raise
        if log:
            log(f"autotune: candidate skipped ({e})")
        return None


def tune_context(idx, val, dims, R, sampler, precision, J, sweeps=2,
                 seed=7, use_cache=True, log=None):
    """Best (sts_leaf, bucket_rows) for one decomposition of this tensor.

    idx, val: the device COO (as for Context).  Returns a dict with the
    chosen parameters, the measured ms per sweep of every candidate tried
    and whether it came from the cache.
    """
    path = cache_path()
    key = problem_key(idx.device, dims, int(val.shape[0]), [R], sampler,
                      precision, J)
    data = _load(path) if use_cache else {}
    if key in data:
        return dict(data[key], cached=True)
    tried = {}
    leaves = LEAVES if sampler == "sts" else (0,)
    best_leaf, best = None, None
    for F in leaves:
        ms = _try(lambda: _time_context(idx, val, dims, R, sampler, precision,
                                        J, F, 0, sweeps, seed), log)
        tried[f"leaf={F},buckets=auto"] = ms
        if ms is None:
            continue
        if log:
            log(f"autotune: leaf {F} -> {ms:.3f} ms/sweep")
        if best is None or ms < best:
            best_leaf, best = F, ms
    best_b = 0
    if best is None:
        raise RuntimeError("autotune: no candidate fits this device")
    for B in BUCKETS:
        ms = _try(lambda: _time_context(idx, val, dims, R, sampler, precision,
                                        J, best_leaf, B, sweeps, seed), log)
        tried[f"leaf={best_leaf},buckets={B}"] = ms
        if ms is None:
            continue
        if log:
            log(f"autotune: buckets {B} -> {ms:.3f} ms/sweep")
        if ms < best:
            best_b, best = B, ms
    res = dict(sts_leaf=best_leaf, bucket_rows=best_b, ms_per_sweep=best,
               tried=tried, at=time.strftime("%Y-%m-%d %H:%M:%S"))
    if use_cache:
        data = _load(path)
        data[key] = res
        _store(path, data)
    return dict(res, cached=False)


def tune_batch(idx, val, dims, ranks, sampler, precision, J, sweeps=2,
               seed=7, use_cache=True, log=None):
    """Best stream count (and leaf size for STS-CP) for a batch of restarts
    of these ranks on this tensor."""
    import torch
    from .binding import Batch
    path = cache_path()
    key = problem_key(idx.device, dims, int(val.shape[0]), ranks, sampler,
                      precision, J) + "|batch"
    data = _load(path) if use_cache else {}
    if key in data:
        return dict(data[key], cached=True)
    dev = idx.device
    N = len(dims)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    uni = torch.rand((len(ranks), N, J, N - 1), dtype=torch.float64,
                     device=dev, generator=g)
    tried, best, choice = {}, None, None
    leaves = LEAVES if sampler == "sts" else (0,)
    for F in leaves:
        for ns in STREAMS:
            if ns > len(ranks):
                continue
            def one():
                bt = Batch(idx, val, dims, ranks, sampler, precision, J=J,
                           sts_leaf=F, nstreams=ns)
                try:
                    for b, R in enumerate(ranks):
                        for k, d in enumerate(dims):
                            bt.set_factor(b, k, torch.randn(
                                (d, R), dtype=torch.float64, device=dev,
                                generator=g))
                    return _time_sweeps(
                        lambda n: [bt.sweep(uni) for _ in range(n)], sweeps)
                finally:
                    bt.close()
                    torch.cuda.empty_cache()
            ms = _try(one, log)
            tried[f"leaf={F},streams={ns}"] = ms
            if ms is None:
                continue
            if log:
                log(f"autotune: batch leaf {F} streams {ns} -> {ms:.3f} ms")
            if best is None or ms < best:
                best, choice = ms, (F, ns)
    if choice is None:
        raise RuntimeError("autotune: no candidate fits this device")
    res = dict(sts_leaf=choice[0], nstreams=choice[1], ms_per_sweep=best,
               tried=tried, at=time.strftime("%Y-%m-%d %H:%M:%S"))
    if use_cache:
        data = _load(path)
        data[key] = res
        _store(path, data)
    return dict(res, cached=False)
