"""Synthetic analogues of the paper's accuracy/time experiments, on one GPU.

    python -m paper_2210_05105_amd.figures --fig 2  [--workload zipf3]
    python -m paper_2210_05105_amd.figures --fig 12 [--workload zipf3]
    python -m paper_2210_05105_amd.figures --fig 13 [--workload zipf3]

Each prints one JSON object per measured point (and a summary line):

- fig 2: running maximum of the fit against elapsed sweep time for STS-CP,
  CP-ARLS-LEV and exact (non-randomized) ALS, same tensor and
  initialisation (the paper's Fig. 2 compares its randomized algorithms
  with exact ALS the same way, on a tensor it does not ship);
- fig 12: per-phase time of a sweep and the fit reached, for J from 32,768
  to 196,608 draws (its Fig. 12 runtime breakdown against J);
- fig 13: fit and time of CP-ARLS-LEV against STS-CP for R in
  {25, 50, 75, 100} (its Fig. 13 sampler comparison across ranks).

Only the library's public API is used (the path under test); the tensors
are the synthetic power-law workloads of `tensorgen`, not the paper's
datasets, so the numbers are analogues, not reproductions.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _tensor(name, dev):
    import torch
    import tensorgen as tg
    if name in ("zipf4", "zipf3xl", "batch3"):
        dims, idx, val = tg.make_tensor_device(name, dev)
        return dims, idx, val.to(torch.float32)
    T = tg.make_tensor(name)
    return (T.dims, torch.from_numpy(T.idx).to(dev),
            torch.from_numpy(T.val.astype(np.float32)).to(dev))


def _init(ctx, dims, R, seed, dev):
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    for k, d in enumerate(dims):
        ctx.set_factor(k, torch.randn((d, R), dtype=torch.float32,
                                      device=dev, generator=g).double())


def _run(dims, idx, val, R, sampler, precision, J, sweeps, seed, dev,
         leaf=0, profile=False):
    """Sweeps one at a time; returns per-sweep (elapsed s, fit), phases."""
    import torch
    from . import Context
    ctx = Context(idx, val, dims, R, sampler, precision,
                  max_J=max(J, 1), sts_leaf=leaf)
    _init(ctx, dims, R, seed, dev)
    N = len(dims)
    g = torch.Generator(device=dev)
    g.manual_seed(seed + 1)
    uni = None
    if sampler != "exact":
        uni = torch.rand((sweeps, N, J, N - 1), dtype=torch.float64,
                         device=dev, generator=g)
    if profile:
        ctx.profile(True)
    out, t_acc = [], 0.0
    for t in range(sweeps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if sampler == "exact":
            ctx.sweep(1)
        else:
            ctx.sweep(1, J, uni[t:t + 1])
        torch.cuda.synchronize()
        t_acc += time.perf_counter() - t0
        out.append((t_acc, ctx.fit()))   # the fit is off the clock
    phases = ctx.profile_read() if profile else None
    ctx.close()
    torch.cuda.empty_cache()
    return out, phases


def fig2(dims, idx, val, R, J, sweeps, dev, emit):
    for sampler in ("sts", "arls", "exact"):
        pts, _ = _run(dims, idx, val, R, sampler, "fp32", J, sweeps, 5, dev)
        best = -1e9
        for t, (el, f) in enumerate(pts):
            best = max(best, f)
            emit(dict(fig=2, sampler=sampler, sweep=t + 1, seconds=el,
                      fit=f, running_max_fit=best))


def fig12(dims, idx, val, R, sweeps, dev, emit):
    for J in (32768, 65536, 98304, 131072, 196608):
        pts, ph = _run(dims, idx, val, R, "sts", "fp32", J, sweeps, 5, dev,
                       profile=True)
        emit(dict(fig=12, J=J, seconds_per_sweep=pts[-1][0] / sweeps,
                  fit=pts[-1][1],
                  phase_ms_per_sweep={k: v[0] / sweeps for k, v in ph.items()}))


def fig13(dims, idx, val, J, sweeps, dev, emit):
    for R in (25, 50, 75, 100):
        for sampler in ("arls", "sts"):
            pts, _ = _run(dims, idx, val, R, sampler, "fp32", J, sweeps, 5,
                          dev)
            emit(dict(fig=13, R=R, sampler=sampler,
                      seconds_per_sweep=pts[-1][0] / sweeps,
                      fit=pts[-1][1]))


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--fig", type=int, required=True, choices=[2, 12, 13])
    p.add_argument("--workload", default="zipf3")
    p.add_argument("--R", type=int, default=32)
    p.add_argument("--J", type=int, default=65536)
    p.add_argument("--sweeps", type=int, default=10)
    a = p.parse_args(argv)
    import torch
    from . import load_library
    load_library()
    dev = torch.device("cuda:0")
    dims, idx, val = _tensor(a.workload, dev)

    def emit(d):
        d["workload"] = a.workload
        print(json.dumps(d), flush=True)

    if a.fig == 2:
        fig2(dims, idx, val, a.R, a.J, a.sweeps, dev, emit)
    elif a.fig == 12:
        fig12(dims, idx, val, a.R, a.sweeps, dev, emit)
    else:
        fig13(dims, idx, val, a.J, a.sweeps, dev, emit)


if __name__ == "__main__":
    main()
