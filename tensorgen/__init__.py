"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module generates sparse tensors, initial factors and uniform streams.
It contains none of the decomposition's arithmetic (no Gram, leverage,
sampling, MTTKRP or solve); both the oracle and the GPU harness read the
same arrays from it, so identical seeds give identical inputs on both sides.

Workloads (sizes follow the five configurations the project benchmarks):

  tiny     : uniform-random distinct coordinates, planted rank-R CP values
  planted  : 200x150x100, 20k nnz, planted rank-8 model + N(0, 0.01) noise
  zipf3    : 100000x80000x60000, 50M nnz, Zipf(1.1) indices, lognormal values
  zipf4    : 1000000x500000x200000x1000, 200M nnz, Zipf(1.2), Poisson(3)+1
  zipf3xl  : 8000000x8000000x200000, 1.5B nnz, Zipf(1.05), lognormal
  batch3   : 500000x300000x100000, 100M nnz, Zipf(1.1), lognormal

The large ones are generated on the GPU (make_tensor_device, torch's
generator); the NumPy path serves the sizes the oracle can take whole.

Zipf(s) on a finite support r = 1..I draws r with probability proportional
to r^-s; labels are then relabelled by a seeded per-mode permutation so that
heavy indices are scattered (the paper permutes indices per mode for load
balance, Section 4.4).  Coordinates are deduplicated and topped up until the
nonzero count is exact.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "SparseTensor", "streams", "zipf_coords", "uniform_coords",
    "planted_values", "lognormal_values", "poisson_values", "init_factors",
    "uniform_block", "uniform_blocks", "make_tensor", "WORKLOADS",
    "zipf_coords_device", "values_device", "init_factors_device",
    "uniforms_device", "make_tensor_device",
]


@dataclasses.dataclass
class SparseTensor:
    dims: tuple            # (I_1, ..., I_N)
    idx: np.ndarray        # int32 [nnz, N], 0-based, distinct tuples
    val: np.ndarray        # float32 or float64 [nnz]

    @property
    def N(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.idx.shape[0])


def streams(tag, n: int = 4):
    """Independent PCG64 generators: coords, values, init, uniforms."""
    ss = np.random.SeedSequence([2210, 5105] + list(np.atleast_1d(tag)))
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def _draw_zipf_mode(rng, n, pmf, perm):
    """n i.i.d. Zipf draws: multinomial bucket counts, then a random order."""
    counts = rng.multinomial(n, pmf)
    r = np.repeat(perm, counts)
    rng.shuffle(r)
    return r


def _bits(d):
    return max(1, int(np.ceil(np.log2(max(d, 2)))))


def _pack(cols, dims):
    """Pack coordinates into one uint64 key (bit fields, mode 1 lowest)."""
    key = np.zeros(cols[0].shape[0], dtype=np.uint64)
    sh = 0
    for k in range(len(dims)):
        key |= cols[k].astype(np.uint64) << np.uint64(sh)
        sh += _bits(dims[k])
    return key


def _unpack(keys, dims):
    out = np.empty((keys.shape[0], len(dims)), dtype=np.int32)
    sh = 0
    for k, d in enumerate(dims):
        b = _bits(d)
        out[:, k] = ((keys >> np.uint64(sh)) & np.uint64((1 << b) - 1)).astype(np.int32)
        sh += b
    return out


def zipf_coords(rng, dims, nnz, s, oversample=1.7):
    """Distinct coordinates with Zipf(s) marginals per mode (see module doc).

    Raw draws are deduplicated; a uniformly random subset of exactly `nnz`
    distinct tuples is kept (topping up with fresh draws while short), and
    the result is returned in random order.
    """
    N = len(dims)
    if sum(_bits(d) for d in dims) > 64:
        return _zipf_coords_wide(rng, dims, nnz, s, oversample)
    pmfs = []
    for I in dims:
        w = np.arange(1, I + 1, dtype=np.float64) ** (-s)
        pmfs.append(w / w.sum())
    perms = [rng.permutation(I).astype(np.int32) for I in dims]
    have = np.zeros(0, dtype=np.uint64)
    while have.shape[0] < nnz:
        n = int((nnz - have.shape[0]) * oversample) + 1024
        cols = [_draw_zipf_mode(rng, n, pmfs[k], perms[k]) for k in range(N)]
        have = np.unique(np.concatenate([have, _pack(cols, dims)]))
        oversample = max(2.0, oversample * 1.5)
    keep = rng.permutation(have.shape[0])[:nnz]
    return _unpack(have[keep], dims)


def _zipf_coords_wide(rng, dims, nnz, s, oversample):
    """Same law as zipf_coords when the packed key needs more than 64 bits."""
    N = len(dims)
    split, acc = 0, 0
    for k in range(N):
        if acc + _bits(dims[k]) > 64:
            break
        acc += _bits(dims[k])
        split = k + 1
    pmfs = []
    for I in dims:
        w = np.arange(1, I + 1, dtype=np.float64) ** (-s)
        pmfs.append(w / w.sum())
    perms = [rng.permutation(I).astype(np.int32) for I in dims]
    rec = np.dtype([("hi", np.uint64), ("lo", np.uint64)])
    have = np.zeros(0, dtype=rec)
    while have.shape[0] < nnz:
        n = int((nnz - have.shape[0]) * oversample) + 1024
        cols = [_draw_zipf_mode(rng, n, pmfs[k], perms[k]) for k in range(N)]
        new = np.empty(n, dtype=rec)
        new["lo"] = _pack(cols[:split], dims[:split])
        new["hi"] = _pack(cols[split:], dims[split:])
        have = np.unique(np.concatenate([have, new]))
        oversample = max(2.0, oversample * 1.5)
    keep = rng.permutation(have.shape[0])[:nnz]
    sel = have[keep]
    return np.concatenate([_unpack(sel["lo"], dims[:split]),
                           _unpack(sel["hi"], dims[split:])], axis=1)


def uniform_coords(rng, dims, nnz):
    """Distinct coordinates drawn uniformly without replacement."""
    total = int(np.prod(dims, dtype=np.float64))
    flat = rng.choice(total, size=nnz, replace=False)
    out = np.empty((nnz, len(dims)), dtype=np.int32)
    for k, d in enumerate(dims):
        out[:, k] = flat % d
        flat = flat // d
    return out


def planted_factors(rng, dims, rank):
    return [rng.standard_normal((d, rank)) for d in dims]


def planted_values(rng, idx, dims, rank, noise_var=0.0, factors=None):
    """Entries of a planted rank-`rank` CP model (unit weights) + N(0, noise_var)."""
    if factors is None:
        factors = planted_factors(rng, dims, rank)
    prod = np.ones((idx.shape[0], rank))
    for k, F in enumerate(factors):
        prod *= F[idx[:, k]]
    v = prod.sum(axis=1)
    if noise_var > 0:
        v = v + rng.standard_normal(v.shape[0]) * np.sqrt(noise_var)
    return v, factors


def lognormal_values(rng, n, dtype=np.float32):
    return np.exp(rng.standard_normal(n)).astype(dtype)


def poisson_values(rng, n, lam=3.0, dtype=np.float32):
    return (rng.poisson(lam, n) + 1).astype(dtype)


def init_factors(rng, dims, R, dtype=np.float64):
    """Unit-variance Gaussian initial factors (Alg. 1, first line)."""
    out = [rng.standard_normal((d, R)) for d in dims]
    if dtype == np.float32:
        out = [f.astype(np.float32).astype(np.float64) for f in out]
    return out


def uniform_block(rng, J, N):
    """One block of uniforms in [0,1): J rows, one column per mode != j."""
    return rng.random((J, N - 1))


def uniform_blocks(rng, sweeps, J, N):
    """Uniform blocks in (sweep, mode) order: shape [sweeps, N, J, N-1]."""
    return rng.random((sweeps, N, J, N - 1))


# --------------------------------------------------------------------------
# Device generation (torch on the GPU) for tensors of 10^8 - 10^9 nonzeros.
# Same laws as above (Zipf(s) marginals with a seeded per-mode relabelling,
# distinct coordinates topped up to exactly nnz, lognormal or Poisson(3)+1
# values, N(0,1) initial factors), drawn from torch's counter-based
# generator instead of NumPy's PCG64: a different stream of the same
# distribution.  Input generation only.
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _dev_pack(cols, bits):
    """Pack per-mode coordinates (int64 tensors) into one int64 key per
    nonzero (bit fields, first mode lowest; at most 64 bits in total)."""
    key = None
    sh = 0
    for c, b in zip(cols, bits):
        part = c << sh
        key = part if key is None else key | part
        sh += b
    return key


def _dev_unpack(key, bits, out, col0):
    torch = _torch()
    sh = 0
    for k, b in enumerate(bits):
        out[:, col0 + k] = ((key >> sh) & ((1 << b) - 1)).to(torch.int32)
        sh += b


_GOLD = -7046029254386353131  # 0x9E3779B97F4A7C15 as a signed int64


def _hash_part(a, nparts):
    """Part of each key (same key, same part): top bits of a multiplicative
    hash, so that parts are of about equal size whatever the key law."""
    torch = _torch()
    h = (a * _GOLD) >> 40           # arithmetic shift; wraps like uint64
    return torch.remainder(h, nparts)


_PART = 1 << 30  # elements per sort / mask / unique call (index limits)


def _unique_parts(ka, kb=None, log=None):
    """Distinct keys (or key pairs) of the chunks ka (and kb), as a list of
    (a, b or None) tensors, one per hash part; every call on a tensor stays
    below 2^30 elements."""
    torch = _torch()
    total = sum(x.shape[0] for x in ka)
    nparts = max(1, -(-total // _PART) * 2)
    pieces = [[] for _ in range(nparts)]
    for i, a in enumerate(ka):
        b = None if kb is None else kb[i]
        if nparts == 1:
            pieces[0].append((a, b))
            continue
        part = _hash_part(a if b is None else a ^ (b * 31), nparts)
        for p in range(nparts):
            m = part == p
            pieces[p].append((a[m], None if b is None else b[m]))
            del m
        del part
    ka.clear()
    if kb is not None:
        kb.clear()
    outs = []
    for p in range(nparts):
        if log:
            log(f"tensorgen: part {p + 1} of {nparts}")
        sa = torch.cat([x for x, _ in pieces[p]])
        sb = None if kb is None else torch.cat([y for _, y in pieces[p]])
        pieces[p] = None
        if sb is None:
            outs.append((torch.unique(sa), None))
        else:
            o1 = torch.argsort(sb, stable=True)
            sa, sb = sa[o1], sb[o1]
            o2 = torch.argsort(sa, stable=True)
            sa, sb = sa[o2], sb[o2]
            del o1, o2
            first = torch.ones(sa.shape[0], dtype=torch.bool, device=sa.device)
            first[1:] = (sa[1:] != sa[:-1]) | (sb[1:] != sb[:-1])
            outs.append((sa[first], sb[first]))
            del first
        del sa, sb
    return outs


def zipf_draws_device(g, cdf, perm, m):
    """m i.i.d. labels: rank r (0-based) with probability cdf[r] - cdf[r-1]
    by inverse CDF of a uniform, then relabelled as perm[r]."""
    torch = _torch()
    u = torch.rand(m, dtype=torch.float64, device=cdf.device, generator=g)
    r = torch.searchsorted(cdf, u).clamp_(max=cdf.shape[0] - 1)
    return perm[r]


def zipf_coords_device(seed, dims, nnz, s, device, oversample=1.6,
                       chunk=1 << 27, log=None):
    """Distinct coordinates with Zipf(s) marginals per mode, on `device`.

    Raw draws are packed into one or two int64 keys (modes split where 64
    bits would be exceeded), deduplicated, and a random subset of exactly
    nnz distinct tuples is returned (int32 [nnz, N], grouped by hash part,
    sorted by key within a part).
    """
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    N = len(dims)
    bits = [_bits(d) for d in dims]
    split, acc = N, 0  # modes [0, split) in key A, [split, N) in key B
    for k in range(N):
        if acc + bits[k] > 64:
            split = k
            break
        acc += bits[k]
    cdfs, perms = [], []
    for I in dims:
        w = torch.arange(1, I + 1, dtype=torch.float64, device=device) ** (-s)
        c = torch.cumsum(w, 0)
        cdfs.append(c / c[-1])
        perms.append(torch.randperm(I, generator=g, device=device))
        del w, c
    parts = []  # distinct keys so far, per hash part: [(a, b or None)]
    chunk = min(chunk, _PART)
    have = 0
    while have < nnz:
        n = int((nnz - have) * oversample) + 1024
        ka = [x for x, _ in parts]
        kb = [y for _, y in parts] if split < N else None
        parts = None
        for c0 in range(0, n, chunk):
            m = min(chunk, n - c0)
            cols = [zipf_draws_device(g, cdfs[k], perms[k], m)
                    for k in range(N)]
            ka.append(_dev_pack(cols[:split], bits[:split]))
            if split < N:
                kb.append(_dev_pack(cols[split:], bits[split:]))
            del cols
        if log:
            log(f"tensorgen: {n} draws packed; deduplicating")
        parts = _unique_parts(ka, kb, log)
        have = sum(x.shape[0] for x, _ in parts)
        if log:
            log(f"tensorgen: {have} distinct of {nnz} wanted")
        oversample = max(1.3, oversample * 1.2)
    # exactly nnz of them: each part keeps its share k of its n distinct
    # tuples by Bernoulli(k / n) thinning, the few (about sqrt(k)) kept too
    # many or too few settled at the part's end
    out = torch.empty((nnz, N), dtype=torch.int32, device=device)
    at, left = 0, nnz
    for i, (a, b) in enumerate(parts):
        n_p = a.shape[0]
        k = left if i == len(parts) - 1 else int(round(nnz * n_p / have))
        k = min(k, n_p, left)
        keep = torch.rand(n_p, generator=g, device=device) < (k / n_p)
        m = int(keep.sum())
        if m > k:  # drop the last m - k kept
            pos = torch.nonzero(keep).squeeze(1)
            keep[pos[k:]] = False
            del pos
        elif m < k:  # add the first k - m not kept
            pos = torch.nonzero(~keep).squeeze(1)
            keep[pos[:k - m]] = True
            del pos
        _dev_unpack(a[keep], bits[:split], out[at:at + k], 0)
        if split < N:
            _dev_unpack(b[keep], bits[split:], out[at:at + k], split)
        at += k
        left -= k
        del keep
    assert at == nnz, (at, nnz)
    del parts, cdfs, perms
    return out


def values_device(seed, n, kind, device):
    """lognormal exp(N(0,1)) or Poisson(3) + 1 values, FP32, on `device`."""
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    if kind == "poisson":
        lam = torch.full((n,), 3.0, dtype=torch.float32, device=device)
        return torch.poisson(lam, generator=g) + 1.0
    return torch.exp(torch.randn(n, dtype=torch.float32, device=device,
                                 generator=g))


def init_factors_device(seed, dims, R, device, dtype=None):
    """Unit-variance Gaussian initial factors (Alg. 1, first line) as FP32
    tensors (so that every precision form starts from identical factors;
    the library takes them as FP64, converted one mode at a time)."""
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return [torch.randn((d, R), dtype=torch.float32, device=device,
                        generator=g) for d in dims]


def init_factors_slice_scaled_device(seed, dims, R, idx):
    """Gaussian initial factors whose row i of mode k is scaled by
    sqrt(number of nonzeros in slice i of mode k) (rows of empty slices are
    zero), FP32.  A data-aware start for
    tensors whose unfoldings have far more columns than nonzeros (the 4-way
    workload: about 1e14 columns per unfolding for 2e8 nonzeros): from
    unscaled Gaussian rows the leverage laws are nearly uniform, the draws
    of the first solve hit almost no nonempty column and the sampled
    MTTKRP is zero."""
    torch = _torch()
    U = init_factors_device(seed, dims, R, idx.device)
    for k, d in enumerate(dims):
        cnt = torch.bincount(idx[:, k].long(), minlength=d).to(torch.float32)
        U[k] = U[k] * cnt.sqrt()[:, None]
    return U


def uniforms_device(seed, shape, device):
    """Uniform [0, 1) blocks (FP64) on `device`."""
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.rand(shape, dtype=torch.float64, device=device, generator=g)


def make_tensor_device(name, device, nnz=None, dims=None, log=None):
    """Build one named power-law workload on `device`: (dims, idx int32
    [nnz, N], val float32 [nnz]) as torch tensors."""
    w = WORKLOADS[name]
    dims = tuple(dims or w["dims"])
    nnz = int(nnz or w["nnz"])
    base = 2210_5105 * 16 + int(w["tag"])
    idx = zipf_coords_device(base, dims, nnz, w["s"], device, log=log)
    val = values_device(base + 7, nnz,
                        "poisson" if name == "zipf4" else "lognormal", device)
    return dims, idx, val


WORKLOADS = {
    "planted": dict(dims=(200, 150, 100), nnz=20_000, R=8, J=4096,
                    sampler="arls", sweeps=10, tag=1),
    "zipf3": dict(dims=(100_000, 80_000, 60_000), nnz=50_000_000, s=1.1,
                  R=32, J=65536, sampler="sts", sweeps=20, tag=2),
    "zipf4": dict(dims=(1_000_000, 500_000, 200_000, 1_000),
                  nnz=200_000_000, s=1.2, R=64, J=131072, sampler="arls",
                  sweeps=20, tag=3, init="slice_scaled"),
    "zipf3xl": dict(dims=(8_000_000, 8_000_000, 200_000),
                    nnz=1_500_000_000, s=1.05, R=100, J=262144,
                    sampler="sts", sweeps=10, tag=4),
    "batch3": dict(dims=(500_000, 300_000, 100_000), nnz=100_000_000, s=1.1,
                   J=32768, sampler="arls", sweeps=10, tag=5),
}


def make_tensor(name, nnz=None, dims=None):
    """Build one named workload (optionally shrunk: nnz/dims override)."""
    w = WORKLOADS[name]
    dims = tuple(dims or w["dims"])
    nnz = int(nnz or w["nnz"])
    rc, rv, _, _ = streams(w["tag"])
    if name == "planted":
        idx = uniform_coords(rc, dims, nnz)
        v, _ = planted_values(rv, idx, dims, w["R"], noise_var=0.01)
        return SparseTensor(dims, idx, v.astype(np.float64))
    idx = zipf_coords(rc, dims, nnz, w["s"])
    if name == "zipf4":
        v = poisson_values(rv, nnz)
    else:
        v = lognormal_values(rv, nnz)
    return SparseTensor(dims, idx, v)


def tiny_tensor(seed, dims, nnz, rank=3, noise_var=0.0, dtype=np.float64):
    """Small tensor for tests: uniform distinct coordinates, planted values."""
    rc, rv, _, _ = streams([99, seed])
    idx = uniform_coords(rc, dims, nnz)
    v, F = planted_values(rv, idx, dims, rank, noise_var=noise_var)
    return SparseTensor(tuple(dims), idx, v.astype(dtype)), F


def zipf_tensor(seed, dims, nnz, s=1.1, dtype=np.float32):
    """Small power-law tensor for tests (lognormal values)."""
    rc, rv, _, _ = streams([98, seed])
    idx = zipf_coords(rc, dims, nnz, s)
    return SparseTensor(tuple(dims), idx, lognormal_values(rv, nnz, dtype))
