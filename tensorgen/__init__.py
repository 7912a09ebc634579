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
  batch3   : 500000x300000x100000, 100M nnz, Zipf(1.1), lognormal

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


WORKLOADS = {
    "planted": dict(dims=(200, 150, 100), nnz=20_000, R=8, J=4096,
                    sampler="arls", sweeps=10, tag=1),
    "zipf3": dict(dims=(100_000, 80_000, 60_000), nnz=50_000_000, s=1.1,
                  R=32, J=65536, sampler="sts", sweeps=20, tag=2),
    "zipf4": dict(dims=(1_000_000, 500_000, 200_000, 1_000),
                  nnz=200_000_000, s=1.2, R=64, J=131072, sampler="arls",
                  sweeps=20, tag=3),
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
