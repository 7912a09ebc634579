"""CPU-only checks of the C ABI library and the host-side logic.

No compute call reaches the GPU here: the library is loaded, its exported
symbols are compared with include/cpr.h, and argument validation that
happens before any HIP call is exercised.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import tensorgen as tg
import paper_2210_05105_amd as pkg
from paper_2210_05105_amd import binding


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2210_05105_amd.build import build_library
        build_library()
    return pkg.load_library()


def test_every_declared_symbol_is_exported(lib):
    decl = pkg.declared_symbols()
    assert len(decl) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [s for s in decl if s not in exported]
    assert not missing, missing
    for s in decl:
        assert hasattr(lib, s)


def test_library_is_gfx950_only(lib):
    import re
    with open(binding.LIB_PATH, "rb") as f:
        blob = f.read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa-+(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}


def _init(lib, N=3, dims=(4, 5, 6), nnz=10, R=4, sampler=0, precision=0,
          max_J=8, leaf=0, idx=1, val=1, bucket_rows=0, solve_gram=0,
          solve_refine=0):
    d = (C.c_int64 * max(N, 1))(*list(dims)[:max(N, 1)])
    t = binding._Tensor(N, d, nnz, idx, val, 1)
    cfg = binding._Config(R, sampler, precision, leaf, max_J, bucket_rows,
                          solve_gram, solve_refine)
    h = C.c_void_p()
    st = lib.cp_init(C.byref(t), C.byref(cfg), None, C.byref(h))
    return st, h


@pytest.mark.parametrize("kw", [dict(N=2, dims=(4, 5)), dict(N=9, dims=(2,) * 9),
                                dict(nnz=0), dict(R=0), dict(R=129),
                                dict(sampler=3), dict(precision=3),
                                dict(max_J=0), dict(leaf=8),
                                dict(bucket_rows=48), dict(bucket_rows=512),
                                dict(bucket_rows=8), dict(solve_gram=2),
                                dict(solve_refine=3), dict(solve_refine=-1),
                                dict(dims=(4, 0, 6)), dict(dims=(4, 2**31, 6)),
                                dict(idx=None), dict(val=None)])
def test_init_rejects_bad_arguments_before_touching_the_gpu(lib, kw):
    st, h = _init(lib, **kw)
    assert st == -1 and not h.value


def test_status_and_phase_names(lib):
    assert lib.cp_status_string(0) == b"CP_OK"
    assert lib.cp_status_string(-5) == b"CP_EDEGENERATE"
    names = [lib.cp_phase_name(i).decode() for i in range(8)]
    assert names == binding.PHASES
    assert lib.cp_last_error(None) == b"null context"
    # calls on a null context fail cleanly
    assert lib.cp_sync(None) == -1
    assert lib.cp_fit(None, None) == -1


def test_binding_fails_loudly_without_library(tmp_path):
    saved = binding._lib
    binding._lib = None
    try:
        with pytest.raises(ImportError):
            binding.load_library(str(tmp_path / "missing.so"))
    finally:
        binding._lib = saved


# ------------------------------------------------------------ generators

def test_zipf_generator_exact_distinct_and_in_range():
    dims = (5000, 4000, 3000)
    idx = tg.zipf_coords(np.random.default_rng(1), dims, 200_000, 1.1)
    assert idx.shape == (200_000, 3) and idx.dtype == np.int32
    for k, d in enumerate(dims):
        assert idx[:, k].min() >= 0 and idx[:, k].max() < d
    key = idx[:, 0].astype(np.int64) * 10**8 + idx[:, 1] * 10**4 + idx[:, 2]
    assert np.unique(key).shape[0] == idx.shape[0]
    # power law: the most frequent index of a mode is much heavier than the
    # median one
    c = np.bincount(idx[:, 0], minlength=dims[0])
    assert c.max() > 50 * max(1, np.median(c))


def test_zipf_generator_wide_keys():
    dims = (1_000_000, 500_000, 200_000, 1_000)   # > 64 bits of coordinates
    idx = tg.zipf_coords(np.random.default_rng(2), dims, 20_000, 1.2)
    assert idx.shape == (20_000, 4)
    assert np.unique(idx, axis=0).shape[0] == 20_000


def test_uniform_generator_and_planted_values():
    T = tg.make_tensor("planted")
    assert T.nnz == 20_000 and T.dims == (200, 150, 100)
    flat = (T.idx[:, 0].astype(np.int64) * 150 + T.idx[:, 1]) * 100 + T.idx[:, 2]
    assert np.unique(flat).shape[0] == T.nnz
    rng = np.random.default_rng(3)
    v, F = tg.planted_values(rng, T.idx[:10], T.dims, 2)
    ref = sum(F[0][T.idx[:10, 0], r] * F[1][T.idx[:10, 1], r] *
              F[2][T.idx[:10, 2], r] for r in range(2))
    np.testing.assert_allclose(v, ref)


def test_autotune_cache_roundtrip(tmp_path, monkeypatch):
    """The tuner's cache file: stored results are returned for the same
    problem key, and nothing else is touched."""
    from paper_2210_05105_amd import autotune as at
    path = tmp_path / "tune.json"
    monkeypatch.setenv("CPR_TUNE_CACHE", str(path))
    assert at.cache_path() == str(path)
    assert at._load(str(path)) == {}
    at._store(str(path), {"k": {"sts_leaf": 32, "bucket_rows": 128}})
    assert at._load(str(path))["k"]["sts_leaf"] == 32
    assert at.LEAVES == (0, 16, 32, 64) and 128 in at.BUCKETS
