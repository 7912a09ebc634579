"""HIP path vs FP64 oracle, element by element, through the C ABI.

Tolerances (from the project's parity bar): sample indices bit-exact except
within 1e-12 of a CDF boundary; extracted nonzero sets and merged draws
bit-exact; MTTKRP and factors within 1e-4 relative Frobenius error in FP32
(1e-10 in FP64, where only summation order differs); fit within 1e-3 (FP32)
and 1e-9 (FP64).
"""
import numpy as np
import pytest

import oracle as O
import tensorgen as tg
from tests.gpu_common import check_mode_solve, init_ctx, make_ctx
from tests.helpers import (compare_sts_indices, gpu_state, pinv_rtol,
                           rel_fro, to_np)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import load_library
    load_library()
    return torch.device("cuda:0")


# ------------------------------------------------------------------ Grams

@pytest.mark.parametrize("R", [1, 8, 17, 32, 48, 100, 128])
def test_gram_mfma_matches_oracle(dev, R):
    dims = (1000, 77, 33)
    T, _ = tg.tiny_tensor(40, dims, 3000)
    ctx = make_ctx(dev, T, R, "exact", "fp64", 1)
    U0, _ = init_ctx(ctx, dims, R, 1)
    for k in range(3):
        Un = O.normalize_columns(U0[k])[0]
        np.testing.assert_allclose(to_np(ctx.get_factor(k)), Un, rtol=1e-14,
                                   atol=1e-15)
        np.testing.assert_allclose(to_np(ctx.get_gram(k)), O.gram(Un),
                                   rtol=1e-13, atol=1e-13)
    ctx.close()


@pytest.mark.parametrize("R,rank", [(8, 8), (32, 32), (24, 20), (128, 100),
                                    (128, 128), (5, 1), (64, 0), (100, 100)])
def test_pinv_matches_oracle(dev, R, rank):
    from paper_2210_05105_amd import pinv
    rng = np.random.default_rng(R * 1000 + rank)
    if rank == 0:
        G = np.zeros((R, R))
    else:
        rows = rank if rank < R else R + 40
        U = rng.standard_normal((rows, R))
        U /= np.linalg.norm(U, axis=0)
        G = U.T @ U
    Gp = to_np(pinv(torch.from_numpy(G).to(dev)))
    ref = O.pinv_psd(G)
    assert rel_fro(Gp, ref) < 1e-10, rel_fro(Gp, ref)


# --------------------------------------------------------- mode solves

@pytest.mark.parametrize("R,J", [(8, 4096), (17, 1000), (1, 33), (128, 300)])
def test_arls_fp64_mode_solves(dev, R, J):
    T = tg.make_tensor("planted")
    ctx = make_ctx(dev, T, R, "arls", "fp64", J)
    _, runi = init_ctx(ctx, T.dims, R, 2)
    acc = 0
    for j in range(3):
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, "arls", 1e-10)
    assert acc <= 2
    f = ctx.fit()
    U, _ = gpu_state(ctx)
    fo = O.fit(T.idx, T.val, to_np(ctx.get_sigma()), U)
    assert abs(f - fo) < 1e-9
    ctx.close()


@pytest.mark.parametrize("R,J,leaf", [(8, 2048, 16), (16, 1500, 32),
                                      (32, 1024, 64), (48, 333, 16),
                                      (64, 256, 16), (72, 300, 64),
                                      (100, 256, 16), (100, 500, 32),
                                      (128, 200, 16)])
def test_sts_fp64_mode_solves(dev, R, J, leaf):
    T, _ = tg.tiny_tensor(41, (300, 250, 190), 30000, rank=4, noise_var=0.01)
    ctx = make_ctx(dev, T, R, "sts", "fp64", J, leaf)
    _, runi = init_ctx(ctx, T.dims, R, 3)
    acc = 0
    for j in range(3):
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, "sts", 1e-10)
    assert acc <= 2
    ctx.close()


@pytest.mark.parametrize("dims", [(300, 100, 90), (300, 60, 50)])
def test_sts_wide_rank_small_trees(dev, dims):
    """Rank 100 with 64-row leaves on tree factors of 65-128 rows (two
    leaves: the block that forms the pair of leaves also writes their
    parent, the root, and the factor's Gram) and of at most 64 rows (one
    leaf, the root)."""
    T, _ = tg.tiny_tensor(52, dims, 20000, rank=4, noise_var=0.01)
    R, J = 100, 256
    ctx = make_ctx(dev, T, R, "sts", "fp64", J, 64)
    _, runi = init_ctx(ctx, T.dims, R, 53)
    acc = 0
    for j in (0, 1, 2, 0):
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, "sts", 1e-10)
    assert acc <= 2
    ctx.close()


def test_sts_fp32_zipf_mode_solves(dev):
    T = tg.zipf_tensor(42, (3000, 2400, 1800), 200_000, s=1.1)
    R, J = 32, 4096
    ctx = make_ctx(dev, T, R, "sts", "fp32", J)
    _, runi = init_ctx(ctx, T.dims, R, 4, fp32=True)
    for j in range(3):
        u = tg.uniform_block(runi, J, 3)
        check_mode_solve(ctx, T, j, u, J, "sts", 1e-4)
    f = ctx.fit()
    U, _ = gpu_state(ctx)
    fo = O.fit(T.idx, T.val.astype(np.float64), to_np(ctx.get_sigma()), U)
    assert abs(f - fo) < 1e-3
    ctx.close()


def test_sts_wide_rank_fp32_deep_tree(dev):
    """Rank 100 (the streamed-fragment kernels) in FP32: mode 1 has 320,000
    rows, so it is drawn from a 20,000-leaf tree (depth 15) in mode 2's
    solve and as the flat first factor in mode 0's.  The tensor is dense
    enough in every mode's columns that a solve extracts nonzeros."""
    T, _ = tg.tiny_tensor(50, (30, 320_000, 24), 600_000, rank=3,
                          noise_var=0.01, dtype=np.float32)
    R, J = 100, 1536
    ctx = make_ctx(dev, T, R, "sts", "fp32", J, 16)
    _, runi = init_ctx(ctx, T.dims, R, 51, fp32=True)
    acc = 0
    for j in (2, 0, 1):
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, "sts", 1e-4)
    assert acc <= 2
    ctx.close()


def test_sts_leaf_per_factor(dev):
    """With sts_leaf = 0 each tree factor gets its own leaf size: F nearest
    to sqrt(94 I / (d J)) among 16, 32, 64, d = draws from the tree per
    sweep (mode 1: one, mode 2: two).  Here mode 1 (40,000 rows) gets 64-row
    leaves and mode 2 (2,000 rows) 16-row leaves in one context; the draws
    from both trees follow the oracle."""
    T, _ = tg.tiny_tensor(57, (300, 40_000, 2000), 80_000, rank=3,
                          noise_var=0.01)
    R, J = 24, 512
    ctx = make_ctx(dev, T, R, "sts", "fp64", J)
    for k, d in ((1, 1), (2, 2)):
        f = np.sqrt(94.0 * T.dims[k] / (d * J))
        want = 16 if f < 22.6 else 32 if f < 45.3 else 64
        F, n = ctx.sts_leaf(k)
        assert F == want, (k, F, want)
        assert n == 1 << int(np.ceil(np.log2(-(-T.dims[k] // F)))), (k, n)
    assert ctx.sts_leaf(0) == (0, 0)  # always drawn first: no tree
    assert ctx.sts_leaf(1)[0] == 64 and ctx.sts_leaf(2)[0] == 16
    _, runi = init_ctx(ctx, T.dims, R, 58)
    acc = 0
    for j in (2, 0, 1):
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, "sts", 1e-10)
    assert acc <= 2
    ctx.close()


def test_sts_long_first_factor(dev):
    """First drawn factor of 300k rows: more 64-row blocks than one level of
    group sums holds, so draws walk two 64-row blocks per group."""
    T, _ = tg.tiny_tensor(48, (300_000, 60, 45), 60_000, rank=3,
                          noise_var=0.01)
    R, J = 8, 4096
    ctx = make_ctx(dev, T, R, "sts", "fp64", J)
    _, runi = init_ctx(ctx, T.dims, R, 11)
    acc = 0
    for j in (1, 2):  # mode 0 is drawn first
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, "sts", 1e-10)
    assert acc <= 2
    ctx.close()


def test_mode_order_with_growing_bucket_count(dev):
    """Solves in the order 0, 1, 2, 1 where mode 1 has the most output-row
    buckets: per-mode bucket state must not leak between modes."""
    T, _ = tg.tiny_tensor(49, (200, 700, 300), 20_000, rank=3, noise_var=0.01)
    R, J = 8, 512
    ctx = make_ctx(dev, T, R, "sts", "fp64", J)
    _, runi = init_ctx(ctx, T.dims, R, 12)
    acc = 0
    for j in (0, 1, 2, 1):
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, "sts", 1e-10)
    assert acc <= 2
    ctx.close()


@pytest.mark.parametrize("sampler,prec,tol,B", [("arls", "fp32", 1e-4, 256),
                                               ("sts", "fp64", 1e-10, 256),
                                               ("arls", "fp64", 1e-10, 64)])
def test_bucket_rows_caller_set(dev, sampler, prec, tol, B):
    """Output-row buckets of the size the caller sets, up to 256 rows (the
    largest: a record keeps row mod B in 8 bits, and each bucket size has
    its own record regions in the context), for modes of 20,000, 6,000 and
    300 rows; solves in the order 0, 2, 1, 0."""
    T = tg.zipf_tensor(45, (20000, 6000, 300), 120_000, s=1.1)
    R, J = 16, 6000
    ctx = make_ctx(dev, T, R, sampler, prec, J, bucket_rows=B)
    _, runi = init_ctx(ctx, T.dims, R, 22, fp32=(prec != "fp64"))
    acc = 0
    for j in (0, 2, 1, 0):
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, sampler, tol)
    assert acc <= 2
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_two_pass_record_placement(dev, prec, tol):
    """Modes with more than 256 output-row buckets place the sampled
    MTTKRP's records in two passes (super buckets of 2^sh buckets, then
    buckets): 16-row buckets give mode 0 1,250 buckets (two passes, 8 per
    super bucket), mode 1 375 (two passes, 2 per super bucket) and mode 2 19
    (one pass).  Power-law rows put long runs in a few buckets.  The order
    0, 2, 1, 0 checks that the super-bucket cursors are left clear."""
    T = tg.zipf_tensor(44, (20000, 6000, 300), 120_000, s=1.1)
    R, J = 16, 6000
    ctx = make_ctx(dev, T, R, "arls", prec, J, bucket_rows=16)
    _, runi = init_ctx(ctx, T.dims, R, 21, fp32=(prec != "fp64"))
    for j in (0, 2, 1, 0):
        u = tg.uniform_block(runi, J, 3)
        check_mode_solve(ctx, T, j, u, J, "arls", tol)
    ctx.close()


def test_arls_fp32_4way_mode_solves(dev):
    T = tg.zipf_tensor(43, (2000, 1000, 400, 20), 150_000, s=1.2)
    R, J = 24, 3000
    ctx = make_ctx(dev, T, R, "arls", "fp32", J)
    _, runi = init_ctx(ctx, T.dims, R, 5, fp32=True)
    for j in range(4):
        u = tg.uniform_block(runi, J, 4)
        check_mode_solve(ctx, T, j, u, J, "arls", 1e-4)
    ctx.close()


# ----------------------------------------------------- end to end (C1)

def test_planted_end_to_end_fp64_ten_sweeps(dev):
    """200x150x100, 20k nnz, R=8, J=4096, CP-ARLS-LEV, 10 sweeps, FP64:
    identical init and uniforms, no teacher forcing; indices compared in
    every mode solve."""
    w = tg.WORKLOADS["planted"]
    T = tg.make_tensor("planted")
    R, J, sweeps = w["R"], w["J"], w["sweeps"]
    _, _, rinit, runi = tg.streams(w["tag"])
    U0 = tg.init_factors(rinit, T.dims, R)
    uni = tg.uniform_blocks(runi, sweeps, J, 3)
    ctx = make_ctx(dev, T, R, "arls", "fp64", J)
    for k in range(3):
        ctx.set_factor(k, torch.from_numpy(U0[k]))
    f0 = ctx.fit()
    U = [O.normalize_columns(x)[0] for x in U0]
    G = [O.gram(x) for x in U]
    st = {k: O.arls_build(U[k], G[k]) for k in range(3)}
    mism = 0
    for t in range(sweeps):
        for j in range(3):
            u = uni[t, j]
            gidx, _ = ctx.sample(j, torch.from_numpy(u))
            oidx, prob, h = O.arls_sample(U, st, j, u)
            mism += int(np.sum(to_np(gidx) != oidx))
            ctx.sampled_mttkrp(j, want_M=False)
            ctx.solve_factor(j)
            keys, rep, cnt, wts = O.dedup(oidx, prob, T.dims, j, J)
            ck, rows, vals, slot = O.extract(T.idx, T.val, T.dims, j, keys)
            M = O.sampled_mttkrp(T.dims[j], rows, vals, slot, wts, h[rep])
            U[j], sig = O.solve(M, O.pinv_psd(O.gram_hadamard(G, j)))
            G[j] = O.gram(U[j])
            st[j] = O.arls_build(U[j], G[j])
    assert mism == 0
    Ug, _ = gpu_state(ctx)
    for k in range(3):
        assert rel_fro(Ug[k], U[k]) < 1e-8
    f = ctx.fit()
    fo = O.fit(T.idx, T.val, sig, U)
    assert abs(f - fo) < 1e-9 and f > f0
    ctx.close()


def test_sweep_entry_point_matches_stepwise(dev):
    w = tg.WORKLOADS["planted"]
    T = tg.make_tensor("planted")
    R, J = w["R"], 1024
    uni = tg.uniform_blocks(np.random.default_rng(5), 3, J, 3)
    a = make_ctx(dev, T, R, "arls", "fp64", J)
    b = make_ctx(dev, T, R, "arls", "fp64", J)
    init_ctx(a, T.dims, R, 7)
    init_ctx(b, T.dims, R, 7)
    a.sweep(3, J, torch.from_numpy(uni))
    for t in range(3):
        for j in range(3):
            b.sample(j, torch.from_numpy(uni[t, j]), outputs=False)
            b.sampled_mttkrp(j, want_M=False)
            b.solve_factor(j)
    assert abs(a.fit() - b.fit()) < 1e-12
    for k in range(3):
        assert rel_fro(to_np(a.get_factor(k)), to_np(b.get_factor(k))) < 1e-12
    a.close()
    b.close()


# -------------------------------------------------------------- exact

def test_exact_mttkrp_and_als(dev):
    """Exact sampler: M is the exact MTTKRP; a solve and 3 sweeps track the
    oracle's exact ALS step for step."""
    dims, R = (40, 30, 20), 5
    T, _ = tg.tiny_tensor(44, dims, 5000, rank=R, noise_var=0.0)
    ctx = make_ctx(dev, T, R, "exact", "fp64", 1)
    U0, _ = init_ctx(ctx, dims, R, 8)
    U, G = gpu_state(ctx)
    M, n = ctx.sampled_mttkrp(1, want_nnz=True)
    assert n == T.nnz
    assert rel_fro(to_np(M), O.mttkrp_exact(T.idx, T.val, U, 1)) < 1e-13
    ctx.solve_factor(1)
    ctx.sweep(3)
    U = [O.normalize_columns(x)[0] for x in U0]
    G = [O.gram(x) for x in U]
    for j in [1] + [0, 1, 2] * 3:
        Mo = O.mttkrp_exact(T.idx, T.val, U, j)
        U[j], sig = O.solve(Mo, O.pinv_psd(O.gram_hadamard(G, j)))
        G[j] = O.gram(U[j])
    Ug, _ = gpu_state(ctx)
    for k in range(3):
        assert rel_fro(Ug[k], U[k]) < 1e-10
    assert abs(ctx.fit() - O.fit(T.idx, T.val, sig, U)) < 1e-10
    ctx.close()


# -------------------------------------------------------- invariances

def test_sts_leaf_size_invariance(dev):
    """The map u -> index does not depend on the leaf size F: for each F the
    draws match the oracle (which bisects prefix Grams of 64-row blocks and
    scans rows, no tree) outside the 1e-12 band."""
    T, _ = tg.tiny_tensor(45, (500, 300, 200), 20000, rank=3)
    R, J = 16, 2048
    u = tg.uniform_block(np.random.default_rng(6), J, 3)
    out = []
    for leaf in (16, 32, 64):
        ctx = make_ctx(dev, T, R, "sts", "fp64", J, leaf)
        init_ctx(ctx, T.dims, R, 9)
        U, G = gpu_state(ctx)
        gidx, gprob = ctx.sample(0, torch.from_numpy(u))
        gidx = to_np(gidx).astype(np.int64)
        for block in (64, 7):
            oidx, oprob, _ = O.sts_sample(U, G, 0, u, block=block)
            assert compare_sts_indices(gidx, oidx, U, G, 0, u) <= 1
        out.append(gidx)
        ctx.close()
    for gidx in out[1:]:
        assert np.sum(np.any(gidx != out[0], axis=1)) <= 1


# -------------------------------------------------------------- errors

def test_error_paths(dev):
    from paper_2210_05105_amd import CprError
    dims = (20, 10, 8)
    T, _ = tg.tiny_tensor(46, dims, 300)
    bad = tg.SparseTensor(dims, T.idx.copy(), T.val.copy())
    bad.idx[5, 1] = 10  # out of range
    with pytest.raises(CprError) as e:
        make_ctx(dev, bad, 4, "arls", "fp64", 16)
    assert e.value.name == "CP_EINVAL"
    dup = tg.SparseTensor(dims, T.idx.copy(), T.val.copy())
    dup.idx[7] = dup.idx[3]
    with pytest.raises(CprError) as e:
        make_ctx(dev, dup, 4, "arls", "fp64", 16)
    assert e.value.name == "CP_EINVAL"
    ctx = make_ctx(dev, T, 4, "arls", "fp64", 16)
    with pytest.raises(CprError) as e:
        ctx.sampled_mttkrp(0)
    assert e.value.name == "CP_ESTATE"  # factors not set yet
    init_ctx(ctx, dims, 4, 10)
    with pytest.raises(CprError) as e:
        ctx.sampled_mttkrp(0)
    assert e.value.name == "CP_ESTATE"  # no samples yet
    u = np.full((16, 2), 0.5)
    u[3, 1] = 1.0
    ctx.sample(0, torch.from_numpy(u))
    with pytest.raises(CprError) as e:
        ctx.sync()
    assert e.value.name == "CP_EINVAL"
    with pytest.raises(CprError) as e:
        ctx.sample(0, torch.from_numpy(np.full((17, 2), 0.5)))  # J > max_J
    assert e.value.name == "CP_EINVAL"
    ctx.set_factor(1, torch.zeros(dims[1], 4, dtype=torch.float64))
    with pytest.raises(CprError) as e:
        ctx.sync()
    assert e.value.name == "CP_EDEGENERATE"
    ctx.close()


def test_rank_deficient_gram_uses_pseudo_inverse(dev):
    dims, R, J = (60, 50, 40), 4, 512
    T, _ = tg.tiny_tensor(47, dims, 4000, rank=3)
    ctx = make_ctx(dev, T, R, "arls", "fp64", J)
    rng = np.random.default_rng(11)
    U0 = [rng.standard_normal((d, R)) for d in dims]
    U0[1][:, 3] = U0[1][:, 0]  # duplicated column: G_1 is singular
    for k in range(3):
        ctx.set_factor(k, torch.from_numpy(U0[k]))
    u = tg.uniform_block(rng, J, 3)
    check_mode_solve(ctx, T, 0, u, J, "arls", 1e-9)
    ctx.sync()
    ctx.close()
