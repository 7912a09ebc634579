"""Shared GPU-test helpers: context construction and the teacher-forced
check of one mode solve (HIP path vs FP64 oracle).  Imported only by tests
marked gpu."""
import numpy as np
import torch

import oracle as O
import tensorgen as tg
from tests.helpers import (compare_arls_indices, compare_sts_indices,
                           gpu_state, oracle_sampled_M, pinv_rtol, rel_fro,
                           to_np)


def make_ctx(dev, T, R, sampler, precision, J, leaf=0, refine=None,
             bucket_rows=0):
    from paper_2210_05105_amd import Context
    vdt = np.float64 if precision == "fp64" else np.float32
    return Context(torch.from_numpy(np.ascontiguousarray(T.idx)).to(dev),
                   torch.from_numpy(T.val.astype(vdt)).to(dev), T.dims, R,
                   sampler, precision, max_J=J, sts_leaf=leaf, refine=refine,
                   bucket_rows=bucket_rows)


def init_ctx(ctx, dims, R, seed, fp32=False):
    _, _, rinit, runi = tg.streams([96, seed])
    U0 = tg.init_factors(rinit, dims, R,
                         dtype=np.float32 if fp32 else np.float64)
    for k in range(len(dims)):
        ctx.set_factor(k, torch.from_numpy(U0[k]))
    return U0, runi


def gram_rtol(ctx):
    """Tolerance of a factor Gram against the oracle's U^T U of the stored
    factor: FP64 Grams differ only in summation order; FP32-MFMA Grams
    accumulate FP32 partial sums; the split-BF16 Grams of the mixed form
    carry about 2^-16 relative error per product."""
    return {"fp64": 1e-12, "fp32": 1e-5, "mixed": 1e-4}[ctx.precision]


def check_draws(ctx, T, j, u, sampler):
    """The GPU's draws for uniforms u against the oracle's, teacher-forced
    with the GPU's factors and Grams.  Returns (gidx, gprob, U, G, n_acc)."""
    dims = T.dims
    U, G = gpu_state(ctx)
    gidx, gprob = ctx.sample(j, torch.from_numpy(u))
    gidx, gprob = to_np(gidx).astype(np.int64), to_np(gprob)
    if sampler == "arls":
        st = {k: O.arls_build(U[k], G[k]) for k in range(len(dims)) if k != j}
        oidx, oprob, _ = O.arls_sample(U, st, j, u)
        n_acc = compare_arls_indices(gidx, oidx, U, G, j, u)
    else:
        # prefix-Gram blocks of the oracle: 64 rows, or coarser for long
        # factors at high rank (its prefix Grams are (I / block) R^2 long
        # doubles); the draws do not depend on the block size
        big = max(U[k].shape[0] for k in range(len(dims)) if k != j)
        block = 64 if big * U[0].shape[1] ** 2 <= 4e9 else 1024
        oidx, oprob, _ = O.sts_sample(U, G, j, u, block=block)
        n_acc = compare_sts_indices(gidx, oidx, U, G, j, u)
    same = np.all(gidx == oidx, axis=1)
    others = [G[k] for k in range(len(dims)) if k != j]
    if sampler == "sts":
        others.append(O.gram_hadamard(G, j))
    np.testing.assert_allclose(gprob[same], oprob[same],
                               rtol=pinv_rtol(1e-11, *others))
    return gidx, gprob, U, G, n_acc


def _sorted_triples(ck, row, rep):
    ck = np.asarray(ck).astype(np.uint64)
    row = np.asarray(row).astype(np.int64)
    rep = np.asarray(rep).astype(np.int64)
    o = np.lexsort((rep, row, ck))
    return ck[o], row[o], rep[o]


def check_after_draws(ctx, T, j, gidx, gprob, U, G, J, tol):
    """Merge, extraction, M, U_j, sigma and G_j for the draws (gidx, gprob)
    the context holds, against the oracle on the same draws."""
    dims = T.dims
    ref = oracle_sampled_M(T, dims, j, gidx, gprob, U, J)
    uq = ctx.get_unique(J)
    order = np.argsort(to_np(uq["col_key"]).astype(np.uint64))
    # sampled columns without nonzeros contribute nothing and are not listed
    live = np.isin(ref["keys"], O.column_key(T.idx, dims, j))
    np.testing.assert_array_equal(to_np(uq["col_key"])[order].astype(np.uint64),
                                  ref["keys"][live])
    np.testing.assert_array_equal(to_np(uq["rep"])[order], ref["rep"][live])
    np.testing.assert_array_equal(to_np(uq["count"])[order],
                                  ref["counts"][live])
    np.testing.assert_allclose(to_np(uq["weight"])[order], ref["w"][live],
                               rtol=1e-14)
    ex = ctx.get_extracted(max(1, ref["rows"].shape[0] + 16))
    assert ex["n"] == ref["rows"].shape[0]
    g = _sorted_triples(to_np(ex["col_key"]), to_np(ex["row"]),
                        to_np(ex["rep"]))
    o = _sorted_triples(ref["ck"], ref["rows"], ref["rep"][ref["slot"]])
    for a, b in zip(g, o):
        np.testing.assert_array_equal(a, b)
    M, nnz = ctx.sampled_mttkrp(j, want_nnz=True)
    assert nnz == ref["rows"].shape[0]
    M = to_np(M).astype(np.float64)
    assert rel_fro(M, ref["M"]) < tol, rel_fro(M, ref["M"])
    # solve from the GPU's M
    ctx.solve_factor(j)
    Uj = to_np(ctx.get_factor(j))
    sig = to_np(ctx.get_sigma())
    Gh = O.gram_hadamard(G, j)
    Uo, so = O.solve(M, O.pinv_psd(Gh))
    stol = pinv_rtol(tol, Gh)
    assert rel_fro(Uj, Uo) < stol, (rel_fro(Uj, Uo), stol)
    np.testing.assert_allclose(sig, so, rtol=stol)
    gt = gram_rtol(ctx)
    np.testing.assert_allclose(to_np(ctx.get_gram(j)), O.gram(Uj),
                               rtol=gt, atol=gt)
    return ref


def check_mode_solve(ctx, T, j, u, J, sampler, tol):
    """One teacher-forced mode solve: draws, merge, extraction, M, U_j, G_j.
    Returns the number of accepted in-band index mismatches."""
    gidx, gprob, U, G, n_acc = check_draws(ctx, T, j, u, sampler)
    check_after_draws(ctx, T, j, gidx, gprob, U, G, J, tol)
    return n_acc
