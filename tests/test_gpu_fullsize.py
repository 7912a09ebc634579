"""Parity at the full benchmark size, in the benchmark's configuration.

100,000 x 80,000 x 60,000 Zipf(1.1) tensor with 50M nonzeros, R = 32,
J = 65,536 STS-CP draws per mode solve, FP32 MTTKRP with FP64 sampler and
solve.  The oracle cannot redo a whole solve at this size, so it checks
sampled outputs one by one, teacher-forced with the GPU's state: a random
subset of the draws (exact conditional inverse CDF), every merged column
weight (a full recount), a random subset of the rows of M (from the
nonzeros the oracle itself extracts by scanning the tensor), and the same
rows of the solved factor.
"""
import numpy as np
import pytest

import oracle as O
import tensorgen as tg
from tests.helpers import compare_sts_indices, gpu_state, pinv_rtol, rel_fro, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import Context, load_library
    load_library()
    dev = torch.device("cuda:0")
    w = dict(tg.WORKLOADS["zipf3"])
    T = tg.make_tensor("zipf3")
    R, J = w["R"], w["J"]
    ctx = Context(torch.from_numpy(T.idx).to(dev),
                  torch.from_numpy(T.val.astype(np.float32)).to(dev), T.dims,
                  R, "sts", "fp32", max_J=J)
    _, _, rinit, runi = tg.streams(w["tag"])
    U0 = tg.init_factors(rinit, T.dims, R, dtype=np.float32)
    for k in range(T.N):
        ctx.set_factor(k, torch.from_numpy(U0[k]))
    uni = tg.uniform_blocks(runi, 2, J, T.N)
    # one ALS sweep first, so the factors are those of a running solve
    ctx.sweep(1, J, torch.from_numpy(uni[:1]).to(dev))
    ctx.sync()
    yield dict(ctx=ctx, T=T, R=R, J=J, u=uni[1], dev=dev)
    ctx.close()


def test_fullsize_mode_solve(big):
    ctx, T, R, J = big["ctx"], big["T"], big["R"], big["J"]
    dims, j = T.dims, 0
    u = big["u"][j]
    rng = np.random.default_rng(20)
    U, G = gpu_state(ctx)
    gidx, gprob = ctx.sample(j, torch.from_numpy(u))
    gidx, gprob = to_np(gidx).astype(np.int64), to_np(gprob)
    # (1) draws: a random subset against the exact conditional inverse CDF
    S = np.sort(rng.choice(J, 256, replace=False))
    oidx, oprob, _ = O.sts_sample(U, G, j, u[S], block=64)
    n_acc = compare_sts_indices(gidx[S], oidx, U, G, j, u[S])
    assert n_acc <= 2, n_acc  # in-band mismatches are rare: 256 draws
    same = np.all(gidx[S] == oidx, axis=1)
    others = [G[k] for k in range(len(dims)) if k != j]
    others.append(O.gram_hadamard(G, j))
    np.testing.assert_allclose(gprob[S][same], oprob[same],
                               rtol=pinv_rtol(1e-11, *others))
    # (2) merge: every distinct column, its first draw, count and weight
    keys, rep, counts, wts = O.dedup(gidx, gprob, dims, j, J)
    ck, rows, vals, slot = O.extract(T.idx, T.val, dims, j, keys)
    live = np.isin(keys, ck)  # sampled columns holding nonzeros
    uq = ctx.get_unique(J)
    order = np.argsort(to_np(uq["col_key"]))
    np.testing.assert_array_equal(to_np(uq["col_key"])[order].astype(np.uint64),
                                  keys[live])
    np.testing.assert_array_equal(to_np(uq["rep"])[order], rep[live])
    np.testing.assert_array_equal(to_np(uq["count"])[order], counts[live])
    np.testing.assert_allclose(to_np(uq["weight"])[order], wts[live],
                               rtol=1e-14)
    # (3) M on a random subset of rows, from the oracle's own extraction
    Mg, nz = ctx.sampled_mttkrp(j, want_nnz=True)
    Mg = to_np(Mg).astype(np.float64)
    assert nz == rows.shape[0]
    modes = [k for k in range(len(dims)) if k != j]
    h = np.ones((J, R))
    for q, k in enumerate(modes):
        h = h * U[k][gidx[:, q]]
    pick = np.sort(rng.choice(dims[j], 1500, replace=False))
    sel = np.isin(rows, pick)
    Mo = O.sampled_mttkrp(dims[j], rows[sel], vals[sel], slot[sel], wts,
                          h[rep])
    assert rel_fro(Mg[pick], Mo[pick]) < 1e-4
    # (4) the solved rows, teacher-forced with the GPU's M
    ctx.solve_factor(j)
    Uj = to_np(ctx.get_factor(j))
    sig = to_np(ctx.get_sigma())
    Gp = O.pinv_psd(O.gram_hadamard(G, j))
    X = Mg[pick] @ Gp
    nz_cols = sig > 0
    Xn = np.zeros_like(X)
    Xn[:, nz_cols] = X[:, nz_cols] / sig[nz_cols]
    assert rel_fro(Uj[pick], Xn) < pinv_rtol(1e-5, O.gram_hadamard(G, j))
