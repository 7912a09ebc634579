"""Parity at the billion-nonzero size, in the benchmark's configuration.

8,000,000 x 8,000,000 x 200,000 Zipf tensor with 1.5B nonzeros (generated
on the device), R = 100, J = 262,144 STS-CP draws per mode solve, mixed
precision (FP32 factors and MTTKRP, split-BF16 Grams, FP64 sampler, FP32
row solve), leaf rows chosen per tree factor (64 for mode 1, 16 for mode
2).  After one ALS sweep the mode-2 solve is checked, teacher-forced with
the GPU's factors and Grams, on outputs the oracle's definitions fix one by
one (a whole oracle solve does not fit this size):
- every draw of the first factor (mode 0, 8M rows, drawn flat): the index
  min{i : uZ < F(i)} over the 8M row masses U[i] G_{>0} U[i]^T (R5, R10);
- four draws of the tree factor (mode 1, a 131,072-leaf tree): the same
  over their conditional law given the first factor's row (Appendix B);
- every merged column: first draw, count and weight count/(J p); every
  sampled column the GPU does not list holds no nonzero;
- 1,000 rows of M from the nonzeros the oracle selects in those rows;
- the same rows of the solved factor.
Index mismatches are accepted only within 1e-12 of a CDF boundary; the
CDFs are prefix sums in extended precision.
"""
import numpy as np
import pytest

import oracle as O
import tensorgen as tg
from oracle.cpals import _g_after
from tests.helpers import BAND, gpu_state, pinv_rtol, rel_fro, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CH = 1 << 20  # rows per host chunk


def _masses(U, W, h=None):
    """m_i = (U[i] (*) h) W (U[i] (*) h)^T for every row, FP64 (chunked)."""
    m = np.empty(U.shape[0])
    for c0 in range(0, U.shape[0], CH):
        X = U[c0:c0 + CH] if h is None else U[c0:c0 + CH] * h
        m[c0:c0 + CH] = np.einsum("ia,ia->i", X @ W, X)
    return np.where(m > 0, m, 0.0)  # zero-mass rows are never chosen


def _draw_check(m, u, gi):
    """GPU indices gi against min{i : uZ < F(i)}; returns mismatches (each
    asserted to lie within BAND of a CDF boundary)."""
    F = np.cumsum(m.astype(np.longdouble))
    Z = F[-1]
    oi = np.searchsorted(F, np.asarray(u, dtype=np.longdouble) * Z,
                         side="right")
    oi = np.minimum(oi, m.shape[0] - 1)
    bad = np.nonzero(oi != gi)[0]
    for s in bad:
        lo, hi = sorted((int(oi[s]), int(gi[s])))
        gap = max(abs(F[lo] / Z - u[s]), abs(F[hi - 1] / Z - u[s]))
        assert gap <= BAND, (s, gi[s], oi[s], float(gap))
    return bad.size


@pytest.fixture(scope="module")
def xl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import Context, load_library
    load_library()
    dev = torch.device("cuda:0")
    w = dict(tg.WORKLOADS["zipf3xl"])
    dims, idx, val = tg.make_tensor_device("zipf3xl", dev)
    R, J = w["R"], w["J"]
    base = 2210_5105 * 16 + int(w["tag"])
    ctx = Context(idx, val, dims, R, "sts", "mixed", max_J=J)
    U0 = tg.init_factors_device(base + 11, dims, R, dev)
    for k in range(3):
        ctx.set_factor(k, U0[k])
    del U0
    uni = tg.uniforms_device(base + 29, (2, 3, J, 2), dev)
    ctx.sweep(1, J, uni[:1])  # the factors of a running solve
    ctx.sync()
    yield dict(ctx=ctx, dims=dims, idx=idx, val=val, R=R, J=J,
               u=uni[1, 2].cpu().numpy(), dev=dev)
    ctx.close()
    del idx, val, uni
    torch.cuda.empty_cache()


def test_xl_mode_solve(xl):
    ctx, dims, R, J, dev = xl["ctx"], xl["dims"], xl["R"], xl["J"], xl["dev"]
    idx, val, u = xl["idx"], xl["val"], xl["u"]
    j, modes = 2, [0, 1]
    assert ctx.sts_leaf(1) == (64, 131072) and ctx.sts_leaf(2) == (16, 16384)
    rng = np.random.default_rng(30)
    U, G = gpu_state(ctx)
    gidx, gprob = ctx.sample(j, torch.from_numpy(u))
    gidx, gprob = to_np(gidx).astype(np.int64), to_np(gprob)
    Gh = O.gram_hadamard(G, j)
    Gp = O.pinv_psd(Gh)
    # (1) the first factor's draws, all J of them
    m0 = _masses(U[0], _g_after(Gp, G, modes, 0))
    assert _draw_check(m0, u[:, 0], gidx[:, 0]) <= 8
    del m0
    # (2) four draws of the tree factor given their first row
    W1 = _g_after(Gp, G, modes, 1)
    n_acc = 0
    for s in rng.choice(J, 4, replace=False):
        m1 = _masses(U[1], W1, U[0][gidx[s, 0]])
        n_acc += _draw_check(m1, u[s:s + 1, 1], gidx[s:s + 1, 1])
    assert n_acc <= 1
    # (3) merge: every listed column against the oracle's recount; the
    # sampled columns the GPU leaves out hold no nonzero
    keys, rep, counts, wts = O.dedup(gidx, gprob, dims, j, J)
    uq = ctx.get_unique(J)
    gk = to_np(uq["col_key"]).astype(np.uint64)
    pos = np.searchsorted(keys, gk)
    assert np.all(pos < keys.size) and np.all(keys[np.minimum(pos, keys.size - 1)] == gk)
    np.testing.assert_array_equal(to_np(uq["rep"]), rep[pos])
    np.testing.assert_array_equal(to_np(uq["count"]), counts[pos])
    np.testing.assert_allclose(to_np(uq["weight"]), wts[pos], rtol=1e-14)
    missing = np.setdiff1d(keys, gk)
    if missing.size:
        miss_t = torch.from_numpy(missing.astype(np.int64)).to(dev)
        for c0 in range(0, idx.shape[0], 1 << 27):
            ck = (idx[c0:c0 + (1 << 27), 0].long() +
                  idx[c0:c0 + (1 << 27), 1].long() * dims[0])
            assert not bool(torch.isin(ck, miss_t).any())
    # (4) 1,000 rows of M from the nonzeros the oracle selects in them
    Mg, nz = ctx.sampled_mttkrp(j, want_nnz=True)
    Mg = to_np(Mg).astype(np.float64)
    pick = np.sort(rng.choice(dims[j], 1000, replace=False))
    pick_t = torch.from_numpy(pick.astype(np.int32)).to(dev)
    sel_i, sel_v = [], []
    for c0 in range(0, idx.shape[0], 1 << 27):
        blk = idx[c0:c0 + (1 << 27)]
        mask = torch.isin(blk[:, j], pick_t)
        sel_i.append(blk[mask].cpu().numpy())
        sel_v.append(val[c0:c0 + (1 << 27)][mask].double().cpu().numpy())
    sel_i, sel_v = np.concatenate(sel_i), np.concatenate(sel_v)
    h = np.ones((J, R))
    for q, k in enumerate(modes):
        h = h * U[k][gidx[:, q]]
    ck, rows, vals, slot = O.extract(sel_i, sel_v, dims, j, keys)
    Mo = O.sampled_mttkrp(dims[j], rows, vals, slot, wts, h[rep])
    assert rows.shape[0] > 0
    assert rel_fro(Mg[pick], Mo[pick]) < 1e-4, rel_fro(Mg[pick], Mo[pick])
    # (5) the solved rows, teacher-forced with the GPU's M
    ctx.solve_factor(j)
    Uj = to_np(ctx.get_factor(j))
    sig = to_np(ctx.get_sigma())
    X = Mg[pick] @ Gp
    live = sig > 0
    Xn = np.zeros_like(X)
    Xn[:, live] = X[:, live] / sig[live]
    assert rel_fro(Uj[pick], Xn) < pinv_rtol(1e-5, Gh)
