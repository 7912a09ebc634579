"""Batched restarts (cp_batch_*) against single decompositions and the oracle.

A batch runs B independent decompositions of one tensor (Alg. 1 as
independent trials) with uneven ranks: one shared index, restarts spread
over several streams, and each sweep one replay of a captured HIP graph.
Each restart must follow the same path as a single context given the same
inputs and uniforms, replay after replay (eager work and synchronisation in
between), and, for one restart per rank class, the FP64 oracle's ALS.
"""
import numpy as np
import pytest

import oracle as O
import tensorgen as tg
from tests.helpers import rel_fro, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import load_library
    load_library()
    return torch.device("cuda:0")


def _inputs(T, ranks, J, sweeps, seed, fp32=False):
    rng = np.random.default_rng(seed)
    U0 = []
    for R in ranks:
        u = [rng.standard_normal((d, R)) for d in T.dims]
        if fp32:
            u = [x.astype(np.float32).astype(np.float64) for x in u]
        U0.append(u)
    uni = rng.random((sweeps, len(ranks), T.N, J, T.N - 1))
    return U0, uni


def _run_pair(dev, T, ranks, sampler, prec, J, sweeps, tol, nstreams,
              leaf=0, seed=5):
    from paper_2210_05105_amd import Batch, Context
    vdt = np.float64 if prec == "fp64" else np.float32
    idx = torch.from_numpy(np.ascontiguousarray(T.idx)).to(dev)
    val = torch.from_numpy(T.val.astype(vdt)).to(dev)
    U0, uni = _inputs(T, ranks, J, sweeps, seed, fp32=(prec != "fp64"))
    bt = Batch(idx, val, T.dims, ranks, sampler, prec, J=J, sts_leaf=leaf,
               nstreams=nstreams)
    assert len({bt.stream_of(b) for b in range(len(ranks))}) == \
        min(nstreams, len(ranks))
    singles = []
    for b, R in enumerate(ranks):
        bt_U = [torch.from_numpy(u) for u in U0[b]]
        for k in range(T.N):
            bt.set_factor(b, k, bt_U[k])
        c = Context(idx, val, T.dims, R, sampler, prec, max_J=J,
                    sts_leaf=leaf)
        for k in range(T.N):
            c.set_factor(k, bt_U[k])
        singles.append(c)
    ubuf = torch.empty((len(ranks), T.N, J, T.N - 1), dtype=torch.float64,
                       device=dev)
    for t in range(sweeps):
        ubuf.copy_(torch.from_numpy(uni[t]))      # same buffer every sweep
        bt.sweep(ubuf)                            # graph replay
        bt.sync()
        for b, c in enumerate(singles):           # eager reference sweeps
            c.sweep(1, J, torch.from_numpy(uni[t, b][None]))
            c.sync()
            for k in range(T.N):
                e = rel_fro(to_np(bt.get_factor(b, k)), to_np(c.get_factor(k)))
                assert e < tol, (t, b, k, e)
    fits = bt.fit()
    for b, c in enumerate(singles):
        assert abs(fits[b] - c.fit()) < max(tol, 1e-12) * 10
        c.close()
    bt.close()
    return U0, uni, fits


@pytest.mark.parametrize("sampler,leaf", [("arls", 0), ("sts", 16)])
def test_batch_matches_single_contexts_fp64(dev, sampler, leaf):
    T = tg.make_tensor("planted")
    ranks = [8, 3, 16, 5, 8, 1, 40]
    _run_pair(dev, T, ranks, sampler, "fp64", 2048, 3, 1e-10, 3, leaf)


def test_batch_uneven_ranks_mixed_precision(dev):
    """Ranks of the batched configuration ({8, 16, 32, 64, 128}) on a small
    power-law tensor in the mixed form; several restarts per stream.

    In FP32 the sampled MTTKRP's order of accumulation within a row is not
    fixed (records reach their bucket through atomics), so two runs differ
    in the last bits of M, and the ill-conditioned sampled systems of the
    high ranks magnify that.  Compared are: the first mode solve of the
    first sweep, where both sides draw exactly the same samples (same
    initial factors and uniforms), to the FP32 bar (1e-4); after several
    sweeps, where later draws may cross a CDF boundary differently and the
    trajectories of the high ranks diverge, each restart's fit against the
    oracle's fit of that restart's own factors (1e-4: the model norm uses
    the split-BF16 Grams).  The trajectories themselves are compared in FP64
    above."""
    from paper_2210_05105_amd import Batch, Context
    T = tg.zipf_tensor(90, (3000, 2000, 1000), 150_000, s=1.1)
    ranks = [128, 8, 32, 16, 64, 8, 32, 128, 16, 64]
    J, sweeps = 16384, 4
    idx = torch.from_numpy(np.ascontiguousarray(T.idx)).to(dev)
    val = torch.from_numpy(T.val.astype(np.float32)).to(dev)
    U0, uni = _inputs(T, ranks, J, sweeps, 5, fp32=True)
    bt = Batch(idx, val, T.dims, ranks, "arls", "mixed", J=J, nstreams=4)
    assert len({bt.stream_of(b) for b in range(len(ranks))}) == 4
    singles = []
    for b, R in enumerate(ranks):
        c = Context(idx, val, T.dims, R, "arls", "mixed", max_J=J)
        for k in range(T.N):
            u = torch.from_numpy(U0[b][k])
            bt.set_factor(b, k, u)
            c.set_factor(k, u)
        singles.append(c)
    ubuf = torch.empty((len(ranks), T.N, J, T.N - 1), dtype=torch.float64,
                       device=dev)
    # first mode solve of the first sweep, both sides: mode 0 of the
    # single contexts against the batch's mode 0 after its first sweep
    firsts = []
    for b, c in enumerate(singles):
        c.sample(0, torch.from_numpy(uni[0, b, 0]), outputs=False)
        c.sampled_mttkrp(0, want_M=False)
        c.solve_factor(0)
        c.sync()
        firsts.append(to_np(c.get_factor(0)))
    for c in singles:
        c.close()
    for t in range(sweeps):
        ubuf.copy_(torch.from_numpy(uni[t]))      # same buffer every sweep
        bt.sweep(ubuf)                            # graph replay
        bt.sync()
        if t == 0:
            for b in range(len(ranks)):
                e = rel_fro(to_np(bt.get_factor(b, 0)), firsts[b])
                assert e < 1e-4, (b, ranks[b], e)
    # later sweeps: each restart's fit is the fit of its own factors
    fits = bt.fit()
    for b in range(len(ranks)):
        U = [to_np(bt.get_factor(b, k)) for k in range(T.N)]
        f = O.fit(T.idx, T.val.astype(np.float32).astype(np.float64),
                  to_np(bt.get_sigma(b)), U)
        assert np.isfinite(fits[b]) and abs(fits[b] - f) < 1e-4, \
            (b, ranks[b], fits[b], f)
    bt.close()


def test_batch_restarts_track_the_oracle(dev):
    """One restart per rank class against the oracle's ALS (FP64, same
    initial factors and uniforms, CP-ARLS-LEV): every draw identical, so
    the factors agree to rounding after two sweeps."""
    from paper_2210_05105_amd import Batch
    T = tg.make_tensor("planted")
    ranks, J, sweeps = [2, 5, 8, 13], 2048, 2
    idx = torch.from_numpy(np.ascontiguousarray(T.idx)).to(dev)
    val = torch.from_numpy(T.val).to(dev)
    U0, uni = _inputs(T, ranks, J, sweeps, 7)
    bt = Batch(idx, val, T.dims, ranks, "arls", "fp64", J=J, nstreams=2)
    for b in range(len(ranks)):
        for k in range(3):
            bt.set_factor(b, k, torch.from_numpy(U0[b][k]))
    ubuf = torch.empty((len(ranks), 3, J, 2), dtype=torch.float64, device=dev)
    for t in range(sweeps):
        ubuf.copy_(torch.from_numpy(uni[t]))
        bt.sweep(ubuf)
    bt.sync()
    fits = bt.fit()
    for b, R in enumerate(ranks):
        Uo, so, _ = O.als(T.idx, T.val, T.dims, R, "arls", U0[b],
                          uniforms=uni[:, b], sweeps=sweeps, J=J)
        for k in range(3):
            e = rel_fro(to_np(bt.get_factor(b, k)), Uo[k])
            assert e < 1e-8, (R, k, e)
        np.testing.assert_allclose(to_np(bt.get_sigma(b)), so, rtol=1e-8)
        assert abs(fits[b] - O.fit(T.idx, T.val, so, Uo)) < 1e-9
    bt.close()


def test_batch_rejects_bad_arguments(dev):
    from paper_2210_05105_amd import Batch, CprError
    T = tg.make_tensor("planted")
    idx = torch.from_numpy(np.ascontiguousarray(T.idx)).to(dev)
    val = torch.from_numpy(T.val).to(dev)
    for ranks in ([0, 4], [129], []):
        with pytest.raises(CprError):
            Batch(idx, val, T.dims, ranks, "arls", "fp64", J=16)
    bt = Batch(idx, val, T.dims, [4, 2], "arls", "fp64", J=16)
    with pytest.raises(CprError) as e:  # factors not set
        bt.sweep(torch.zeros((2, 3, 16, 2), dtype=torch.float64, device=dev))
    assert e.value.name == "CP_ESTATE"
    bt.close()
