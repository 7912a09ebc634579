"""The sketched-Gram update (Fig. 3) on the GPU against the FP64 oracle.

With CP_GRAM_SKETCHED the update is U_j = M G~^+ with
G~ = (S U_{!=j})^T (S U_{!=j}) = sum_s h_s h_s^T / (J p_s) over the solve's
draws (the draws themselves still follow the exact leverage laws).
"""
import numpy as np
import pytest

import oracle as O
import tensorgen as tg
from tests.gpu_common import init_ctx
from tests.helpers import gpu_state, oracle_sampled_M, pinv_rtol, rel_fro, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import load_library
    load_library()
    return torch.device("cuda:0")


def _ctx(dev, T, R, sampler, prec, J):
    from paper_2210_05105_amd import Context
    vdt = np.float64 if prec == "fp64" else np.float32
    return Context(torch.from_numpy(np.ascontiguousarray(T.idx)).to(dev),
                   torch.from_numpy(T.val.astype(vdt)).to(dev), T.dims, R,
                   sampler, prec, max_J=J, sketched=True)


@pytest.mark.parametrize("sampler,prec,R,tol", [("arls", "fp64", 8, 1e-10),
                                                ("sts", "fp64", 12, 1e-10),
                                                ("sts", "fp32", 40, 1e-4)])
def test_sketched_solve_teacher_forced(dev, sampler, prec, R, tol):
    T, _ = tg.tiny_tensor(91, (300, 250, 190), 30000, rank=4, noise_var=0.01)
    J = 3000
    ctx = _ctx(dev, T, R, sampler, prec, J)
    _, runi = init_ctx(ctx, T.dims, R, 92, fp32=(prec != "fp64"))
    for j in range(3):
        U, G = gpu_state(ctx)
        u = tg.uniform_block(runi, J, 3)
        gidx, gprob = ctx.sample(j, torch.from_numpy(u))
        gidx, gprob = to_np(gidx).astype(np.int64), to_np(gprob)
        M, _ = ctx.sampled_mttkrp(j)
        M = to_np(M).astype(np.float64)
        ref = oracle_sampled_M(T, T.dims, j, gidx, gprob, U, J)
        assert rel_fro(M, ref["M"]) < tol
        ctx.solve_factor(j)
        Gs = O.sketched_gram(ref["h"], gprob, J)
        Uo, so = O.solve(M, O.pinv_psd(Gs))
        stol = pinv_rtol(tol, Gs)
        assert rel_fro(to_np(ctx.get_factor(j)), Uo) < stol
        np.testing.assert_allclose(to_np(ctx.get_sigma()), so, rtol=stol)
    ctx.close()


def test_sketched_als_end_to_end_fp64(dev):
    """Three sweeps of sketched CP-ARLS-LEV ALS, identical init and
    uniforms: every draw identical to the oracle's, factors and fit equal
    to rounding."""
    T = tg.make_tensor("planted")
    R, J, sweeps = 8, 4096, 3
    _, _, rinit, runi = tg.streams([93, 1])
    U0 = tg.init_factors(rinit, T.dims, R)
    uni = tg.uniform_blocks(runi, sweeps, J, 3)
    ctx = _ctx(dev, T, R, "arls", "fp64", J)
    for k in range(3):
        ctx.set_factor(k, torch.from_numpy(U0[k]))
    ctx.sweep(sweeps, J, torch.from_numpy(uni))
    Uo, so, _ = O.als(T.idx, T.val, T.dims, R, "arls", U0, uni,
                      sweeps=sweeps, J=J, sketched=True)
    Ug, _ = gpu_state(ctx)
    for k in range(3):
        assert rel_fro(Ug[k], Uo[k]) < 1e-8, k
    assert abs(ctx.fit() - O.fit(T.idx, T.val, so, Uo)) < 1e-9
    ctx.close()
