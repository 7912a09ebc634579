"""Edge cases of the method on the GPU, against the FP64 oracle.

- rows and whole leaf subtrees of zero mass are never drawn (inverse-CDF
  rule min{i : u Z < F(i)} of Appendix A and B);
- the end points u = 0 and u = 1 - 2^-53 of the uniform domain;
- data errors found on the device: bad uniforms and zero mass for STS-CP,
  non-finite factors and tensor values, bad teacher-forced draws;
- teacher forcing through cp_set_samples with the oracle's own draws;
- CP-ARLS-LEV with a drawn factor of 1.2M rows (many tiles of the FP64
  CDF scan and grid-stride rounds of the leverage pass).
"""
import numpy as np
import pytest

import oracle as O
import tensorgen as tg
from tests.gpu_common import (check_after_draws, check_mode_solve, init_ctx,
                              make_ctx)
from tests.helpers import gpu_state, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U_TOP = float(np.nextafter(1.0, 0.0))  # 1 - 2^-53


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import load_library
    load_library()
    return torch.device("cuda:0")


def _zeroed_factors(dims, R, seed, zero_rows):
    rng = np.random.default_rng(seed)
    U0 = [rng.standard_normal((d, R)) for d in dims]
    for k, rows in zero_rows.items():
        U0[k][rows] = 0.0
    return U0


def _edge_uniforms(rng, J, N):
    u = tg.uniform_block(rng, J, N)
    u[:8] = 0.0
    u[8:16] = U_TOP
    u[16:24, 0] = 0.0
    u[16:24, 1:] = U_TOP
    u[24:32, 0] = U_TOP
    u[24:32, 1:] = 0.0
    return u


@pytest.mark.parametrize("sampler,R,leaf", [("arls", 8, 0), ("sts", 8, 16),
                                            ("sts", 32, 16), ("sts", 20, 32)])
def test_zero_mass_rows_and_uniform_end_points(dev, sampler, R, leaf):
    dims, J = (300, 260, 200), 2048
    T, _ = tg.tiny_tensor(60, dims, 30000, rank=3, noise_var=0.01)
    # zero rows at both ends and a run covering whole leaves (rows 96..175
    # hold leaves 6..10 of 16 rows): zero-mass leaves and subtrees
    zr = {1: np.r_[0:5, 96:176, 259], 2: np.r_[0:3, 64:128, 199]}
    U0 = _zeroed_factors(dims, R, 61, zr)
    ctx = make_ctx(dev, T, R, sampler, "fp64", J, leaf)
    for k in range(3):
        ctx.set_factor(k, torch.from_numpy(U0[k]))
    rng = np.random.default_rng(62)
    acc = 0
    for j in (0, 1, 2):
        u = _edge_uniforms(rng, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, sampler, 1e-10)
    assert acc <= 2
    # the draws never land on a zero row of a factor that still has them
    u = _edge_uniforms(rng, J, 3)
    U, _ = gpu_state(ctx)
    gidx, _ = ctx.sample(0, torch.from_numpy(u))
    gidx = to_np(gidx)
    for q, k in enumerate((1, 2)):
        zero = np.all(U[k] == 0.0, axis=1)
        assert not np.any(zero[gidx[:, q]]), (k, np.nonzero(zero[gidx[:, q]]))
    ctx.close()


@pytest.mark.parametrize("bad", [1.0, -0.25, float("nan"), 1.5])
def test_sts_bad_uniform_is_reported(dev, bad):
    from paper_2210_05105_amd import CprError
    dims = (40, 30, 20)
    T, _ = tg.tiny_tensor(63, dims, 2000)
    ctx = make_ctx(dev, T, 4, "sts", "fp64", 64)
    init_ctx(ctx, dims, 4, 64)
    for col in (0, 1):  # first (flat) factor, then the tree factor
        u = np.full((64, 2), 0.5)
        u[10, col] = bad
        ctx.sample(0, torch.from_numpy(u))
        with pytest.raises(CprError) as e:
            ctx.sync()
        assert e.value.name == "CP_EINVAL"
    # the context stays usable after the error is read
    ctx.sample(0, torch.from_numpy(np.full((64, 2), 0.5)))
    ctx.sync()
    ctx.close()


def test_sts_zero_factor_is_degenerate(dev):
    from paper_2210_05105_amd import CprError
    dims = (40, 30, 20)
    T, _ = tg.tiny_tensor(64, dims, 2000)
    ctx = make_ctx(dev, T, 4, "sts", "fp64", 64)
    init_ctx(ctx, dims, 4, 65)
    ctx.set_factor(2, torch.zeros(dims[2], 4, dtype=torch.float64))
    ctx.sync()  # an all-zero factor is valid input (sigma = 0 columns)
    ctx.sample(0, torch.from_numpy(np.full((64, 2), 0.5)))
    with pytest.raises(CprError) as e:
        ctx.sync()
    assert e.value.name == "CP_EDEGENERATE"
    ctx.close()


@pytest.mark.parametrize("sampler", ["arls", "sts"])
def test_nonfinite_factor_is_reported(dev, sampler):
    from paper_2210_05105_amd import CprError
    dims = (40, 30, 20)
    T, _ = tg.tiny_tensor(66, dims, 2000)
    ctx = make_ctx(dev, T, 4, sampler, "fp64", 64)
    init_ctx(ctx, dims, 4, 67)
    U = np.random.default_rng(68).standard_normal((dims[1], 4))
    U[7, 2] = np.nan
    ctx.set_factor(1, torch.from_numpy(U))
    with pytest.raises(CprError) as e:
        ctx.sync()
    assert e.value.name == "CP_ENUMERIC"
    U[7, 2] = np.inf
    ctx.set_factor(1, torch.from_numpy(U))
    with pytest.raises(CprError) as e:
        ctx.sync()
    assert e.value.name == "CP_ENUMERIC"
    ctx.close()


def test_nonfinite_tensor_value_is_rejected(dev):
    from paper_2210_05105_amd import CprError
    dims = (20, 10, 8)
    T, _ = tg.tiny_tensor(69, dims, 300)
    bad = tg.SparseTensor(dims, T.idx.copy(), T.val.copy())
    bad.val[11] = np.nan
    with pytest.raises(CprError) as e:
        make_ctx(dev, bad, 4, "arls", "fp64", 16)
    assert e.value.name == "CP_EINVAL"


@pytest.mark.parametrize("sampler,prec,tol", [("arls", "fp64", 1e-10),
                                              ("sts", "fp64", 1e-10),
                                              ("arls", "fp32", 1e-4)])
def test_set_samples_teacher_forcing(dev, sampler, prec, tol):
    """The oracle draws from its own sampler on the GPU's state; the draws
    go in through cp_set_samples; merge, extraction, M and the solve are
    compared with the oracle on those draws."""
    dims, R, J = (300, 250, 190), 12, 3000
    T, _ = tg.tiny_tensor(70, dims, 30000, rank=4, noise_var=0.01)
    ctx = make_ctx(dev, T, R, sampler, prec, J)
    _, runi = init_ctx(ctx, dims, R, 71, fp32=(prec != "fp64"))
    for j in (0, 2, 1):
        U, G = gpu_state(ctx)
        u = tg.uniform_block(runi, J, 3)
        if sampler == "arls":
            st = {k: O.arls_build(U[k], G[k]) for k in range(3) if k != j}
            oidx, oprob, _ = O.arls_sample(U, st, j, u)
        else:
            oidx, oprob, _ = O.sts_sample(U, G, j, u, block=32)
        ctx.set_samples(j, torch.from_numpy(oidx.astype(np.int32)),
                        torch.from_numpy(oprob))
        check_after_draws(ctx, T, j, oidx, oprob, U, G, J, tol)
    ctx.close()


def test_set_samples_rejects_bad_draws(dev):
    from paper_2210_05105_amd import CprError
    dims, J = (40, 30, 20), 32
    T, _ = tg.tiny_tensor(72, dims, 2000)
    ctx = make_ctx(dev, T, 4, "arls", "fp64", J)
    init_ctx(ctx, dims, 4, 73)
    idx = np.zeros((J, 2), dtype=np.int32)
    for p_bad in (0.0, -1e-3, np.nan, np.inf):
        p = np.full(J, 0.01)
        p[5] = p_bad
        ctx.set_samples(0, torch.from_numpy(idx), torch.from_numpy(p))
        with pytest.raises(CprError) as e:
            ctx.sync()
        assert e.value.name == "CP_EINVAL", p_bad
    bad = idx.copy()
    bad[3, 1] = dims[2]  # out of range
    ctx.set_samples(0, torch.from_numpy(bad), torch.from_numpy(np.full(J, .01)))
    with pytest.raises(CprError) as e:
        ctx.sync()
    assert e.value.name == "CP_EINVAL"
    ctx.close()


def test_arls_long_drawn_factor(dev):
    """A drawn factor of 1.2M rows: the FP64 CDF is scanned over ~300 tiles
    and the leverage pass takes many grid-stride rounds; draws are compared
    bit-exactly outside the 1e-12 band, as is the whole mode solve."""
    dims, R, J = (1_200_000, 50, 40), 16, 16384
    T, _ = tg.tiny_tensor(74, dims, 150_000, rank=3, noise_var=0.01)
    ctx = make_ctx(dev, T, R, "arls", "fp64", J)
    _, runi = init_ctx(ctx, dims, R, 75)
    acc = 0
    for j in (1, 2, 0, 1):
        u = tg.uniform_block(runi, J, 3)
        acc += check_mode_solve(ctx, T, j, u, J, "arls", 1e-10)
    assert acc <= 2
    ctx.close()
