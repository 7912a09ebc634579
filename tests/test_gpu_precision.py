"""Reduced-precision forms against the FP64 oracle.

CP_FP32 forms the factor Grams (Eq. 5) on FP32 MFMA, CP_MIXED on BF16 MFMA
(each FP32 value split into a high and a low BF16 part, three products,
FP32 accumulation); both keep FP32 factors and MTTKRP and an FP64
pseudo-inverse, sampler and refined solve.  Checked here:
- each Gram against U^T U of the stored factor in FP64;
- teacher-forced mode solves (the oracle receives the GPU's Grams, so the
  draws stay bit-exact outside the 1e-12 band);
- the error of every result of one mode solve (G_k, G^+, M, U_j, fit)
  against an FP64 recomputation from the same stored factors, reported;
- ALS sweeps in FP64 and in the mixed form from identical inputs end at
  the same fit within 1e-3.
"""
import numpy as np
import pytest

import oracle as O
import tensorgen as tg
from tests.gpu_common import check_mode_solve, init_ctx, make_ctx
from tests.helpers import cond_psd, gpu_state, rel_fro, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# bound on |G_gpu - U^T U| entrywise for unit-norm columns (|G_ab| <= 1):
# FP32 products and sums flushed to FP64 every <= 256 rows; split BF16
# drops lo_a lo_b (<= 2^-16 relative) and rounds lo to BF16 (2^-17)
GRAM_ATOL = {"fp32": 2e-6, "mixed": 4e-5}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import load_library
    load_library()
    return torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
@pytest.mark.parametrize("R", [1, 8, 17, 32, 48, 100, 128])
def test_gram_reduced_precision(dev, prec, R):
    dims = (20_000, 77, 33)
    T, _ = tg.tiny_tensor(80, dims, 3000)
    ctx = make_ctx(dev, T, R, "arls", prec, 16)
    init_ctx(ctx, dims, R, 81, fp32=True)
    for k in range(3):
        U = to_np(ctx.get_factor(k))  # the stored FP32 factor, exactly
        G = to_np(ctx.get_gram(k))
        ref = O.gram(U)
        err = np.abs(G - ref).max()
        assert err < GRAM_ATOL[prec], (k, err)
        np.testing.assert_array_equal(G, G.T)
    ctx.close()


@pytest.mark.parametrize("sampler,R,leaf", [("arls", 24, 0), ("sts", 32, 16),
                                            ("sts", 100, 32)])
def test_mixed_mode_solves_teacher_forced(dev, sampler, R, leaf):
    if sampler == "arls":
        T = tg.zipf_tensor(82, (2000, 1000, 400, 20), 150_000, s=1.2)
    else:
        T = tg.zipf_tensor(83, (3000, 2400, 1800), 200_000, s=1.1)
    J = 3000
    ctx = make_ctx(dev, T, R, sampler, "mixed", J, leaf)
    _, runi = init_ctx(ctx, T.dims, R, 84, fp32=True)
    acc = 0
    for j in range(T.N):
        u = tg.uniform_block(runi, J, T.N)
        acc += check_mode_solve(ctx, T, j, u, J, sampler, 1e-4)
    assert acc <= 2
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
@pytest.mark.parametrize("R", [6, 16, 25, 75])
def test_fp32_row_solve_any_rank(dev, prec, R):
    """The FP32 row solve at ranks that leave 2, 0, 1 and 1 all-zero k-steps
    of the padded product, with row lengths that are not a multiple of 4
    (element-wise output) or are (16-byte output), on modes whose row counts
    leave a partial last 16-row tile: U_j, sigma and G_j against the oracle,
    teacher-forced."""
    T = tg.zipf_tensor(87, (2001, 1503, 405), 60_000, s=1.1)
    J = 1024
    ctx = make_ctx(dev, T, R, "arls", prec, J)
    _, runi = init_ctx(ctx, T.dims, R, 88, fp32=True)
    for j in range(T.N):
        u = tg.uniform_block(runi, J, T.N)
        check_mode_solve(ctx, T, j, u, J, "arls", 1e-4)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_error_of_each_result_against_fp64(dev, prec):
    """One ARLS mode solve in reduced precision: G_k, G^+, M, U_j and the fit
    against an FP64 recomputation from the same stored factors and draws
    (the draws themselves are the GPU's: a Gram change moves CDF boundaries,
    a sampling effect reported elsewhere)."""
    T = tg.zipf_tensor(85, (3000, 2000, 1500), 200_000, s=1.1)
    R, J, j = 32, 8192, 1
    ctx = make_ctx(dev, T, R, "arls", prec, J)
    _, runi = init_ctx(ctx, T.dims, R, 86, fp32=True)
    U, G = gpu_state(ctx)
    Gx = [O.gram(u) for u in U]                  # FP64 Grams of the factors
    u = tg.uniform_block(runi, J, 3)
    gidx, gprob = ctx.sample(j, torch.from_numpy(u))
    gidx, gprob = to_np(gidx).astype(np.int64), to_np(gprob)
    M, _ = ctx.sampled_mttkrp(j)
    M = to_np(M).astype(np.float64)
    ctx.solve_factor(j)
    Uj = to_np(ctx.get_factor(j))
    Ghx = O.gram_hadamard(Gx, j)
    Gpx = O.pinv_psd(Ghx)
    Gpg = O.pinv_psd(O.gram_hadamard(G, j))
    from tests.helpers import oracle_sampled_M
    Mx = oracle_sampled_M(T, T.dims, j, gidx, gprob, U, J)["M"]
    Ux, sx = O.solve(Mx, Gpx)
    fx_U = [Ux if k == j else U[k] for k in range(3)]
    fit_g = ctx.fit()
    fit_x = O.fit(T.idx, T.val.astype(np.float64), sx, fx_U)
    errs = {
        "G_k": max(np.abs(G[k] - Gx[k]).max() for k in range(3) if k != j),
        "G+": rel_fro(Gpg, Gpx),
        "M": rel_fro(M, Mx),
        "U_j": rel_fro(Uj, Ux),
        "fit": abs(fit_g - fit_x),
    }
    kappa = cond_psd(Ghx)
    print(f"\n[{prec}] error vs FP64 (cond(G) = {kappa:.1f}): " +
          ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert errs["G_k"] < GRAM_ATOL[prec]
    assert errs["G+"] < 10 * kappa * GRAM_ATOL[prec]
    assert errs["M"] < 1e-5
    assert errs["U_j"] < 1e-5 + 10 * kappa * GRAM_ATOL[prec]
    assert errs["fit"] < 1e-3
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_solve_refinement_below_fp32_rounding(dev, prec):
    """The row solve of the FP32 forms: with refinement (refine=True: FP64
    MFMA, X = M G^+ + (M - M G^+ G) G^+) and without (the default: one
    product on FP32 MFMA, G^+ rounded to FP32), from the same stored factors
    and draws, so the same M up to the FP32 MTTKRP's order of accumulation.
    Both are within the FP32 bar of the FP64 solve of the oracle's M: M's
    own FP32 rounding, amplified by the condition of G, is of the same order
    as what the FP32 product adds."""
    T = tg.zipf_tensor(85, (3000, 2000, 1500), 200_000, s=1.1)
    R, J, j = 32, 8192, 1
    errs = {}
    for refine in (True, False):
        ctx = make_ctx(dev, T, R, "arls", prec, J, refine=refine)
        _, runi = init_ctx(ctx, T.dims, R, 86, fp32=True)
        U, _ = gpu_state(ctx)
        u = tg.uniform_block(runi, J, 3)
        gidx, gprob = ctx.sample(j, torch.from_numpy(u))
        gidx, gprob = to_np(gidx).astype(np.int64), to_np(gprob)
        ctx.sampled_mttkrp(j, want_M=False)
        ctx.solve_factor(j)
        Uj = to_np(ctx.get_factor(j))
        ctx.close()
        from tests.helpers import oracle_sampled_M
        Mx = oracle_sampled_M(T, T.dims, j, gidx, gprob, U, J)["M"]
        Ghx = O.gram_hadamard([O.gram(x) for x in U], j)
        Ux, _ = O.solve(Mx, O.pinv_psd(Ghx))
        errs[refine] = rel_fro(Uj, Ux)
        kappa = cond_psd(Ghx)
    print(f"\n[{prec}] U_j error vs FP64 (cond(G) = {kappa:.1f}): refined "
          f"{errs[True]:.2e}, unrefined {errs[False]:.2e}")
    for e in errs.values():
        assert e < 1e-5 + 10 * kappa * GRAM_ATOL[prec]


@pytest.mark.parametrize("sampler", ["arls", "sts"])
def test_mixed_and_fp64_reach_equal_fit(dev, sampler):
    """Identical inputs (FP32-representable tensor values and initial
    factors); 40 sweeps (converged) of each form on a fully observed (every
    entry stored) planted rank-5 tensor with noise, so that a rank-5 model
    fits it well.  Both forms solve with the same sample sets: the FP64
    context draws, and the mixed one takes its draws and probabilities by
    cp_set_samples, so the fits differ by precision alone (free-running
    forms draw differently once their factors differ in the last bits, and
    their fits then differ by the method's sampling noise).  The two fits
    agree within 1e-3."""
    dims = (60, 50, 40)
    T, _ = tg.tiny_tensor(87, dims, int(np.prod(dims)), rank=5,
                          noise_var=0.01, dtype=np.float32)
    R, J, sweeps = 5, 32768, 40
    _, _, rinit, runi = tg.streams([97, 88])
    U0 = tg.init_factors(rinit, T.dims, R, dtype=np.float32)
    uni = torch.from_numpy(tg.uniform_blocks(runi, sweeps, J, 3))
    ctx = {p: make_ctx(dev, T, R, sampler, p, J) for p in ("fp64", "mixed")}
    for c in ctx.values():
        for k in range(3):
            c.set_factor(k, torch.from_numpy(U0[k]))
    for t in range(sweeps):
        for j in range(3):
            idx, prob = ctx["fp64"].sample(j, uni[t, j])
            ctx["mixed"].set_samples(j, idx, prob)
            for c in ctx.values():
                c.sampled_mttkrp(j, want_M=False)
                c.solve_factor(j)
    fits = {p: c.fit() for p, c in ctx.items()}
    for c in ctx.values():
        c.close()
    print(f"\n[{sampler}] fit after {sweeps} sweeps: fp64 {fits['fp64']:.6f}, "
          f"mixed {fits['mixed']:.6f}")
    assert fits["fp64"] > 0.9
    assert abs(fits["fp64"] - fits["mixed"]) < 1e-3, fits
