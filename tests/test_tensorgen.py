"""The seeded input generators (CPU): exact counts, distinct in-range
coordinates and the Zipf marginal law, for the NumPy path and for the
torch path that generates the billion-nonzero workloads on the GPU (run on
the CPU here; it holds none of the method's arithmetic)."""
import numpy as np
import pytest
from scipy import stats

import tensorgen as tg

torch = pytest.importorskip("torch")


def _zipf_pmf(I, s):
    w = np.arange(1, I + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


@pytest.mark.parametrize("dims", [(5000, 4000, 3000), (2000, 500, 300, 40)])
def test_device_generator_counts_and_distinct(dims):
    nnz = 200_000
    idx = tg.zipf_coords_device(3, dims, nnz, 1.1, "cpu").numpy()
    assert idx.shape == (nnz, len(dims)) and idx.dtype == np.int32
    assert np.all(idx >= 0) and np.all(idx < np.array(dims))
    flat = np.ravel_multi_index(idx.T.astype(np.int64), dims)
    assert np.unique(flat).shape[0] == nnz


def test_device_zipf_draws_follow_the_law():
    """Raw device draws, counted by rank through the relabelling, follow the
    Zipf(s) pmf on 1..I (chi-square over the heaviest ranks, tail pooled)."""
    I, s, m = 5000, 1.1, 400_000
    w = torch.arange(1, I + 1, dtype=torch.float64) ** (-s)
    cdf = torch.cumsum(w, 0)
    cdf = cdf / cdf[-1]
    g = torch.Generator(device="cpu")
    g.manual_seed(11)
    perm = torch.randperm(I, generator=g)
    lab = tg.zipf_draws_device(g, cdf, perm, m).numpy()
    counts = np.bincount(lab, minlength=I).astype(float)
    obs = counts[perm.numpy()]  # count of the label holding rank r
    pmf = _zipf_pmf(I, s)
    K = 80
    o = np.r_[obs[:K], obs[K:].sum()]
    e = np.r_[pmf[:K], pmf[K:].sum()] * m
    chi2 = ((o - e) ** 2 / e).sum()
    assert stats.chi2.sf(chi2, K) > 1e-3, chi2
    # a wrong exponent is rejected by the same statistic
    pw = _zipf_pmf(I, 1.2)
    e2 = np.r_[pw[:K], pw[K:].sum()] * m
    assert stats.chi2.sf(((o - e2) ** 2 / e2).sum(), K) < 1e-6


def test_numpy_generator_exact_nnz_and_distinct():
    T = tg.zipf_tensor(5, (3000, 2000, 1000), 100_000)
    flat = np.ravel_multi_index(T.idx.T.astype(np.int64), T.dims)
    assert T.nnz == 100_000 and np.unique(flat).shape[0] == T.nnz
    assert T.val.dtype == np.float32 and np.all(T.val > 0)


def test_slice_scaled_initial_factors():
    """Rows scaled by sqrt(slice nonzero count): empty slices give zero
    rows, and dividing the scale back out leaves the plain Gaussian start
    of the same seed (FP32 values)."""
    dims = (300, 200, 100, 20)
    idx = tg.zipf_coords_device(5, dims, 20_000, 1.2, "cpu")
    U = tg.init_factors_slice_scaled_device(7, dims, 6, idx)
    G = tg.init_factors_device(7, dims, 6, "cpu")
    for k, d in enumerate(dims):
        cnt = np.bincount(idx[:, k].numpy(), minlength=d).astype(np.float64)
        u = U[k].numpy().astype(np.float64)
        assert U[k].dtype == torch.float32 and u.shape == (d, 6)
        assert np.all(u[cnt == 0] == 0)
        nz = cnt > 0
        np.testing.assert_allclose(u[nz] / np.sqrt(cnt[nz])[:, None],
                                   G[k].numpy()[nz], rtol=1e-6)
