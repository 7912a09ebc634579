"""Pins for the FP64 oracle (CPU only).

Each test checks the oracle against something other than itself: a
hand-derived worked example (tests/golden), a closed form, a textbook
identity, a library routine, an explicitly formed Khatri-Rao product, or a
statistical law.  Together they are meant to catch a dropped term, a wrong
sign or index, or a transposed operand anywhere in the oracle.
"""
import json
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O
import tensorgen as tg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def rand_factors(seed, dims, R, scale=None):
    rng = np.random.default_rng(seed)
    U = [rng.standard_normal((d, R)) for d in dims]
    if scale is not None:
        U = [u * scale for u in U]
    return U


# ---------------------------------------------------------------- golden

def test_golden_leverage():
    g = gold("leverage_3x2.json")
    A = np.array(g["A"], dtype=float)
    l = O.leverage_scores(A)
    np.testing.assert_allclose(l, g["leverage"], rtol=0, atol=1e-15)
    assert abs(l.sum() - g["sum"]) < 1e-14
    lev, cdf, Z = O.arls_build(A, O.gram(A))
    np.testing.assert_allclose(lev, g["leverage"], atol=1e-15)
    assert abs(float(Z) - g["sum"]) < 1e-14


def test_golden_krp_order_and_column_keys():
    g = gold("krp_order.json")
    U = [np.array(u, dtype=float) for u in g["U"]]
    A = O.design_matrix(U, g["j"])
    np.testing.assert_array_equal(A, np.array(g["design"], dtype=float))
    dims = [u.shape[0] for u in U]
    t = np.array(g["tuples_i2_i3"])
    idx = np.zeros((4, 3), dtype=np.int64)
    idx[:, 1:] = t
    np.testing.assert_array_equal(O.column_key(idx, dims, 0), g["column_keys"])
    np.testing.assert_array_equal(O.sample_column_key(t, dims, 0),
                                  g["column_keys"])


def _worked_factors(g):
    U1 = np.ones((3, 2))  # mode being solved; not used by the samplers
    return [U1, np.array(g["U2"], float), np.array(g["U3"], float)]


def test_golden_sampler_laws_and_draws():
    g = gold("samplers_worked.json")
    U = _worked_factors(g)
    np.testing.assert_allclose(O.sts_law_bruteforce(U, 0), g["exact_law"],
                               atol=1e-15)
    G = [O.gram(u) for u in U]
    for case in g["sts_cases"]:
        u = np.array([case["u"]])
        idx, prob, h = O.sts_sample(U, G, 0, u, block=1)
        assert list(idx[0]) == case["idx"]
        assert abs(prob[0] - case["prob"]) < 1e-15
        assert list(O.sts_sample_bruteforce(U, 0, u)[0]) == case["idx"]
    states = {k: O.arls_build(U[k], G[k]) for k in range(3)}
    for case in g["arls_cases"]:
        idx, prob, h = O.arls_sample(U, states, 0, np.array([case["u"]]))
        assert list(idx[0]) == case["idx"]
        assert abs(prob[0] - case["prob"]) < 1e-15


def test_golden_fit_rank1():
    g = gold("fit_rank1.json")
    a, b, c = (np.array(g[k], float) for k in "abc")
    T = np.einsum("i,j,k->ijk", a, b, c)
    idx = np.array(np.nonzero(T != 0)).T
    val = T[T != 0]
    U = [a[:, None] / np.linalg.norm(a), b[:, None] / np.linalg.norm(b),
         c[:, None] / np.linalg.norm(c)]
    s0 = np.linalg.norm(a) * np.linalg.norm(b) * np.linalg.norm(c)
    for scale, expect in g["sigma_scale_to_fit"]:
        f = O.fit(idx, val, np.array([scale * s0]), U)
        assert abs(f - expect) < 1e-12


def test_golden_als_rank1_step():
    g = gold("als_rank1_step.json")
    a, b, c = (np.array(g[k], float) for k in "abc")
    T = np.einsum("i,j,k->ijk", a, b, c)
    idx = np.array(np.nonzero(T != 0)).T
    val = T[T != 0]
    U = [np.ones((3, 1)), np.array(g["U2"], float)[:, None],
         np.array(g["U3"], float)[:, None]]
    G = [O.gram(u) for u in U]
    M = O.mttkrp_exact(idx, val, U, 0)
    U1, sigma = O.solve(M, O.pinv_psd(O.gram_hadamard(G, 0)))
    np.testing.assert_allclose(U1[:, 0], g["U1_expected"], atol=1e-15)
    assert abs(sigma[0] - g["sigma_expected"]) < 1e-13


# ---------------------------------------------------------- identities

@pytest.mark.parametrize("dims,j", [((6, 5, 4), 0), ((6, 5, 4), 1),
                                    ((5, 4, 3, 3), 2), ((5, 4, 3, 3), 3)])
def test_gram_hadamard_identity(dims, j):
    """P5: (U_{!=j})^T U_{!=j} = Hadamard of U_k^T U_k (Eq. 5)."""
    U = rand_factors(1, dims, 3)
    A = O.design_matrix(U, j)
    G = [O.gram(u) for u in U]
    np.testing.assert_allclose(A.T @ A, O.gram_hadamard(G, j), rtol=1e-13,
                               atol=1e-13)
    assert A.shape[0] == np.prod([d for k, d in enumerate(dims) if k != j])


def test_pinv_matches_library_and_penrose():
    rng = np.random.default_rng(3)
    for rank in (5, 3):  # full rank, and duplicated / dependent columns
        B = rng.standard_normal((40, rank))
        A = B @ rng.standard_normal((rank, 5))
        G = A.T @ A
        P = O.pinv_psd(G)
        np.testing.assert_allclose(P, np.linalg.pinv(G, rcond=1e-12,
                                                     hermitian=True),
                                   rtol=1e-8, atol=1e-10)
        # Moore-Penrose conditions
        np.testing.assert_allclose(G @ P @ G, G, atol=1e-9 * np.abs(G).max())
        np.testing.assert_allclose(P @ G @ P, P, atol=1e-9 * np.abs(P).max())
        np.testing.assert_allclose(G @ P, (G @ P).T, atol=1e-10)


def test_leverage_sum_is_rank():
    """P2: sum of leverage scores = rank (trace of a projector)."""
    for dims, R in (((6, 5, 4), 3), ((5, 4, 3, 3), 4)):
        U = rand_factors(5, dims, R)
        for j in range(len(dims)):
            l = O.leverage_scores(O.design_matrix(U, j))
            assert abs(l.sum() - R) < 1e-12
            assert l.min() > -1e-14 and l.max() < 1 + 1e-12
        for u in U:
            lev, cdf, Z = O.arls_build(u, O.gram(u))
            assert abs(float(Z) - min(u.shape)) < 1e-12   # rank of U_k
    # a rank-deficient factor: duplicated column -> sum = rank = 2
    u = rand_factors(6, (7,), 2)[0]
    u3 = np.concatenate([u, u[:, :1]], axis=1)
    lev, cdf, Z = O.arls_build(u3, O.gram(u3))
    assert abs(float(Z) - 2) < 1e-12


def test_leverage_closed_form_orthonormal():
    """For A with orthonormal columns, l_i = ||A[i, :]||^2."""
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 4)))
    np.testing.assert_allclose(O.leverage_scores(Q), np.sum(Q * Q, axis=1),
                               atol=1e-14)


def test_normalize_columns_zero_column():
    X = np.array([[3.0, 0.0, 1.0], [4.0, 0.0, -1.0]])
    U, s = O.normalize_columns(X)
    np.testing.assert_allclose(s, [5.0, 0.0, np.sqrt(2)])
    np.testing.assert_allclose(U[:, 0], [0.6, 0.8])
    assert np.all(U[:, 1] == 0)


# ------------------------------------------------------------ MTTKRP

@pytest.mark.parametrize("dims,nnz,j", [((6, 5, 4), 50, 0), ((6, 5, 4), 50, 2),
                                        ((5, 4, 3, 3), 90, 1)])
def test_mttkrp_exact_equals_dense(dims, nnz, j):
    """mat(T, j) U_{!=j} via explicit matricization + KRP == per-nonzero loop."""
    T, _ = tg.tiny_tensor(11, dims, nnz)
    U = rand_factors(2, dims, 3)
    np.testing.assert_allclose(O.mttkrp_exact(T.idx, T.val, U, j),
                               O.mttkrp_dense(T.idx, T.val, dims, U, j),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dims,nnz,j", [((6, 5, 4), 60, 0), ((6, 5, 4), 60, 1),
                                        ((5, 4, 3, 3), 100, 3)])
def test_unit_weight_sampled_mttkrp_is_exact(dims, nnz, j):
    """P6: every nonempty column at unit weight gives the exact MTTKRP."""
    T, _ = tg.tiny_tensor(12, dims, nnz)
    U = rand_factors(4, dims, 3)
    keys = np.unique(O.column_key(T.idx, dims, j))
    ck, rows, vals, slot = O.extract(T.idx, T.val, dims, j, keys)
    assert rows.shape[0] == nnz
    A = O.design_matrix(U, j)
    M = O.sampled_mttkrp(dims[j], rows, vals, slot, np.ones(keys.shape[0]),
                         A[keys.astype(np.int64)])
    np.testing.assert_allclose(M, O.mttkrp_dense(T.idx, T.val, dims, U, j),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("sampler", ["arls", "sts"])
def test_sampled_mttkrp_matches_explicit_sketch(sampler):
    """mat(T,j) S^T S U_{!=j} with S formed explicitly (one 1/sqrt(Jp) per row)."""
    dims, j, J = (6, 5, 4), 1, 40
    T, _ = tg.tiny_tensor(13, dims, 70)
    U = rand_factors(7, dims, 3)
    G = [O.gram(u) for u in U]
    u = np.random.default_rng(9).random((J, 2))
    if sampler == "arls":
        st = {k: O.arls_build(U[k], G[k]) for k in range(3)}
        sidx, prob, h = O.arls_sample(U, st, j, u)
    else:
        sidx, prob, h = O.sts_sample(U, G, j, u, block=2)
    A = O.design_matrix(U, j)
    rows_x = O.sample_column_key(sidx, dims, j).astype(np.int64)
    np.testing.assert_allclose(h, A[rows_x], rtol=1e-14, atol=1e-15)
    S = np.zeros((J, A.shape[0]))
    S[np.arange(J), rows_x] = 1.0 / np.sqrt(J * prob)
    ref = O.matricize_dense(T.idx, T.val, dims, j) @ S.T @ S @ A
    keys, rep, counts, w = O.dedup(sidx, prob, dims, j, J)
    assert counts.sum() == J and np.all(rep == np.array(
        [np.nonzero(rows_x == k)[0].min() for k in keys.astype(np.int64)]))
    ck, rows, vals, slot = O.extract(T.idx, T.val, dims, j, keys)
    M = O.sampled_mttkrp(dims[j], rows, vals, slot, w, h[rep])
    np.testing.assert_allclose(M, ref, rtol=1e-12, atol=1e-12)


def test_extract_is_exactly_the_sampled_columns():
    dims, j = (7, 6, 5), 2
    T, _ = tg.tiny_tensor(14, dims, 120)
    allk = O.column_key(T.idx, dims, j)
    keys = np.unique(allk)[::3]
    keys = np.concatenate([keys, [np.uint64(10**6)]])  # a key with no nonzeros
    keys.sort()
    ck, rows, vals, slot = O.extract(T.idx, T.val, dims, j, keys)
    expect = {(int(c), int(r)) for c, r in zip(allk, T.idx[:, j])
              if c in set(keys.tolist())}
    assert set(zip(ck.tolist(), rows.tolist())) == expect
    assert np.all(np.diff(ck.astype(np.float64)) >= 0)
    assert np.all(keys[slot] == ck)


# -------------------------------------------------------------- samplers

def _tiny_state(seed, dims, R):
    U = rand_factors(seed, dims, R)
    G = [O.gram(u) for u in U]
    return U, G


@pytest.mark.parametrize("dims,j", [((6, 5, 4), 0), ((6, 5, 4), 2),
                                    ((5, 4, 3, 3), 1)])
def test_sts_probability_is_exact_leverage(dims, j):
    """P1 + P9: returned probabilities equal l_x / sum(l) from the explicit KRP."""
    U, G = _tiny_state(21, dims, 3)
    law = O.sts_law_bruteforce(U, j)
    u = np.random.default_rng(4).random((300, len(dims) - 1))
    sidx, prob, h = O.sts_sample(U, G, j, u, block=2)
    rows = O.sample_column_key(sidx, dims, j).astype(np.int64)
    np.testing.assert_allclose(prob, law[rows], rtol=1e-12)


@pytest.mark.parametrize("dims,j", [((6, 5, 4), 1), ((5, 4, 3, 3), 0)])
def test_arls_probability_is_product_of_factor_leverage(dims, j):
    U, G = _tiny_state(22, dims, 3)
    st = {k: O.arls_build(U[k], G[k]) for k in range(len(dims))}
    law = O.arls_law_bruteforce(U, j)
    u = np.random.default_rng(5).random((300, len(dims) - 1))
    sidx, prob, h = O.arls_sample(U, st, j, u)
    rows = O.sample_column_key(sidx, dims, j).astype(np.int64)
    np.testing.assert_allclose(prob, law[rows], rtol=1e-12)
    assert abs(law.sum() - 1) < 1e-12


@pytest.mark.parametrize("dims,j,block", [((6, 5, 4), 0, 1), ((6, 5, 4), 1, 4),
                                          ((5, 4, 3, 3), 2, 2),
                                          ((5, 4, 3, 3), 0, 64)])
def test_sts_map_equals_bruteforce_conditionals(dims, j, block):
    """P4: index(u) equals the sequential inverse CDF of the explicit law."""
    U, G = _tiny_state(23, dims, 3)
    u = np.random.default_rng(6).random((400, len(dims) - 1))
    a, _, _ = O.sts_sample(U, G, j, u, block=block)
    b = O.sts_sample_bruteforce(U, j, u)
    bad = np.nonzero(np.any(a != b, axis=1))[0]
    for s in bad:  # only tolerated within 1e-12 of a CDF boundary
        q = int(np.nonzero(a[s] != b[s])[0][0])
        gap = O.sts_boundary_gap(U, G, j, b, s, q, a[s, q], b[s, q], u[s, q])
        assert gap <= 1e-12, (s, q, gap)
    assert len(bad) == 0  # none expected with random uniforms


def test_arls_map_equals_explicit_inverse_cdf():
    dims, j = (6, 5, 4), 0
    U, G = _tiny_state(24, dims, 3)
    st = {k: O.arls_build(U[k], G[k]) for k in range(3)}
    u = np.random.default_rng(7).random((500, 2))
    a, _, _ = O.arls_sample(U, st, j, u)
    for q, k in enumerate([1, 2]):
        l = O.leverage_scores(U[k])
        c = np.cumsum(l / l.sum())
        ref = np.array([int(np.argmax(x < c)) for x in u[:, q]])
        np.testing.assert_array_equal(a[:, q], ref)


def test_sts_block_size_invariance():
    """P10: the map u -> index does not depend on the block size."""
    dims, j = (40, 30, 20), 1
    U, G = _tiny_state(25, dims, 4)
    u = np.random.default_rng(8).random((600, 2))
    ref, p0, _ = O.sts_sample(U, G, j, u, block=1)
    for block in (3, 8, 64):
        a, p, _ = O.sts_sample(U, G, j, u, block=block)
        np.testing.assert_array_equal(a, ref)
        np.testing.assert_allclose(p, p0, rtol=1e-13)


def test_zero_mass_rows_never_drawn():
    dims, j = (5, 6, 4), 0
    U, _ = _tiny_state(26, dims, 2)
    U[1][2] = 0.0
    U[2][0] = 0.0
    G = [O.gram(u) for u in U]
    u = np.random.default_rng(9).random((2000, 2))
    u[:5] = 0.0  # u = 0 would land on row 0 if zero mass were selectable
    for sidx in (O.sts_sample(U, G, j, u, block=2)[0],
                 O.arls_sample(U, {k: O.arls_build(U[k], G[k])
                                   for k in range(3)}, j, u)[0]):
        assert not np.any(sidx[:, 0] == 2)
        assert not np.any(sidx[:, 1] == 0)


def test_zero_mass_raises():
    U = [np.zeros((4, 2))]
    with pytest.raises(O.OracleError):
        O.arls_build(U[0], O.gram(U[0]))


def _chi2(counts, law, n):
    exp = law * n
    keep = exp >= 5
    obs = np.concatenate([counts[keep], [counts[~keep].sum()]])
    ex = np.concatenate([exp[keep], [exp[~keep].sum()]])
    if ex[-1] == 0:
        obs, ex = obs[:-1], ex[:-1]
    return stats.chisquare(obs, ex).pvalue


@pytest.mark.parametrize("sampler", ["sts", "arls"])
def test_sampler_laws_chi_square(sampler):
    """P3: empirical laws of 2e5 draws match the explicit laws (p > 1e-3)."""
    dims, j, n = (6, 5, 4), 0, 200_000
    U, G = _tiny_state(27, dims, 3)
    u = np.random.default_rng(10).random((n, 2))
    if sampler == "sts":
        sidx, _, _ = O.sts_sample(U, G, j, u, block=2, )
        law = O.sts_law_bruteforce(U, j)
    else:
        st = {k: O.arls_build(U[k], G[k]) for k in range(3)}
        sidx, _, _ = O.arls_sample(U, st, j, u)
        law = O.arls_law_bruteforce(U, j)
    rows = O.sample_column_key(sidx, dims, j).astype(np.int64)
    counts = np.bincount(rows, minlength=law.shape[0])
    assert _chi2(counts, law, n) > 1e-3
    # a wrong law (uniform) must be rejected by the same test
    assert _chi2(counts, np.full(law.shape, 1 / law.shape[0]), n) < 1e-3


@pytest.mark.parametrize("sampler", ["arls", "sts"])
def test_sampled_mttkrp_unbiased(sampler):
    """P7: the mean of K independent sampled MTTKRPs approaches the exact one."""
    dims, j, J, K = (6, 5, 4), 2, 16, 1500
    T, _ = tg.tiny_tensor(15, dims, 60)
    U, G = _tiny_state(28, dims, 3)
    st = {k: O.arls_build(U[k], G[k]) for k in range(3)}
    rng = np.random.default_rng(11)
    acc, acc2 = 0, 0
    for _ in range(K):
        u = rng.random((J, 2))
        if sampler == "arls":
            sidx, prob, h = O.arls_sample(U, st, j, u)
        else:
            sidx, prob, h = O.sts_sample(U, G, j, u, block=4)
        keys, rep, counts, w = O.dedup(sidx, prob, dims, j, J)
        ck, rows, vals, slot = O.extract(T.idx, T.val, dims, j, keys)
        M = O.sampled_mttkrp(dims[j], rows, vals, slot, w, h[rep])
        acc = acc + M
        acc2 = acc2 + M * M
    mean = acc / K
    sd = np.sqrt(np.maximum(acc2 / K - mean ** 2, 0))
    exact = O.mttkrp_exact(T.idx, T.val, U, j)
    z = np.abs(mean - exact) / (sd / np.sqrt(K) + 1e-12)
    assert np.max(z) < 5.0
    # the same test rejects a missing 1/J in the weight
    assert np.max(np.abs(mean * J - exact) / (J * sd / np.sqrt(K) + 1e-12)) > 5.0


# --------------------------------------------------------------- fit / ALS

def test_fit_matches_dense_reconstruction():
    dims = (6, 5, 4)
    T, _ = tg.tiny_tensor(16, dims, 70)
    U = [O.normalize_columns(u)[0] for u in rand_factors(12, dims, 3)]
    sigma = np.array([2.0, -0.5, 1.5])
    assert abs(O.fit(T.idx, T.val, sigma, U)
               - O.fit_dense(T.idx, T.val, dims, sigma, U)) < 1e-12


@pytest.mark.slow
def test_exact_als_recovers_noiseless_dense_low_rank():
    """P8: fit >= 0.999 on a noiseless planted rank-3 tensor (all entries)."""
    dims, R = (8, 7, 6), 3
    F = rand_factors(30, dims, R)
    T = np.einsum("ir,jr,kr->ijk", *F)
    idx = np.array(np.nonzero(np.ones(dims))).T
    val = T[tuple(idx.T)]
    U0 = rand_factors(31, dims, R)
    U, sigma, fits = O.als(idx, val, dims, R, "exact", U0, sweeps=500,
                           record_fit=True)
    assert fits[-1] >= 0.999
    assert abs(fits[-1] - O.fit_dense(idx, val, dims, sigma, U)) < 1e-9


@pytest.mark.slow
def test_exact_als_recovers_block_sparse_low_rank():
    """P8 on a genuinely sparse tensor: factors with disjoint supports."""
    dims, R = (12, 10, 9), 3
    rng = np.random.default_rng(32)
    F = []
    for d in dims:
        f = np.zeros((d, R))
        for r in range(R):
            lo, hi = r * d // R, (r + 1) * d // R
            f[lo:hi, r] = rng.uniform(0.5, 1.5, hi - lo)
        F.append(f)
    T = np.einsum("ir,jr,kr->ijk", *F)
    idx = np.array(np.nonzero(T)).T
    val = T[tuple(idx.T)]
    assert idx.shape[0] < 0.2 * np.prod(dims)
    U0 = rand_factors(33, dims, R)
    U0 = [np.abs(u) for u in U0]
    U, sigma, fits = O.als(idx, val, dims, R, "exact", U0, sweeps=500,
                           record_fit=True)
    assert fits[-1] >= 0.999


def test_randomized_als_tracks_exact_als():
    """Both samplers raise the fit and end near exact ALS (Alg. 1, Thm. 2.1)."""
    dims, R, J = (30, 25, 20), 4, 512
    T, _ = tg.tiny_tensor(17, dims, 3000, rank=R, noise_var=0.01)
    U0 = rand_factors(34, dims, R)
    uni = np.random.default_rng(12).random((6, 3, J, 2))
    _, _, ex = O.als(T.idx, T.val, dims, R, "exact", U0, sweeps=6,
                     record_fit=True)
    for sampler in ("arls", "sts"):
        U, s, fits = O.als(T.idx, T.val, dims, R, sampler, U0, uni, sweeps=6,
                           J=J, block=8, record_fit=True)
        assert fits[-1] > fits[0] + 0.05
        assert abs(fits[-1] - ex[-1]) < 0.03


@pytest.mark.parametrize("sampler", ["arls", "sts"])
def test_sketched_gram_is_explicit_sketch_product(sampler):
    """Fig. 3: G~ = (S A)^T (S A) with S formed explicitly, and the sketched
    update M G~^+ equals the least-squares solution of the explicitly
    sketched problem min ||(S A) X^T - S mat(T, j)^T|| (library lstsq)."""
    dims, j, J = (6, 5, 4), 2, 60
    T, _ = tg.tiny_tensor(14, dims, 90)
    U = rand_factors(8, dims, 3)
    G = [O.gram(u) for u in U]
    u = np.random.default_rng(10).random((J, 2))
    if sampler == "arls":
        st = {k: O.arls_build(U[k], G[k]) for k in range(3)}
        sidx, prob, h = O.arls_sample(U, st, j, u)
    else:
        sidx, prob, h = O.sts_sample(U, G, j, u, block=2)
    A = O.design_matrix(U, j)
    rows_x = O.sample_column_key(sidx, dims, j).astype(np.int64)
    S = np.zeros((J, A.shape[0]))
    S[np.arange(J), rows_x] = 1.0 / np.sqrt(J * prob)
    Gs = O.sketched_gram(h, prob, J)
    np.testing.assert_allclose(Gs, (S @ A).T @ (S @ A), rtol=1e-12,
                               atol=1e-13)
    keys, rep, counts, w = O.dedup(sidx, prob, dims, j, J)
    ck, rows, vals, slot = O.extract(T.idx, T.val, dims, j, keys)
    M = O.sampled_mttkrp(dims[j], rows, vals, slot, w, h[rep])
    X = M @ O.pinv_psd(Gs)
    B = O.matricize_dense(T.idx, T.val, dims, j)
    Xl = np.linalg.lstsq(S @ A, S @ B.T, rcond=None)[0].T
    np.testing.assert_allclose(X, Xl, rtol=1e-9, atol=1e-10)


def test_sketched_als_keeps_a_noiseless_planted_model():
    """With G~ a noiseless planted low-rank tensor is a fixed point of
    sampled ALS (the sketched problem is consistent); started next to the
    planted factors, sketched ALS stays at fit ~ 1 while the exact-G update
    (Eq. 4, Eq. 5) with the same draws moves away from it."""
    dims, R, J = (9, 8, 7), 3, 200
    F = rand_factors(35, dims, R)
    Tdense = np.einsum("ir,jr,kr->ijk", *F)
    idx = np.array(np.nonzero(np.ones(dims))).T
    val = Tdense[tuple(idx.T)]
    rng = np.random.default_rng(36)
    U0 = [f + 1e-9 * rng.standard_normal(f.shape) for f in F]
    uni = rng.random((3, 3, J, 2))
    _, _, fs = O.als(idx, val, dims, R, "arls", U0, uni, sweeps=3, J=J,
                     record_fit=True, sketched=True)
    _, _, fe = O.als(idx, val, dims, R, "arls", U0, uni, sweeps=3, J=J,
                     record_fit=True, sketched=False)
    assert fs[-1] > 1 - 1e-6
    assert fe[-1] < fs[-1] - 1e-4
