"""Pins for the oracle's index-mismatch adjudication (CPU only).

When the HIP path and the oracle draw different indices from the same
uniform, the parity tests accept the difference only if the uniform lies
within 1e-12 of the CDF boundary (or boundaries) separating the two indices
(inverse-CDF rule of Appendix A and Appendix B: index = min{i : u Z < F(i)}).
The helpers that decide this are pinned here against hand-derived values
(tests/golden/samplers_worked.json) and against conditional marginals of the
explicitly formed leverage law, so that a wrong normaliser, a wrong boundary
index or a wrong conditioning would fail.
"""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
BAND = 1e-12


def _worked():
    with open(os.path.join(GOLD, "samplers_worked.json")) as f:
        g = json.load(f)
    U = [np.ones((3, 2)), np.array(g["U2"], float), np.array(g["U3"], float)]
    return g, U, [O.gram(u) for u in U]


def test_conditional_cdf_worked_example():
    g, U, G = _worked()
    for case in g["conditional_cdf_cases"]:
        q = case["q"]
        sidx = np.zeros((1, 2), dtype=np.int64)
        sidx[0, :q] = case["prior"]
        rows = list(range(U[1 + q].shape[0]))
        F = O.sts_conditional_cdf(U, G, 0, sidx, 0, q, rows)
        np.testing.assert_allclose(np.asarray(F, float), case["cdf"],
                                   atol=1e-15)


@pytest.mark.parametrize("dims,j", [((6, 5, 4), 0), ((6, 5, 4), 1),
                                    ((6, 5, 4), 2), ((4, 3, 3, 3), 1)])
def test_conditional_cdf_equals_bruteforce_marginals(dims, j):
    """F(i)/Z of sts_conditional_cdf = cumulative conditional marginals of the
    explicit leverage law l / sum(l) of the Khatri-Rao rows (Eq. 8)."""
    rng = np.random.default_rng(sum(dims) * 10 + j)
    R = 3
    U = [rng.standard_normal((d, R)) for d in dims]
    U[[k for k in range(len(dims)) if k != j][-1]][1] = 0.0  # a zero-mass row
    G = [O.gram(u) for u in U]
    modes = [k for k in range(len(dims)) if k != j]
    law = O.sts_law_bruteforce(U, j)
    # design_matrix rows: first mode != j fastest -> axes in ascending modes
    L = law.reshape([dims[k] for k in reversed(modes)])
    L = np.transpose(L, list(reversed(range(len(modes)))))
    for trial in range(6):
        prior = [int(rng.integers(dims[k])) for k in modes]
        for q in range(len(modes)):
            sub = L[tuple(prior[:q])]
            marg = sub.reshape(sub.shape[0], -1).sum(axis=1)
            if marg.sum() <= 0:
                continue  # conditioning on a zero-probability prefix
            ref = np.cumsum(marg) / marg.sum()
            sidx = np.array([prior], dtype=np.int64)
            F = O.sts_conditional_cdf(U, G, j, sidx, 0, q,
                                      list(range(dims[modes[q]])))
            np.testing.assert_allclose(np.asarray(F, float), ref, atol=1e-12)


def test_arls_boundary_gap_worked_example():
    g, U, G = _worked()
    states = {k: O.arls_build(U[k], G[k]) for k in (1, 2)}
    for case in g["arls_gap_cases"]:
        gap = O.arls_boundary_gap(states, case["mode"], case["u"],
                                  case["i_a"], case["i_b"])
        if "gap_max" in case:
            assert gap <= case["gap_max"], (case, gap)
        else:
            assert gap >= case["gap_min"], (case, gap)


def test_sts_boundary_gap_worked_example():
    g, U, G = _worked()
    for case in g["sts_gap_cases"]:
        sidx = np.array([[case["prior"][0], 0]], dtype=np.int64)
        gap = O.sts_boundary_gap(U, G, 0, sidx, 0, 1, case["i_a"],
                                 case["i_b"], case["u"])
        if "gap_max" in case:
            assert gap <= case["gap_max"], (case, gap)
        else:
            assert gap >= case["gap_min"], (case, gap)


def test_arls_gap_accepts_only_near_boundary_on_random_factor():
    """For every boundary of a random factor's CDF: u 1e-13 past F(i)/Z
    separates indices i and i + 1 within the band (and the oracle itself
    draws i + 1 there); u at the middle of row i's interval does not."""
    rng = np.random.default_rng(7)
    U = rng.standard_normal((50, 4))
    U[10] = 0.0  # zero-mass row: indices 9 and 11 share a boundary
    G = O.gram(U)
    st = {0: O.arls_build(U, G)}
    lev, cdf, Z = st[0]
    Fn = np.asarray(cdf / Z, dtype=float)
    for i in range(49):
        if lev[i + 1] == 0 or lev[i] == 0:
            continue
        u = Fn[i] + 1e-13
        assert O.inverse_cdf(cdf, Z, np.array([u]))[0] == i + 1
        assert O.arls_boundary_gap(st, 0, u, i + 1, i) <= BAND
        mid = (Fn[i] + (Fn[i - 1] if i > 0 else 0.0)) / 2
        assert O.arls_boundary_gap(st, 0, mid, i + 1, i) > 1e-6
    # across the zero-mass row 10: 9 vs 11 is one boundary
    u = Fn[9] + 1e-13
    assert O.inverse_cdf(cdf, Z, np.array([u]))[0] == 11
    assert O.arls_boundary_gap(st, 0, u, 11, 9) <= BAND
    # 8 vs 11 spans row 9's interval of positive mass
    assert O.arls_boundary_gap(st, 0, u, 11, 8) > 1e-6


def test_sts_gap_rejects_mismatch_conditioned_on_wrong_prefix():
    """The gap is computed under the sample's own earlier indices: a
    boundary of a different prefix's conditional law is not accepted."""
    g, U, G = _worked()
    # given i_2 = 1 the CDF of mode 3 is (0, 1/2, 1); u = 1e-13 is at the
    # boundary 0 | 1 there, but given i_2 = 0 (CDF (1/2, 1/2, 1)) it is 1/2
    # away from every boundary
    s1 = np.array([[1, 0]], dtype=np.int64)
    s0 = np.array([[0, 0]], dtype=np.int64)
    assert O.sts_boundary_gap(U, G, 0, s1, 0, 1, 1, 0, 1e-13) <= BAND
    assert O.sts_boundary_gap(U, G, 0, s0, 0, 1, 1, 0, 1e-13) >= 0.49
