"""FP64 oracle: test infrastructure for the randomized sparse CP-ALS path.

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this
module.  Every function restates a definition or an algorithm of the paper
(section / equation / algorithm cited) in the most direct NumPy form.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "LD", "OracleError", "khatri_rao", "design_matrix", "column_key",
    "sample_column_key", "matricize_dense", "pinv_psd", "normalize_columns",
    "gram", "gram_hadamard", "leverage_scores", "arls_build", "inverse_cdf",
    "arls_sample", "sts_prefix_grams", "sts_sample", "sts_sample_bruteforce",
    "sts_law_bruteforce", "arls_law_bruteforce", "dedup", "extract",
    "sampled_mttkrp", "mttkrp_exact", "mttkrp_dense", "solve", "fit",
    "fit_dense", "als", "arls_boundary_gap", "sts_boundary_gap",
    "sts_conditional_cdf", "sketched_gram",
]

LD = np.longdouble
if np.finfo(LD).nmant < 63:  # pragma: no cover - x86-64 Linux has 80-bit
    raise ImportError("oracle needs an extended-precision long double")


class OracleError(ValueError):
    """Raised where the method has no defined result (e.g. zero mass)."""


# --------------------------------------------------------------------------
# Notation (Section 2) and the matricization / Khatri-Rao order (Eq. 3)
# --------------------------------------------------------------------------

def khatri_rao(A, B):
    """Column-wise Kronecker product: (A (.) B)[:, r] = A[:, r] (x) B[:, r]."""
    assert A.shape[1] == B.shape[1]
    return np.stack([np.kron(A[:, r], B[:, r]) for r in range(A.shape[1])],
                    axis=1)


def design_matrix(U, j):
    """U_{!=j} = U_N (.) ... (.) U_{j+1} (.) U_{j-1} (.) ... (.) U_1 (Eq. 3)."""
    order = [k for k in reversed(range(len(U))) if k != j]
    A = U[order[0]]
    for k in order[1:]:
        A = khatri_rao(A, U[k])
    return A


def _strides(dims, j):
    """Column strides of mat(T, j): mode 1 fastest among the modes != j.

    This is the row order of the Khatri-Rao product of Eq. (3): in A (.) B
    the row index of B varies fastest, and U_1 is the last operand.
    """
    s, out = 1, {}
    for k in range(len(dims)):
        if k == j:
            continue
        out[k] = s
        s *= int(dims[k])
    return out


def column_key(idx, dims, j):
    """Column of mat(T, j) for each nonzero coordinate tuple (uint64)."""
    st = _strides(dims, j)
    key = np.zeros(idx.shape[0], dtype=np.uint64)
    for k, s in st.items():
        key += idx[:, k].astype(np.uint64) * np.uint64(s)
    return key


def sample_column_key(sidx, dims, j):
    """Column key of sampled Khatri-Rao rows; sidx[:, q] is the q-th mode != j."""
    modes = [k for k in range(len(dims)) if k != j]
    st = _strides(dims, j)
    key = np.zeros(sidx.shape[0], dtype=np.uint64)
    for q, k in enumerate(modes):
        key += sidx[:, q].astype(np.uint64) * np.uint64(st[k])
    return key


def matricize_dense(idx, val, dims, j):
    """Dense mat(T, j), I_j x prod_{k != j} I_k (tiny tensors only)."""
    ncol = int(np.prod([d for k, d in enumerate(dims) if k != j]))
    M = np.zeros((dims[j], ncol))
    M[idx[:, j], column_key(idx, dims, j).astype(np.int64)] = val
    return M


# --------------------------------------------------------------------------
# Grams, pseudo-inverse, renormalisation (Eq. 4, Eq. 5, Alg. 1)
# --------------------------------------------------------------------------

def gram(U):
    """U^T U."""
    return U.T @ U


def gram_hadamard(G, j):
    """G = Hadamard product of the factor Grams G_k, k != j (Eq. 5)."""
    out = None
    for k, Gk in enumerate(G):
        if k == j:
            continue
        out = Gk.copy() if out is None else out * Gk
    return out


def pinv_psd(G):
    """Moore-Penrose pseudo-inverse of a symmetric PSD matrix (Eq. 4).

    The paper names only the Moore-Penrose inverse.  It is formed from the
    symmetric eigendecomposition; eigenvalues at or below R * 2^-52 *
    lambda_max count as zero.
    """
    G = 0.5 * (G + G.T)
    w, V = np.linalg.eigh(G)
    lmax = max(float(w.max()), 0.0)
    cut = G.shape[0] * 2.0 ** -52 * lmax
    inv = np.zeros_like(w)
    keep = w > cut
    inv[keep] = 1.0 / w[keep]
    return (V * inv) @ V.T


def normalize_columns(X):
    """sigma[r] = ||X[:, r]||_2 and X[:, r] /= sigma[r] (Alg. 1, renorm steps).

    A zero column has sigma = 0 and stays zero.
    """
    sigma = np.sqrt(np.sum(X * X, axis=0))
    U = np.zeros_like(X)
    nz = sigma > 0
    U[:, nz] = X[:, nz] / sigma[nz]
    return U, sigma


def leverage_scores(A):
    """l_i = A[i, :] (A^T A)^+ A[i, :]^T for an explicit matrix (Eq. 8)."""
    P = pinv_psd(A.T @ A)
    return np.einsum("ia,ab,ib->i", A, P, A)


# --------------------------------------------------------------------------
# CP-ARLS-LEV (Section 4.1; Appendix A, Alg. 2 and Alg. 3 on one device)
# --------------------------------------------------------------------------

def arls_build(U, G):
    """Alg. 2 on one device: dist = diag(U G^+ U^T); C = ||dist||_1.

    Returns (scores, cdf, Z): the unnormalised factor leverage scores, their
    inclusive prefix sums in extended precision and the total Z = C.
    """
    P = pinv_psd(G)
    lev = np.maximum(np.einsum("ia,ab,ib->i", U, P, U), 0.0)
    cdf = np.cumsum(lev.astype(LD))
    Z = cdf[-1]
    if not Z > 0:
        raise OracleError("zero sampling mass")
    return lev, cdf, Z


def inverse_cdf(cdf, Z, u):
    """index(u) = min{ i : u * Z < F(i) }, F the inclusive prefix sums.

    Rows of zero mass are never returned.  When u * Z reaches F(last) only
    through rounding, the last row of positive mass is returned.
    """
    t = np.asarray(u, dtype=LD) * LD(Z)
    i = np.searchsorted(cdf, t, side="right")
    last = int(np.searchsorted(cdf, cdf[-1], side="left"))
    return np.minimum(i, last).astype(np.int64)


def arls_sample(U, states, j, u):
    """Alg. 3 on one device: independent inverse-CDF draws per factor != j.

    states[k] = arls_build(U[k], G[k]); u has one column per mode != j in
    ascending order.  Returns (idx [J, N-1], prob [J], h [J, R]) with
    prob = prod_k l_k[idx_k] / Z_k (Appendix A) and h the Hadamard product
    of the drawn rows (a row of the Khatri-Rao design matrix).
    """
    N = len(U)
    modes = [k for k in range(N) if k != j]
    J = u.shape[0]
    R = U[0].shape[1]
    idx = np.zeros((J, N - 1), dtype=np.int64)
    prob = np.ones(J)
    h = np.ones((J, R))
    for q, k in enumerate(modes):
        lev, cdf, Z = states[k]
        i = inverse_cdf(cdf, Z, u[:, q])
        idx[:, q] = i
        prob = prob * (lev[i] / float(Z))
        h = h * U[k][i]
    return idx, prob, h


def arls_law_bruteforce(U, j):
    """Exact CP-ARLS-LEV law over all Khatri-Rao rows, from explicit pinvs.

    Row order is that of design_matrix(U, j); the probability of a row is
    the product over k != j of l_k(i_k) / sum(l_k) (Appendix A).
    """
    N = len(U)
    order = [k for k in reversed(range(N)) if k != j]
    p = None
    for k in order:
        lk = leverage_scores(U[k])
        lk = lk / lk.sum()
        p = lk if p is None else np.kron(p, lk)
    return p


# --------------------------------------------------------------------------
# STS-CP (Section 4.1; Appendix B, Alg. 4 and Alg. 5 on one device)
# --------------------------------------------------------------------------

def _g_after(Gp, G, modes, q):
    """G_{>k} = G^+ (*) Hadamard of G_m over the modes drawn after modes[q]."""
    out = Gp.copy()
    for m in modes[q + 1:]:
        out = out * G[m]
    return out


def sts_prefix_grams(U, block):
    """P[b] = sum over rows below b*block of u_i u_i^T, extended precision.

    A stand-in for the paper's segment tree (Section 4.1, Alg. 4): any node
    Gram is a difference of two prefix Grams, so the conditional CDF at a
    block boundary is h^T (P[b] (*) G_{>k}) h.
    """
    I, R = U.shape
    nb = (I + block - 1) // block
    P = np.zeros((nb + 1, R, R), dtype=LD)
    UL = U.astype(LD)
    for b in range(nb):
        rows = UL[b * block:(b + 1) * block]
        P[b + 1] = P[b] + rows.T @ rows
    return P


def _sts_draw_factor(U, Ggt, h, u, block, P=None, chunk=512):
    """Draw one factor's row for every sample from its conditional law.

    Conditional mass of row i given h (Appendix B):
        m_i = (U[i] (*) h)^T G_{>k} (U[i] (*) h),
    and index(u) = min{ i : u * Z < F(i) } with F the prefix masses.
    Block boundaries are found by bisection on prefix Grams, then the rows
    of the chosen block are scanned.
    """
    I, R = U.shape
    if P is None:
        P = sts_prefix_grams(U, block)
    nb = P.shape[0] - 1
    J = h.shape[0]
    out = np.zeros(J, dtype=np.int64)
    UL = U.astype(LD)
    GL = Ggt.astype(LD)
    for c0 in range(0, J, chunk):
        hs = h[c0:c0 + chunk].astype(LD)
        n = hs.shape[0]
        W = hs[:, :, None] * hs[:, None, :] * GL[None]        # (h h^T) (*) G
        Z = np.einsum("sab,ab->s", W, P[nb])
        if not np.all(Z > 0):
            raise OracleError("zero conditional sampling mass")
        t = np.asarray(u[c0:c0 + chunk], dtype=LD) * Z
        lo = np.zeros(n, dtype=np.int64)
        hi = np.full(n, nb, dtype=np.int64)
        while True:
            act = hi - lo > 1
            if not act.any():
                break
            mid = (lo + hi) // 2
            Fm = np.einsum("sab,sab->s", W, P[mid])
            go = act & (Fm <= t)
            lo = np.where(go, mid, lo)
            hi = np.where(act & ~go, mid, hi)
        # scan the rows of the chosen block for every sample at once
        Fb = np.einsum("sab,sab->s", W, P[lo])
        rid = lo[:, None] * block + np.arange(block)[None, :]
        valid = rid < I
        rows = UL[np.minimum(rid, I - 1)]                     # [n, block, R]
        m = np.einsum("sra,sab,srb->sr", rows, W, rows)
        m = np.where(valid & (m > 0), m, LD(0))
        F = Fb[:, None] + np.cumsum(m, axis=1)
        hit = (t[:, None] < F) & (m > 0)
        found = hit.any(axis=1)
        first = np.argmax(hit, axis=1)
        out[c0:c0 + n] = rid[np.arange(n), first]
        for s in np.nonzero(~found)[0]:  # rounding pushed u*Z past the block
            out[c0 + s] = _scan_from_block(UL, W[s], P, int(lo[s]), t[s],
                                           block)
    return out


def _scan_from_block(UL, Ws, P, b, t, block):
    I = UL.shape[0]
    F = np.sum(Ws * P[b])
    last_pos = -1
    nb = P.shape[0] - 1
    while b < nb:
        rows = UL[b * block:(b + 1) * block]
        m = np.einsum("ra,ab,rb->r", rows, Ws, rows)
        for r in range(rows.shape[0]):
            if m[r] > 0:
                F = F + m[r]
                last_pos = b * block + r
                if t < F:
                    return last_pos
        b += 1
    if last_pos < 0:  # only reachable through rounding at the far end
        for i in range(I - 1, -1, -1):
            if UL[i] @ Ws @ UL[i] > 0:
                return i
        raise OracleError("zero conditional sampling mass")
    return last_pos


def sts_sample(U, G, j, u, block=64, prefix=None):
    """STS-CP draws on one device (Appendix B, Alg. 5 without routing).

    Factors != j are drawn in ascending mode order.  h starts at ones and is
    multiplied by each drawn row.  Returns (idx, prob, h) with the S-matrix
    probability prob = (h^T G^+ h) / <G^+, G> (the exact leverage law).
    `prefix` may hold precomputed sts_prefix_grams per mode.
    """
    N = len(U)
    modes = [k for k in range(N) if k != j]
    J = u.shape[0]
    R = U[0].shape[1]
    Gfull = gram_hadamard(G, j)
    Gp = pinv_psd(Gfull)
    idx = np.zeros((J, N - 1), dtype=np.int64)
    h = np.ones((J, R))
    for q, k in enumerate(modes):
        Ggt = _g_after(Gp, G, modes, q)
        P = None if prefix is None else prefix[k]
        i = _sts_draw_factor(U[k], Ggt, h, u[:, q], block, P)
        idx[:, q] = i
        h = h * U[k][i]
    lev = np.einsum("sa,ab,sb->s", h, Gp, h)
    prob = lev / np.sum(Gp * Gfull)
    return idx, prob, h


def sts_law_bruteforce(U, j):
    """Exact leverage law of the Khatri-Rao rows: l / sum(l) (Eq. 8)."""
    l = leverage_scores(design_matrix(U, j))
    return l / l.sum()


def sts_sample_bruteforce(U, j, u):
    """Sequential conditional inverse CDF from explicit leverage scores.

    For tiny tensors only.  The explicit law over design_matrix rows is
    marginalised onto the ascending modes != j one at a time; each index is
    min{ i : u * Z < F(i) } of its conditional law given the earlier ones.
    """
    N = len(U)
    modes = [k for k in range(N) if k != j]
    dims = [U[k].shape[0] for k in range(N)]
    lev = leverage_scores(design_matrix(U, j))
    # design_matrix row r corresponds to indices with mode 1 fastest among
    # the modes != j; reshape to an (N-1)-way array indexed [i_{m1}, ...].
    shape = [dims[k] for k in reversed(modes)]
    L = lev.reshape(shape)                       # axes: last mode first
    L = np.transpose(L, list(reversed(range(N - 1))))  # axes: ascending modes
    J = u.shape[0]
    out = np.zeros((J, N - 1), dtype=np.int64)
    for s in range(J):
        sub = L
        for q in range(N - 1):
            marg = sub.reshape(sub.shape[0], -1).sum(axis=1)
            cdf = np.cumsum(marg.astype(LD))
            i = int(inverse_cdf(cdf, cdf[-1], np.array([u[s, q]]))[0])
            out[s, q] = i
            sub = sub[i]
    return out


def sts_conditional_cdf(U, G, j, sidx, s, q, rows):
    """Normalised conditional CDF values F(i)/Z, i in rows, for draw (s, q).

    Used to adjudicate index mismatches: it recomputes, in extended
    precision and directly from the definition, the conditional law of
    factor modes[q] given the sample's earlier indices.
    """
    N = len(U)
    modes = [k for k in range(N) if k != j]
    Gp = pinv_psd(gram_hadamard(G, j))
    h = np.ones(U[0].shape[1], dtype=LD)
    for p in range(q):
        h = h * U[modes[p]][sidx[s, p]].astype(LD)
    Ggt = _g_after(Gp, G, modes, q).astype(LD)
    W = h[:, None] * h[None, :] * Ggt
    Uk = U[modes[q]].astype(LD)
    m = np.einsum("ra,ab,rb->r", Uk, W, Uk)
    m = np.maximum(m, 0)
    F = np.cumsum(m)
    return F[np.asarray(rows)] / F[-1]


def arls_boundary_gap(states, k, u, i_a, i_b):
    """Distance from u to the CDF boundaries separating indices i_a and i_b."""
    lev, cdf, Z = states[k]
    lo, hi = min(i_a, i_b), max(i_a, i_b)
    Fs = np.array([cdf[lo] / Z, cdf[hi - 1] / Z], dtype=LD)
    return float(np.max(np.abs(Fs - LD(u))))


def sts_boundary_gap(U, G, j, sidx, s, q, i_a, i_b, u):
    lo, hi = min(i_a, i_b), max(i_a, i_b)
    Fs = sts_conditional_cdf(U, G, j, sidx, s, q, [lo, hi - 1])
    return float(np.max(np.abs(Fs - LD(u))))


# --------------------------------------------------------------------------
# Sketch application and sampled MTTKRP (Section 2.2, Eq. 7; Section 4.3)
# --------------------------------------------------------------------------

def dedup(sidx, prob, dims, j, J):
    """Merge duplicate draws (Section 2.2: S extracts and reweights rows).

    Each draw of Khatri-Rao row x contributes 1/(J p_x) to S^T S, so the
    distinct columns get weight count / (J p_x).  Returns (keys, rep,
    counts, w): sorted distinct column keys of mat(T, j), the first draw of
    each key, draw counts and weights.
    """
    keys = sample_column_key(sidx, dims, j)
    uk, first, counts = np.unique(keys, return_index=True, return_counts=True)
    w = counts / (J * prob[first])
    return uk, first, counts, w


def extract(idx, val, dims, j, keys, chunk=1 << 24):
    """Nonzeros of mat(T, j) lying in the sampled columns (Section 4.3).

    A brute-force scan over all nonzeros (no index): keep e iff its column
    key is one of `keys`.  Output sorted by (column key, row i_j): arrays
    (col_key, row, val, slot) with slot the position of the key in `keys`.
    """
    sel = []
    for c0 in range(0, idx.shape[0], chunk):
        c = column_key(idx[c0:c0 + chunk], dims, j)
        sel.append(np.nonzero(np.isin(c, keys))[0] + c0)
    sel = np.concatenate(sel) if sel else np.zeros(0, dtype=np.int64)
    ck = column_key(idx[sel], dims, j)
    rows = idx[sel, j].astype(np.int64)
    order = np.lexsort((rows, ck))
    sel, ck, rows = sel[order], ck[order], rows[order]
    slot = np.searchsorted(keys, ck)
    return ck, rows, val[sel].astype(np.float64), slot


def sampled_mttkrp(I_j, rows, vals, slot, w, h_rep):
    """mat(T, j) S^T S U_{!=j} (Eq. 7): M[i, :] += w_x v h_x per extracted nonzero."""
    R = h_rep.shape[1]
    M = np.zeros((I_j, R))
    contrib = (w[slot] * vals)[:, None] * h_rep[slot]
    np.add.at(M, rows, contrib)
    return M


def mttkrp_exact(idx, val, U, j):
    """mat(T, j) U_{!=j} as a per-nonzero Hadamard loop (Section 2.1)."""
    R = U[0].shape[1]
    H = np.asarray(val, dtype=np.float64)[:, None] * np.ones((1, R))
    for k in range(len(U)):
        if k != j:
            H = H * U[k][idx[:, k]]
    M = np.zeros((U[j].shape[0], R))
    np.add.at(M, idx[:, j], H)
    return M


def mttkrp_dense(idx, val, dims, U, j):
    """mat(T, j) U_{!=j} with explicit matricization and Khatri-Rao product."""
    return matricize_dense(idx, val, dims, j) @ design_matrix(U, j)


def sketched_gram(h, prob, J):
    """G~ = (S U_{!=j})^T (S U_{!=j}) of the sketched least-squares problem
    (Fig. 3): every draw s adds h_s h_s^T / (J p_s), h_s its Khatri-Rao row
    (a row of S carries 1/sqrt(J p_s)).  Duplicates add up as S^T S does."""
    wt = 1.0 / (J * np.asarray(prob, dtype=np.float64))
    return (h * wt[:, None]).T @ h


def solve(M, Gp):
    """U_j = M G^+ (Eq. 4), then sigma and renormalisation (Alg. 1)."""
    return normalize_columns(M @ Gp)


# --------------------------------------------------------------------------
# Fit (Section 5.1) and the ALS driver (Alg. 1)
# --------------------------------------------------------------------------

def fit(idx, val, sigma, U):
    """fit = 1 - ||[sigma; U] - T||_F / ||T||_F for a sparse T (Section 5.1).

    ||[sigma; U] - T||^2 = ||T||^2 - 2 <T, [sigma; U]> + sigma^T (*G_k) sigma,
    expanded over the nonzeros and clamped at zero.
    """
    v = np.asarray(val, dtype=np.float64)
    t2 = float(np.sum(v * v))
    P = np.ones((idx.shape[0], sigma.shape[0])) * sigma[None, :]
    for k in range(len(U)):
        P = P * U[k][idx[:, k]]
    inner = float(np.sum(v * P.sum(axis=1)))
    Gh = np.ones((sigma.shape[0], sigma.shape[0]))
    for Uk in U:
        Gh = Gh * (Uk.T @ Uk)
    m2 = float(sigma @ Gh @ sigma)
    res2 = max(0.0, t2 - 2.0 * inner + m2)
    return 1.0 - np.sqrt(res2) / np.sqrt(t2)


def fit_dense(idx, val, dims, sigma, U):
    """The same fit from an explicitly reconstructed dense tensor (tiny only)."""
    T = np.zeros(dims)
    T[tuple(idx[:, k] for k in range(len(dims)))] = val
    X = np.zeros(dims)
    for r in range(sigma.shape[0]):
        comp = np.array(sigma[r])
        for k in range(len(dims)):
            comp = np.multiply.outer(comp, U[k][:, r])
        X = X + comp
    return 1.0 - np.linalg.norm((X - T).ravel()) / np.linalg.norm(T.ravel())


def als(idx, val, dims, R, sampler, U0, uniforms=None, sweeps=1, J=None,
        block=64, record_fit=False, sketched=False):
    """Randomized CP-ALS (Alg. 1 with the three steps of Section 4 per mode).

    sampler: "arls", "sts" or "exact" (every nonempty column at weight 1).
    U0: initial factors (float64); they are column-normalised and sigma = 1.
    uniforms[t, j] holds the J x (N-1) uniforms of mode j in sweep t.
    sketched: solve with the sketched Gram G~ of the draws (Fig. 3) instead
    of the exact Hadamard Gram G (Eq. 5); the draws still follow G.
    Returns (U, sigma, fits) where fits is per sweep if record_fit.
    """
    N = len(dims)
    U, sigma = [], np.ones(R)
    for k in range(N):
        Uk, _ = normalize_columns(np.asarray(U0[k], dtype=np.float64))
        U.append(Uk)
    G = [gram(Uk) for Uk in U]
    states = {k: arls_build(U[k], G[k]) for k in range(N)} \
        if sampler == "arls" else None
    fits = []
    for t in range(sweeps):
        for j in range(N):
            Gp = pinv_psd(gram_hadamard(G, j))
            if sampler == "exact":
                M = mttkrp_exact(idx, val, U, j)
            else:
                u = uniforms[t, j]
                if sampler == "arls":
                    sidx, prob, h = arls_sample(U, states, j, u)
                else:
                    sidx, prob, h = sts_sample(U, G, j, u, block)
                keys, rep, counts, w = dedup(sidx, prob, dims, j, J)
                ck, rows, vals, slot = extract(idx, val, dims, j, keys)
                M = sampled_mttkrp(dims[j], rows, vals, slot, w, h[rep])
                if sketched:
                    Gp = pinv_psd(sketched_gram(h, prob, J))
            U[j], sigma = solve(M, Gp)
            G[j] = gram(U[j])
            if sampler == "arls":
                states[j] = arls_build(U[j], G[j])
        if record_fit:
            fits.append(fit(idx, val, sigma, U))
    return U, sigma, fits
