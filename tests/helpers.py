"""Shared helpers for the GPU parity tests (HIP path vs FP64 oracle)."""
import numpy as np

import oracle as O

BAND = 1e-12  # CDF-boundary exemption for sample indices


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_state(ctx):
    """Factors and factor Grams as the GPU holds them (exact FP64 copies)."""
    U = [to_np(ctx.get_factor(k)) for k in range(ctx.N)]
    G = [to_np(ctx.get_gram(k)) for k in range(ctx.N)]
    return U, G


def cond_psd(G):
    """Condition number over the eigenvalues the pseudo-inverse keeps."""
    w = np.linalg.eigvalsh(0.5 * (G + G.T))
    cut = G.shape[0] * 2.0 ** -52 * max(w.max(), 0)
    keep = w[w > cut]
    return float(keep.max() / keep.min()) if keep.size else 1.0


def pinv_rtol(base, *grams):
    """Relative tolerance for results that go through a pseudo-inverse:
    two correct FP64 pseudo-inverses differ by about cond * eps."""
    k = max(cond_psd(G) for G in grams)
    return max(base, 100.0 * k * 2.0 ** -52)


def rel_fro(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def compare_arls_indices(gidx, oidx, U, G, j, u):
    """Indices must match except within BAND of a CDF boundary.

    Returns the number of accepted (in-band) mismatches; fails on others.
    Later factors of a sample depend only on their own uniforms for ARLS.
    """
    modes = [k for k in range(len(U)) if k != j]
    states = {k: O.arls_build(U[k], G[k]) for k in modes}
    bad = np.argwhere(gidx != oidx)
    for s, q in bad:
        gap = O.arls_boundary_gap(states, modes[q], u[s, q], int(gidx[s, q]),
                                  int(oidx[s, q]))
        assert gap <= BAND, (s, q, gidx[s, q], oidx[s, q], gap)
    return len(bad)


def compare_sts_indices(gidx, oidx, U, G, j, u):
    """As compare_arls_indices for STS-CP.  After the first in-band mismatch
    of a sample its later factors are conditioned differently and skipped."""
    n_acc = 0
    rows = np.nonzero(np.any(gidx != oidx, axis=1))[0]
    for s in rows:
        q = int(np.nonzero(gidx[s] != oidx[s])[0][0])
        gap = O.sts_boundary_gap(U, G, j, oidx, s, q, int(gidx[s, q]),
                                 int(oidx[s, q]), u[s, q])
        assert gap <= BAND, (s, q, gidx[s, q], oidx[s, q], gap)
        n_acc += 1
    return n_acc


def oracle_sampled_M(T, dims, j, sidx, prob, U, J):
    """Oracle sampled MTTKRP for given draws (teacher forcing)."""
    R = U[0].shape[1]
    h = np.ones((sidx.shape[0], R))
    modes = [k for k in range(len(dims)) if k != j]
    for q, k in enumerate(modes):
        h = h * U[k][sidx[:, q]]
    keys, rep, counts, w = O.dedup(sidx, prob, dims, j, J)
    ck, rows, vals, slot = O.extract(T.idx, T.val, dims, j, keys)
    M = O.sampled_mttkrp(dims[j], rows, vals, slot, w, h[rep])
    return dict(keys=keys, rep=rep, counts=counts, w=w, ck=ck, rows=rows,
                slot=slot, M=M, h=h)
