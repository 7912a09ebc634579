"""cp_pinv_noalloc (no device allocation) against cp_pinv, through the C ABI.

Two calls in a row on one device, the second with a smaller input, each
compared with the allocating entry point on the same input (same kernels:
the results must agree to the pseudo-inverse parity bar, 1e-10 relative
Frobenius), and both against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _psd(rng, R, rank):
    B = rng.standard_normal((max(rank, 1) + 30, R))
    if rank < R:
        B = B[:, :rank] @ rng.standard_normal((rank, R))
    B /= np.maximum(np.linalg.norm(B, axis=0), 1e-300)
    return B.T @ B


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_pinv_noalloc_matches_allocating_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import CprError, load_library, pinv, pinv_noalloc
    load_library()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(77)
    # second call smaller than the first; a rank-deficient case exercises
    # the eigen fallback, whose work area is the static scratch
    for R, rank in ((100, 100), (24, 24), (48, 30), (7, 7)):
        G = _psd(rng, R, rank)
        Gd = torch.from_numpy(G).to(dev)
        out = torch.full((R, R), float("nan"), dtype=torch.float64, device=dev)
        pinv_noalloc(Gd, out)
        ref = pinv(Gd).cpu().numpy()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert _rel(got, ref) < 1e-10, (R, _rel(got, ref))
        assert _rel(got, O.pinv_psd(G)) < 1e-8, (R, _rel(got, O.pinv_psd(G)))
    # beyond the scratch's maximum size: a clear error, nothing launched
    big = torch.eye(129, dtype=torch.float64, device=dev)
    with pytest.raises(CprError) as e:
        pinv_noalloc(big, torch.empty_like(big))
    assert e.value.name == "CP_EINVAL"
    # non-finite input is reported, and the next call starts clean
    bad = torch.from_numpy(_psd(rng, 16, 16)).to(dev)
    bad[3, 3] = float("nan")
    with pytest.raises(CprError) as e:
        pinv_noalloc(bad, torch.empty_like(bad))
    assert e.value.name == "CP_ENUMERIC"
    G = _psd(rng, 16, 16)
    out = torch.empty((16, 16), dtype=torch.float64, device=dev)
    pinv_noalloc(torch.from_numpy(G).to(dev), out)
    assert _rel(out.cpu().numpy(), O.pinv_psd(G)) < 1e-8
