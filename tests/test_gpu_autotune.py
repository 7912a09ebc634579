"""The autotuner on the GPU, on a small tensor: every candidate of the
context tuner (per-factor or fixed leaf sizes, then bucket sizes up to 256
rows) and of the batch tuner (stream counts) builds, sweeps and closes; the
choice is one of the candidates, is cached, and is read back."""
import numpy as np
import pytest

import tensorgen as tg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_05105_amd import load_library
    load_library()
    return torch.device("cuda:0")


def test_context_and_batch_tuners(dev, tmp_path, monkeypatch):
    monkeypatch.setenv("CPR_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_2210_05105_amd import autotune as at
    T = tg.zipf_tensor(46, (3000, 2400, 1800), 100_000, s=1.1)
    idx = torch.from_numpy(np.ascontiguousarray(T.idx)).to(dev)
    val = torch.from_numpy(T.val.astype(np.float32)).to(dev)
    res = at.tune_context(idx, val, T.dims, 32, "sts", "fp32", 2048, sweeps=2)
    assert not res["cached"]
    assert len(res["tried"]) == len(at.LEAVES) + len(at.BUCKETS)
    assert all(ms is not None and ms > 0 for ms in res["tried"].values())
    assert res["sts_leaf"] in at.LEAVES
    assert res["bucket_rows"] in (0,) + at.BUCKETS
    again = at.tune_context(idx, val, T.dims, 32, "sts", "fp32", 2048)
    assert again["cached"] and again["sts_leaf"] == res["sts_leaf"]
    ranks = [8, 16, 32]
    rb = at.tune_batch(idx, val, T.dims, ranks, "arls", "mixed", 1024,
                       sweeps=1)
    assert rb["nstreams"] in (1, 2) and rb["sts_leaf"] == 0
    assert len(rb["tried"]) == 2
