"""Sweep autotuner: tuned and default launch configurations give the same products (they only
change how rows and columns are spread over waves and workgroups), and the tuned choice lands in
the JSON cache."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from helpers import import_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1507_04396_amd import _lib
    _lib.load()


def test_tuned_products_equal_default_and_cache_written(tmp_path, monkeypatch):
    A = workloads.knn_points_matrix(1500, 3, 10, 0.01, 6)
    ref = oracle.factor(A, k=3, eta=0.5, core=64, cluster=(64, 256), seed=2)
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PMMF_TUNE_CACHE", str(cache))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    X = torch.randn(A.n, 96, generator=gen, device="cuda")
    Yb = torch.randn(A.n, 96, generator=gen, device="cuda")
    monkeypatch.setenv("PMMF_AUTOTUNE", "0")
    f0 = import_oracle(ref)
    y0 = f0.apply(X)
    b0 = f0.backward(X, Yb, want=("x", "hdiag", "hcore"))
    torch.cuda.synchronize()
    monkeypatch.setenv("PMMF_AUTOTUNE", "1")
    f1 = import_oracle(ref)
    print("[autotune] tuning apply and adjoint", flush=True)
    y1 = f1.apply(X)
    b1 = f1.backward(X, Yb, want=("x", "hdiag", "hcore"))
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    for u, v in zip(b0, b1):
        if u is not None:
            assert torch.equal(u, v)
    text = cache.read_text()
    entries = json.loads(text)
    print(f"[autotune] cache: {entries}", flush=True)
    assert any("|apply|k3|" in k for k in entries)
    assert any("|adjoint|k3|" in k for k in entries)
    for v in entries.values():
        assert v["wpb"] in (1, 2, 4) and v["W"] >= 1 and v["ms"] > 0
