"""Captured products: mmf_graph_capture / mmf_graph_launch replayed against eager mmf_apply and
mmf_apply_inverse (bit-identical: the graph holds the same kernels on the same data), with eager
work and synchronizations between replays, and the refusals that keep a stale graph from running.
"""
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    ("grid20x20_k2", lambda: workloads.small_grid((20, 20), sigma=0.5, shift=0.3, seed=2),
     dict(k=2, core=24, cluster=(16, 64), seed=3), 37),
    ("knn2d_n600_k3", lambda: workloads.knn_points_matrix(600, 2, 8, 0.01, 5),
     dict(k=3, core=40, cluster=(32, 128), seed=1), 64),
]


@pytest.mark.parametrize("name,make,params,nrhs", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("inverse", [False, True, "sqrt"])
def test_graph_replays_match_eager(name, make, params, nrhs, inverse):
    A = make()
    ref = oracle.factor(A, **params)
    fac = import_oracle(ref)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(17)
    X = torch.randn(A.n, nrhs, generator=gen, device="cuda")
    Y = torch.empty_like(X)
    _say(f"[graph] {name} inverse={inverse}: capture")
    g = fac.capture(X, Y, inverse=inverse)
    torch.cuda.synchronize()
    assert torch.equal(Y, fac.apply(X, inverse=inverse))
    for rep in range(4):
        X.copy_(torch.randn(A.n, nrhs, generator=gen, device="cuda"))  # eager work between replays
        torch.cuda.synchronize()
        Y.zero_()
        g.launch()
        torch.cuda.synchronize()
        want = fac.apply(X, inverse=inverse)
        torch.cuda.synchronize()
        _say(f"[graph] {name} replay {rep}: max |diff| {(Y - want).abs().max().item()}")
        assert torch.equal(Y, want)
    g.close()


def test_graph_refuses_stale_inverse_and_destroyed_handle():
    from paper_1507_04396_amd import MMFError
    A = workloads.small_grid((20, 20), sigma=0.5, shift=0.3, seed=2)
    ref = oracle.factor(A, k=2, core=24, cluster=(16, 64), seed=3)
    fac = import_oracle(ref)
    X = torch.ones(A.n, 8, device="cuda")
    Yf, Yi = torch.empty_like(X), torch.empty_like(X)
    gf = fac.capture(X, Yf, inverse=False)
    gi = fac.capture(X, Yi, inverse=True)
    theta, hdiag, hcore = fac.params()
    fac.set_params(hdiag=hdiag * 2.0)
    gf.launch()  # the forward product reads the handle's current H
    torch.cuda.synchronize()
    assert torch.equal(Yf, fac.apply(X))
    with pytest.raises(MMFError) as e:
        gi.launch()
    assert e.value.name == "MMF_ESTATE"
    fac.close()
    with pytest.raises(MMFError) as e:
        gf.launch()
    assert e.value.name == "MMF_ESTATE"
    gf.close()
    gi.close()
