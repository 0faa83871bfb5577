"""Data-driven clustering (MMF_CUT_CLUSTERS, reading R16) on the GPU against the FP64 oracle: the
boundary counts and the dynamic program give the same clusters in every stage, and the
factorization then matches the oracle's under the usual parity rules."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from helpers import check_factor_parity

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
    ("grid24x24", lambda: workloads.small_grid((24, 24), seed=3),
     dict(k=2, eta=0.5, core=40, cluster=(32, 96), seed=5)),
    ("knn2d_n700_k3", lambda: workloads.knn_points_matrix(700, 2, 8, 0.01, 4),
     dict(k=3, eta=0.5, core=50, cluster=(40, 120), seed=1)),
    ("grid_ragged_n257", lambda: workloads.small_grid((1, 257), seed=4),
     dict(k=2, eta=0.5, core=3, cluster=(5, 17), seed=4)),
]


@pytest.mark.parametrize("name,make,params", CASES, ids=[c[0] for c in CASES])
def test_cut_clusters_match_oracle(name, make, params):
    from paper_1507_04396_amd.api import Factorization
    A = make()
    _say(f"[cut] {name}: gpu factor n={A.n} params={params}")
    fac = Factorization.from_csr(A, cut_clusters=True, **params)
    ref = check_factor_parity(A, dict(params, cut_clusters=True), fac, name, say=_say)
    st = fac.stage_info()
    assert [s["clusters"] for s in st] == [len(s["cluster_sizes"]) for s in ref.stages]
    seeded = oracle.factor(A, **params)
    _say(f"[cut] {name}: loss cut {ref.loss:.6g}, seeded {seeded.loss:.6g}")


def test_cut_clusters_reject_even_flag():
    from paper_1507_04396_amd._lib import MMFError
    from paper_1507_04396_amd.api import Factorization
    A = workloads.small_grid((10, 10), seed=1)
    with pytest.raises(MMFError):
        Factorization.from_csr(A, k=2, core=10, cluster=(8, 24), seed=0, cut_clusters=True,
                               even_clusters=True)
