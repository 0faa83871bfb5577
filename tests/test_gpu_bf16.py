"""BF16 form of the cluster Gram (gram_mode 1) against the FP64 oracle.

The BF16 Gram only shortlists partners; the pick and G[T,T] come from exact FP32 dots of the
slab columns, which every rotation right-rotates.  So the decisions follow the same rule as the
FP32 path, and the same replay check applies: every decision that is not a near-tie equals the
oracle's, then rotation blocks, H and the loss are compared.
"""
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
    ("knn2d_n512", lambda: workloads.make_matrix("knn2d_n512"),
     dict(workloads.WORKLOADS["knn2d_n512"]["params"])),
    ("grid24x24_clusters", lambda: workloads.small_grid((24, 24), seed=3),
     dict(k=2, eta=0.5, core=40, cluster=(32, 96), seed=5)),
    ("knn3d_n1500_k3", lambda: workloads.knn_points_matrix(1500, 3, 10, 0.01, 6),
     dict(k=3, eta=0.5, core=64, cluster=(64, 256), seed=2)),
]


@pytest.mark.parametrize("name,make,params", CASES, ids=[c[0] for c in CASES])
def test_bf16_form_matches_oracle(name, make, params):
    from paper_1507_04396_amd.api import Factorization
    A = make()
    _say(f"[bf16] {name}: gpu gram_mode 1")
    fac = Factorization.from_csr(A, gram_mode=1, **params)
    inf = fac.info()
    stg = fac.stage_info()
    assert all(st["dense_gram"] == 1 for st in stg)
    cut = sum(st["bf16_long"] for st in stg)
    scored = sum(st["bf16_rescored"] for st in stg)
    R = inf["num_rotations"]
    _say(f"[bf16] {name}: {scored} candidates rescored over {R} steps, {cut} long shortlists")
    assert scored >= R * (params["k"] - 1)
    check_factor_parity(A, dict(params), fac, f"bf16 {name}", say=_say)


def test_bf16_form_full_grid_close_to_fp32_form():
    from paper_1507_04396_amd.api import Factorization
    A = workloads.make_matrix("grid2d_n65536")
    prm = dict(workloads.WORKLOADS["grid2d_n65536"]["params"])
    _say("[bf16] grid2d_n65536: FP32 and BF16 forms")
    f32 = Factorization.from_csr(A, **prm).info()
    fb = Factorization.from_csr(A, gram_mode=1, **prm)
    bf = fb.info()
    stg = fb.stage_info()
    _say(f"[bf16] loss fp32 {f32['loss']:.8g} bf16 {bf['loss']:.8g}; "
         f"long shortlists {sum(s['bf16_long'] for s in stg)} of {bf['num_rotations']} steps")
    assert bf["num_rotations"] == f32["num_rotations"]
    assert abs(bf["loss"] - f32["loss"]) <= 1e-3 * f32["loss"]
