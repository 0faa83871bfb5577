"""Pins of the data-driven clustering (reading R16): boundary cut counts against closed forms and
the cut-minimizing partition against brute-force enumeration of every partition."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads


def _sym(n, density, seed):
    rng = np.random.default_rng(seed)
    a = sp.random(n, n, density=density, random_state=rng, format="csr")
    a = a + a.T + sp.eye(n)
    return sp.csr_matrix(a)


def test_boundary_cuts_closed_forms():
    # a path graph cuts one entry at every interior boundary
    n = 9
    path = sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
    assert oracle.boundary_cuts(path).tolist() == [0] + [1] * (n - 1) + [0]
    # the cuts add up to the total span sum over entries i < j
    a = _sym(30, 0.15, 1)
    coo = a.tocoo()
    up = coo.row < coo.col
    assert oracle.boundary_cuts(a).sum() == int((coo.col[up] - coo.row[up]).sum())
    # a block-diagonal matrix has no cut at its block boundaries
    b = sp.block_diag([np.ones((3, 3)), np.ones((4, 4))], format="csr")
    w = oracle.boundary_cuts(b)
    assert w[3] == 0 and w[0] == 0 and w[7] == 0 and (w[1:3] > 0).all() and (w[4:7] > 0).all()


def _brute(a, lo, hi):
    """Every composition of S into parts in [lo, hi]: least total cut, ties to the sizes that read
    backwards largest (lexicographically)."""
    S = a.shape[0]
    coo = a.tocoo()
    edges = [(i, j) for i, j in zip(coo.row, coo.col) if i < j]
    best = None
    def parts(r):
        if r == 0:
            yield []
            return
        for s in range(lo, min(hi, r) + 1):
            for rest in parts(r - s):
                yield [s] + rest
    for sizes in parts(S):
        bounds = set(itertools.accumulate(sizes[:-1]))
        cut = sum(1 for i, j in edges for b in bounds if i < b <= j)
        key = (cut, [-x for x in reversed(sizes)])
        if best is None or key < best[0]:
            best = (key, sizes)
    return best[1]


@pytest.mark.parametrize("n,lo,hi,seed", [(12, 2, 4, 0), (13, 2, 5, 1), (14, 3, 6, 2), (11, 2, 4, 3)])
def test_cut_sizes_match_brute_force(n, lo, hi, seed):
    a = _sym(n, 0.25, seed)
    assert oracle.cut_cluster_sizes(a, lo, hi) == _brute(a, lo, hi)


def test_cut_sizes_follow_block_structure():
    b = sp.block_diag([np.ones((3, 3)), np.ones((4, 4)), np.ones((3, 3))], format="csr")
    assert oracle.cut_cluster_sizes(b, 2, 4) == [3, 4, 3]


def test_cut_sizes_small_stage_and_bounds():
    a = _sym(8, 0.3, 4)
    assert oracle.cut_cluster_sizes(a, 2, 8) == [8]     # at most hi: one cluster
    assert oracle.cut_cluster_sizes(a, 0, 0) == [8]
    with pytest.raises(ValueError):
        oracle.cut_cluster_sizes(a, 3, 5)


def test_cut_factorization_runs_and_is_valid():
    A = workloads.knn_points_matrix(400, 2, 8, 0.01, 3)
    f = oracle.factor(A, k=2, core=40, cluster=(32, 96), seed=0, cut_clusters=True)
    for st in f.stages:
        sizes = st["cluster_sizes"]
        assert sum(sizes) == st["size"]
        assert all(32 <= c <= 96 for c in sizes) or len(sizes) == 1
    # the exact residual equals the product's distance to A (R12)
    Ad = A.to_scipy().toarray()
    resid = float(((Ad - oracle.dense_reconstruction(f)) ** 2).sum())
    assert f.loss == pytest.approx(resid, rel=1e-9, abs=1e-9)
