"""Seeded synthetic inputs shaped like the workloads the pMMF paper factors.

The paper times pMMF on Laplacians of sparse, bounded-degree graphs (Sec. 2.4, Fig. 2) and
preconditions sparse SPD systems (Sec. 4); its datasets are not available, so these generators
build graph Laplacians of the same kind from a seeded ``numpy.random.Generator(PCG64)``.

This module holds none of the factorization's arithmetic.  Both the FP64 oracle and the HIP
library consume what it returns: values are formed in FP64 and rounded once to FP32, and the
oracle upcasts those FP32 values exactly.

Matrices are returned as 0-based CSR with ``int64`` row pointers, ``int32`` column indices and
``float32`` values, both triangles present, columns ascending within each row.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.spatial


@dataclasses.dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int64 [n+1]
    colind: np.ndarray  # int32 [nnz]
    val: np.ndarray     # float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self, dtype=np.float64) -> sp.csr_matrix:
        return sp.csr_matrix((self.val.astype(dtype), self.colind, self.rowptr),
                             shape=(self.n, self.n))

    def to_dense(self, dtype=np.float64) -> np.ndarray:
        return self.to_scipy(dtype).toarray()


def _csr_from_scipy(m: sp.spmatrix) -> CSR:
    m = sp.csr_matrix(m)
    m.sum_duplicates()
    m.sort_indices()
    return CSR(n=m.shape[0], rowptr=m.indptr.astype(np.int64),
               colind=m.indices.astype(np.int32), val=m.data.astype(np.float32))


def csr_from_dense(a: np.ndarray) -> CSR:
    """CSR of a dense symmetric matrix (zeros dropped); values rounded to FP32."""
    return _csr_from_scipy(sp.csr_matrix(np.asarray(a, dtype=np.float32)))


# --------------------------------------------------------------------------- locality order

def _spread_bits(v: np.ndarray, bits: int, stride: int) -> np.ndarray:
    out = np.zeros_like(v, dtype=np.uint64)
    v = v.astype(np.uint64)
    for b in range(bits):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * stride)
    return out


def morton_order(points: np.ndarray) -> np.ndarray:
    """Permutation sorting points in [0,1]^d (d = 2 or 3) by a 30-bit Morton code.

    Contiguous runs of this order are compact regions of space, which is the locality the
    clustering step relies on.  Equal codes keep their original order (stable sort).
    """
    d = points.shape[1]
    bits = 30 // d
    q = np.clip((points * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(points.shape[0], dtype=np.uint64)
    for a in range(d):
        code |= _spread_bits(q[:, a], bits, d) << np.uint64(a)
    return np.argsort(code, kind="stable")


# --------------------------------------------------------------------------- graphs

def knn_normalized_laplacian(points: np.ndarray, knn: int, sigma2: float) -> CSR:
    """Symmetric normalized Laplacian I - D^-1/2 W D^-1/2 of an exact kNN graph.

    Edges join each point to its ``knn`` nearest neighbours (self excluded); the edge set is the
    union over both directions, with Gaussian weights exp(-d^2 / sigma2).
    """
    n = points.shape[0]
    tree = scipy.spatial.cKDTree(points)
    dist, idx = tree.query(points, k=knn + 1)
    rows = np.repeat(np.arange(n), knn + 1)
    cols = idx.reshape(-1)
    d2 = dist.reshape(-1).astype(np.float64) ** 2
    keep = cols != rows
    rows, cols, d2 = rows[keep], cols[keep], d2[keep]
    w = np.exp(-d2 / sigma2)
    W = sp.coo_matrix((w, (rows, cols)), shape=(n, n)).tocsr()
    W = W.maximum(W.T)  # union symmetrization; both directions carry the same weight
    deg = np.asarray(W.sum(axis=1)).ravel()
    inv_sqrt = 1.0 / np.sqrt(deg)
    W = W.tocoo()
    off = -W.data * inv_sqrt[W.row] * inv_sqrt[W.col]
    L = sp.coo_matrix((np.concatenate([off, np.ones(n)]),
                       (np.concatenate([W.row, np.arange(n)]),
                        np.concatenate([W.col, np.arange(n)]))), shape=(n, n))
    return _csr_from_scipy(_symmetrize_exact(L.tocsr()))


def _symmetrize_exact(m: sp.csr_matrix) -> sp.csr_matrix:
    """Make the FP64 pattern and values exactly symmetric before the single FP32 rounding."""
    up = sp.triu(m, k=1)
    return (up + up.T + sp.diags(m.diagonal())).tocsr()


def grid_laplacian(shape: tuple, sigma: float, shift: float, rng: np.random.Generator) -> CSR:
    """Combinatorial Laplacian D - W + shift*I of a 2D (4-point) or 3D (7-point) grid.

    Vertices are numbered lexicographically (last axis fastest).  Edge weights are iid
    LogNormal(0, sigma), drawn axis by axis (axis 0 edges first), each in lexicographic order of
    the lower endpoint.
    """
    dims = tuple(int(d) for d in shape)
    n = int(np.prod(dims))
    ids = np.arange(n).reshape(dims)
    rows, cols, ws = [], [], []
    for ax in range(len(dims)):
        lo = [slice(None)] * len(dims)
        hi = [slice(None)] * len(dims)
        lo[ax] = slice(0, dims[ax] - 1)
        hi[ax] = slice(1, dims[ax])
        a = ids[tuple(lo)].ravel()
        b = ids[tuple(hi)].ravel()
        w = rng.lognormal(mean=0.0, sigma=sigma, size=a.size)
        rows.append(a)
        cols.append(b)
        ws.append(w)
    a = np.concatenate(rows)
    b = np.concatenate(cols)
    w = np.concatenate(ws)
    W = sp.coo_matrix((w, (a, b)), shape=(n, n)).tocsr()
    W = W + W.T
    deg = np.asarray(W.sum(axis=1)).ravel()
    L = sp.diags(deg + shift) - W
    return _csr_from_scipy(_symmetrize_exact(L.tocsr()))


# --------------------------------------------------------------------------- named workloads

# Factorization parameters: k = rotation order, eta = fraction of the active set retired per
# stage, core = size of the dense core, cluster = (lo, hi) bounds of the random uneven cluster
# sizes ((0, 0) means one cluster per stage, i.e. plain MMF), seed = algorithm seed.
WORKLOADS = {
    "knn2d_n512": dict(kind="knn", n=512, dim=2, knn=8, sigma2=0.01,
                       params=dict(k=2, eta=0.5, core=64, cluster=(0, 0), seed=0)),
    "grid2d_n65536": dict(kind="grid", shape=(256, 256), sigma=1.0, shift=0.0,
                          params=dict(k=2, eta=0.5, core=512, cluster=(256, 2048), seed=0)),
    "knn3d_n262144": dict(kind="knn", n=262144, dim=3, knn=10, sigma2=0.01,
                          params=dict(k=3, eta=0.5, core=1024, cluster=(512, 2048), seed=0)),
    "grid3d_n1050703": dict(kind="grid", shape=(101, 101, 103), sigma=1.5, shift=1e-2,
                            params=dict(k=2, eta=0.5, core=1024, cluster=(512, 2048), seed=0)),
}


def make_matrix(name: str, data_seed: int = 0) -> CSR:
    """The workload's matrix, generated from ``PCG64(data_seed)``."""
    w = WORKLOADS[name]
    rng = np.random.Generator(np.random.PCG64(data_seed))
    if w["kind"] == "knn":
        pts = rng.random((w["n"], w["dim"]))
        pts = pts[morton_order(pts)]
        return knn_normalized_laplacian(pts, w["knn"], w["sigma2"])
    return grid_laplacian(w["shape"], w["sigma"], w["shift"], rng)


def knn_points_matrix(n: int, dim: int, knn: int, sigma2: float, seed: int) -> CSR:
    """kNN normalized Laplacian on ``n`` Morton-sorted uniform points (any size, for tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, dim))
    pts = pts[morton_order(pts)]
    return knn_normalized_laplacian(pts, knn, sigma2)


def small_grid(shape: tuple, sigma: float = 1.0, shift: float = 0.0, seed: int = 0) -> CSR:
    rng = np.random.Generator(np.random.PCG64(seed))
    return grid_laplacian(shape, sigma, shift, rng)


def gaussian_block(n: int, ncols: int, seed: int) -> np.ndarray:
    """Row-major ``[n][ncols]`` FP32 block of iid N(0,1) values (right-hand sides, probes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n, ncols)).astype(np.float32)


def rbf_kernel_matrix(n: int, dim: int, gamma: float, seed: int) -> CSR:
    """Dense Gaussian kernel matrix exp(-gamma |x_i - x_j|^2) on ``n`` Morton-sorted uniform points
    in [0,1]^dim, stored as CSR with every entry (the kernel-matrix workload of the compression
    curve)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, dim))
    pts = pts[morton_order(pts)]
    d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    k = np.exp(-gamma * d2)
    return csr_from_dense(0.5 * (k + k.T))


def random_symmetric(n: int, density: float, seed: int, diag_shift: float = 0.0) -> CSR:
    """Random sparse symmetric matrix with N(0,1) entries (edge and special-case tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    a = np.triu(a, 1)
    a = a + a.T + np.diag(rng.standard_normal(n) + diag_shift)
    return csr_from_dense(a)


def block_diag_pairs(n: int, seed: int, permute: bool = True):
    """Symmetric matrix that is block diagonal in 2x2 blocks, under a random permutation.

    Each block's two eigenvalues have distinct absolute values, so its Gram block has a nonzero
    off-diagonal entry.  Returns (matrix, perm) where the block pairs are (perm[2q], perm[2q+1]).
    """
    assert n % 2 == 0
    rng = np.random.Generator(np.random.PCG64(seed))
    a = np.zeros((n, n))
    perm = rng.permutation(n) if permute else np.arange(n)
    for q in range(n // 2):
        i, j = perm[2 * q], perm[2 * q + 1]
        l1 = rng.uniform(1.0, 2.0)
        l2 = rng.uniform(2.5, 4.0) * (1 if rng.random() < 0.5 else -1)
        th = rng.uniform(0.1, 1.4)
        c, s = np.cos(th), np.sin(th)
        R = np.array([[c, -s], [s, c]])
        B = R @ np.diag([l1, l2]) @ R.T
        B = (B + B.T) / 2
        a[i, i], a[i, j], a[j, i], a[j, j] = B[0, 0], B[0, 1], B[1, 0], B[1, 1]
    return csr_from_dense(a), perm
