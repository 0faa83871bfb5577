"""Plain FP64 reference implementation of pMMF (Kondor, Teneva & Mudrakarta, "Parallel MMF").

TEST INFRASTRUCTURE ONLY.  This module is the oracle the HIP library is checked against.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it; the library never does,
and this module imports nothing from the library.

Everything here runs on the CPU in float64 (NumPy/SciPy), one step at a time, in the order the
paper gives: Algorithm 1 (stages: cluster, reblock, find rotations per cluster, rotate the whole
matrix from both sides, merge) with Algorithm 2 (randomized greedy search inside a cluster) inside
it.  Inputs are the FP32 values of the test matrix, upcast exactly.

Readings of points the paper leaves open (each is also listed in the design notes):
  R1  Givens sign (Sec. 2, item 1 is garbled): Q_ii = cos, Q_ij = -sin, Q_ji = sin, Q_jj = cos.
  R2  Partner score (Sec. 2.2 and Alg. 2): |<A_:i, A_:j>| / ||A_:j||, i.e. |G_ij| / sqrt(G_jj);
      a zero column scores 0; ties go to the lower local index.
  R3  k > 2: the objective is separable, so the k-1 partners are the top k-1 single scores;
      slot order is (seed, partners by descending score).
  R4  The cluster Gram runs over the rows active at the start of the stage (S_{p-1}); rows retired
      in earlier stages are peeled into H.  Inside a stage the Gram is only rotated (Eq. for the
      Gram recursion in Sec. 2), never downdated.
  R5  Elimination (Sec. 2.2, Alg. 2): off-diagonal column norm off^2_t = max(0, G_tt - D_tt^2)
      with D the cluster's diagonal block; retire the argmin, ties to the later slot (the
      paper's strict '<').
  R6  Rotation from the k x k Gram block (Sec. 2.2): k = 2 uses the symmetric Schur / Jacobi
      rotation with |theta| <= pi/4 (O = I when G_ij = 0); k = 3 takes the eigenvectors in
      descending eigenvalue order as rows, then the row permutation and signs that maximize
      trace(O) with O_rr >= 0 (ties: lexicographically smallest permutation).
  R7  One index retired per rotation (Sec. 2, item 2, simplest case).
  R8  eta is the fraction of the active set retired per stage: t_p = min(|S|-core, floor(eta|S|));
      cluster u gets floor(t_p c_u / |S|) rotations plus one of the leftovers by largest
      remainder (ties to the lower u).
  R9  The uniformly random seed index (Alg. 2) is I[mulhi(h, |I|)] with h a SplitMix64 chain of
      (seed, tag=1, p, u, s) and I in ascending order.
  R10 Clustering (Alg. 1 "cluster"): contiguous chunks of the ascending active list with seeded
      sizes in [lo, hi] (tag 2); (0, 0) means one cluster per stage (plain MMF).
  R11 H (Alg. 1 output): retired index e keeps its diagonal entry at retirement; the core is the
      remaining active block of the final matrix.
  R12 Loss: the exact residual ||A - U^T H U||_F^2 equals 2 * sum_e m_e, where m_e is the squared
      mass of row e over the indices still active just after e retires; the literal per-retirement
      sum of 2 off^2_e is an upper bound and is reported beside it.
  R13 Decision margins (not part of the factorization): the seed-partner score gap relative to
      sqrt(G_ii) (the Cauchy-Schwarz bound of every score), the k = 2 angle-branch switch as
      |G_jj - G_ii| / (|G_ii| + |G_jj| + 2|G_ij|), the k = 3 eigengap and trace gap, and the
      elimination gap relative to max_t G_tt.  A margin below 1e-5 marks a step where two
      choices are equally correct at working precision.
  R15 Angles of a 3-point rotation (the paper parametrizes only Givens rotations by an angle):
      O(w) = expm(w_0 G_01 + w_1 G_02 + w_2 G_12) O0, with O0 the rotation the search found and
      G_pq = E_qp - E_pq the generator of the (p, q) plane in slot order (G_01 extends the Givens
      J = [[0, -1], [1, 0]]); w = 0 at the start.
  R16 A data-driven clustering (optional, Alg. 1 "cluster"): clusters stay contiguous chunks of
      the active list, with sizes in [lo, hi], but their boundaries are chosen to cut the fewest
      entries of the active matrix: boundary b (between positions b-1 and b) cuts the entries
      (i, j), i < j, with i < b <= j, and the chosen boundaries minimize the total count.  Among
      optimal partitions the one whose cluster sizes, read from the last cluster backwards, are
      lexicographically largest is taken.  A stage with at most hi active indices is one cluster.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp

MASK64 = (1 << 64) - 1
GOLDEN64 = 0x9E3779B97F4A7C15
TAG_SEED_ROW = 1
TAG_CLUSTER_SIZE = 2


# --------------------------------------------------------------------------- counter-based RNG

def mix64(z: int) -> int:
    """SplitMix64 output finalizer (Steele, Lea & Flood, OOPSLA 2014), on Python ints mod 2^64."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def chain_hash(seed: int, *vals: int) -> int:
    """x <- mix64((x xor v) + golden) over the values, starting from x = seed."""
    x = seed & MASK64
    for v in vals:
        x = mix64(((x ^ (v & MASK64)) + GOLDEN64) & MASK64)
    return x


def mulhi(x: int, n: int) -> int:
    """floor(x * n / 2^64): maps a 64-bit hash to [0, n) (Lemire's multiply-shift)."""
    return (x * n) >> 64


# --------------------------------------------------------------------------- schedule (R8, R10)

def stage_schedule(n: int, core: int, eta: float) -> List[tuple]:
    """[(|S_{p-1}|, t_p)] for p = 1..P: the active-set sizes and rotations per stage."""
    if not (1 <= core <= n):
        raise ValueError("core size must be in [1, n]")
    if not (0.0 < eta <= 0.5):
        raise ValueError("eta must be in (0, 0.5]")
    out = []
    s = n
    while s > core:
        t = min(s - core, int(math.floor(eta * s)))
        if t < 1:
            raise ValueError("eta * |S| < 1: the schedule cannot reach the core")
        out.append((s, t))
        s -= t
    return out


def cluster_sizes(total: int, lo: int, hi: int, seed: int, p: int, even: bool = False) -> List[int]:
    """Sizes of the contiguous clusters of a stage with ``total`` active indices (R10)."""
    if lo == 0 and hi == 0:
        return [total]
    if lo < 2 or hi < 2 * lo:
        raise ValueError("cluster bounds need lo >= 2 and hi >= 2*lo")
    sizes = []
    r = total
    q = 0
    while r > hi:
        s = lo + mulhi(chain_hash(seed, TAG_CLUSTER_SIZE, p, q, 0), hi - lo + 1)
        s = min(s, r - lo)
        if even:
            s -= s % 2
        sizes.append(s)
        r -= s
        q += 1
    sizes.append(r)
    return sizes


def boundary_cuts(M) -> np.ndarray:
    """w[b] for b = 0..S: the number of entries (i, j), i < j, of the symmetric active matrix M
    with i < b <= j, i.e. the entries a cluster boundary at b separates (R16).  w[0] = w[S] = 0."""
    M = sp.csr_matrix(M)
    S = M.shape[0]
    coo = M.tocoo()
    upper = coo.row < coo.col
    w = np.zeros(S + 1, dtype=np.int64)
    for i, j in zip(coo.row[upper], coo.col[upper]):
        w[i + 1:j + 1] += 1
    return w


def cut_cluster_sizes(M, lo: int, hi: int) -> List[int]:
    """Contiguous cluster sizes in [lo, hi] whose boundaries cut the fewest entries of M (R16).

    f[b] is the least total cut of a partition of positions [0, b) into clusters, counting the
    boundary at b itself (for b < S); the last cluster of an optimal partition of [0, b) starts at
    the smallest optimal predecessor, which makes the sizes read backwards lexicographically
    largest."""
    S = sp.csr_matrix(M).shape[0]
    if lo == 0 and hi == 0:
        return [S]
    if lo < 2 or hi < 2 * lo:
        raise ValueError("cluster bounds need lo >= 2 and hi >= 2*lo")
    if S <= hi:
        return [S]
    w = boundary_cuts(M)
    INF = None
    f: List[Optional[int]] = [INF] * (S + 1)
    back = [-1] * (S + 1)
    f[0] = 0
    for b in range(lo, S + 1):
        best, arg = INF, -1
        for prev in range(max(0, b - hi), b - lo + 1):   # ascending: ties keep the smallest
            if f[prev] is not INF and (best is INF or f[prev] < best):
                best, arg = f[prev], prev
        if best is not INF:
            f[b] = best + (int(w[b]) if b < S else 0)
            back[b] = arg
    sizes = []
    b = S
    while b > 0:
        sizes.append(b - back[b])
        b = back[b]
    return sizes[::-1]


def allocate_rotations(t: int, sizes: List[int]) -> List[int]:
    """Rotations per cluster: floor(t c_u / |S|) plus leftovers by largest remainder (R8)."""
    total = sum(sizes)
    base = [(t * c) // total for c in sizes]
    rem = [(t * c) % total for c in sizes]
    left = t - sum(base)
    order = sorted(range(len(sizes)), key=lambda u: (-rem[u], u))
    for u in order[:left]:
        base[u] += 1
    return base


# --------------------------------------------------------------------------- rotations (R6)

def rotation_k2(g: np.ndarray):
    """2x2 rotation O = [[c, -s], [s, c]] with O g O^T diagonal and |theta| <= pi/4.

    The symmetric Schur decomposition of a 2x2 block (Golub & Van Loan, Alg. 8.4.1), with the
    smaller-magnitude root of t^2 + 2 tau t - 1 = 0.  Returns (O, |tau|); |tau| -> 0 is where the
    choice of root switches sign.
    """
    a, b, d = float(g[0, 0]), float(g[0, 1]), float(g[1, 1])
    if b == 0.0:
        return np.eye(2), math.inf
    tau = (d - a) / (2.0 * b)
    sgn = 1.0 if tau >= 0.0 else -1.0
    t = sgn / (abs(tau) + math.hypot(1.0, tau))
    c = 1.0 / math.sqrt(1.0 + t * t)
    s = t * c
    return np.array([[c, -s], [s, c]]), abs(tau)


def rotation_k3(g: np.ndarray):
    """k x k orthogonal O whose rows are eigenvectors of g, arranged closest to the identity.

    Rows are eigenvectors in descending eigenvalue order (LAPACK), then permuted and signed to
    maximize trace(O) with nonnegative diagonal; ties go to the lexicographically smallest
    permutation.  Returns (O, relative margin between the best and second-best trace).
    """
    kk = g.shape[0]
    w, v = np.linalg.eigh(g)
    base = v[:, ::-1].T  # row r = eigenvector of the r-th largest eigenvalue
    traces = []
    for perm in itertools.permutations(range(kk)):
        traces.append((sum(abs(base[perm[r], r]) for r in range(kk)), perm))
    best = max(tr for tr, _ in traces)
    perm = min(pm for tr, pm in traces if tr == best)
    others = sorted((tr for tr, pm in traces if pm != perm), reverse=True)
    margin = (best - others[0]) / best if best > 0 else 0.0
    O = np.empty((kk, kk))
    for r in range(kk):
        row = base[perm[r]]
        O[r] = row if row[r] >= 0.0 else -row
    return O, margin


# --------------------------------------------------------------------------- factorization

@dataclasses.dataclass
class Rotation:
    stage: int               # p, 1-based
    cluster: int             # u, 0-based within the stage
    step: int                # s, 0-based within the cluster
    ids: np.ndarray          # global indices (i_1..i_k), slot order
    O: np.ndarray            # k x k block: x[ids] <- O @ x[ids]
    retired: int             # global index eliminated after this rotation
    seed_pos: int            # local position of the seed row inside the cluster
    margin: float            # smallest relative decision margin of the step (R13 in the notes)


@dataclasses.dataclass
class Factorization:
    n: int
    k: int
    rotations: List[Rotation]
    stages: List[dict]       # per stage: active ids, cluster offsets, rotations per cluster, stats
    hdiag: np.ndarray        # float64[n]; retired entries of H's diagonal (0 on core indices)
    core_ids: np.ndarray     # ascending global ids of the core
    hcore: np.ndarray        # float64[core, core]
    loss: float              # exact residual 2 * sum_e m_e
    loss_literal: float      # sum of 2 * off^2 at retirement (upper bound)
    retired_order: np.ndarray  # global ids in retirement order (stage, cluster, step)

    @property
    def num_stages(self) -> int:
        return len(self.stages)


def _as_csr64(A) -> sp.csr_matrix:
    if hasattr(A, "rowptr"):
        A = A.to_scipy(np.float64)
    if sp.issparse(A):
        m = sp.csr_matrix(A, dtype=np.float64)
    else:
        m = sp.csr_matrix(np.asarray(A, dtype=np.float64))
    m.sum_duplicates()
    m.sort_indices()
    return m


def factor(A, k: int = 2, eta: float = 0.5, core: int = 64, cluster=(0, 0), seed: int = 0,
           even_clusters: bool = False, cut_clusters: bool = False,
           on_step: Optional[Callable[[dict], None]] = None) -> Factorization:
    """pMMF factorization A ~ U^T H U (Eq. 1 / Eq. 4) by Algorithm 1 with Algorithm 2 inside.

    ``A`` is symmetric (a CSR from ``workloads``, a SciPy sparse matrix or a dense array).
    ``on_step`` (tests only) receives the cluster's state after every rotation.
    """
    if k not in (2, 3):
        raise ValueError("k must be 2 or 3")
    M = _as_csr64(A)
    n = M.shape[0]
    if (abs(M - M.T) > 0).nnz:
        raise ValueError("matrix is not symmetric")
    lo, hi = cluster
    schedule = stage_schedule(n, core, eta)
    S = np.arange(n)                    # global ids of the active positions, ascending
    hdiag = np.zeros(n)
    rotations: List[Rotation] = []
    stages = []
    retired_order = []
    loss = 0.0
    loss_literal = 0.0

    for p, (size, t) in enumerate(schedule, start=1):
        assert size == len(S)
        if cut_clusters:                 # R16
            if even_clusters:
                raise ValueError("even and cut clusters exclude each other")
            sizes = cut_cluster_sizes(M, lo, hi)
        else:
            sizes = cluster_sizes(size, lo, hi, seed, p, even=even_clusters)
        r_u = allocate_rotations(t, sizes)
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        nnz_start = M.nnz
        fro_start = math.sqrt((M.data ** 2).sum())
        q_blocks = []
        retired_pos = []                # compact positions retired in this stage, in order
        Mc = M.tocsc()

        for u, c in enumerate(sizes):
            off = int(offsets[u])
            slab = Mc[:, off:off + c]                            # rows: all of S_{p-1} (R4)
            G = (slab.T @ slab).toarray()                        # local Gram, Sec. 2.1
            D = M[off:off + c, off:off + c].toarray()            # diagonal block [[A]]_{u,u}
            Qu = np.eye(c)
            active = np.ones(c, dtype=bool)                      # I = [c]
            for s in range(r_u[u]):
                live = np.flatnonzero(active)
                i = int(live[mulhi(chain_hash(seed, TAG_SEED_ROW, p, u, s), live.size)])
                kk = k if live.size >= k else 2
                # normalized inner products with the seed column, in absolute value (R2)
                gdiag = np.diag(G)
                score = np.zeros(c)
                pos = gdiag > 0.0
                score[pos] = np.abs(G[i, pos]) / np.sqrt(gdiag[pos])
                cand = live[live != i]
                order = cand[np.lexsort((cand, -score[cand]))]  # descending score, then lower j
                partners = [int(j) for j in order[:kk - 1]]
                T = [i] + partners
                # decision margins (R13): each gap is measured against the scale at which the
                # compared quantities are formed, so a small margin flags a numerical tie
                margins = []
                if order.size >= kk:
                    s_in, s_out = score[order[kk - 2]], score[order[kk - 1]]
                    bound = math.sqrt(G[i, i]) if G[i, i] > 0 else 0.0   # Cauchy-Schwarz
                    margins.append((s_in - s_out) / bound if bound > 0 else 0.0)
                # rotation that diagonalizes the k x k Gram block (R6)
                gTT = G[np.ix_(T, T)]
                if kk == 2:
                    O, _ = rotation_k2(gTT)
                    a_, b_, d_ = gTT[0, 0], gTT[0, 1], gTT[1, 1]
                    den = abs(a_) + abs(d_) + 2.0 * abs(b_)
                    margins.append(abs(d_ - a_) / den if (den > 0 and b_ != 0.0) else math.inf)
                else:
                    O, tr_margin = rotation_k3(gTT)
                    margins.append(tr_margin)
                # G <- O G O^T and the same for the diagonal block and the accumulated Q (Alg. 2)
                G[T, :] = O @ G[T, :]
                G[:, T] = G[:, T] @ O.T
                D[T, :] = O @ D[T, :]
                D[:, T] = D[:, T] @ O.T
                Qu[T, :] = O @ Qu[T, :]
                # eliminate the slot with the smallest off-diagonal norm, ties to the later (R5)
                off2 = [max(0.0, G[tt, tt] - D[tt, tt] ** 2) for tt in T]
                e_slot = 0
                for sl in range(1, kk):
                    if off2[sl] <= off2[e_slot]:
                        e_slot = sl
                srt = sorted(off2)
                gscale = max(G[tt, tt] for tt in T)   # off^2 = G_tt - D_tt^2 is formed at this scale
                margins.append((srt[1] - srt[0]) / gscale if gscale > 0 else 0.0)
                e = T[e_slot]
                active[e] = False
                gid_e = int(S[off + e])
                hdiag[gid_e] = D[e, e]
                loss_literal += 2.0 * off2[e_slot]
                retired_pos.append(off + e)
                retired_order.append(gid_e)
                rotations.append(Rotation(stage=p, cluster=u, step=s,
                                          ids=S[off + np.asarray(T)].copy(), O=O.copy(),
                                          retired=gid_e, seed_pos=i,
                                          margin=float(min(margins))))
                if on_step is not None:
                    on_step(dict(stage=p, cluster=u, step=s, G=G, D=D, T=list(T), O=O,
                                 e=e, active=active.copy(), offset=off, S=S.copy()))
            q_blocks.append(Qu)

        # rotate the whole (blocked) matrix from both sides with the stage's rotations (Alg. 1)
        Qbar = sp.block_diag([sp.csr_matrix(q) for q in q_blocks], format="csr")
        row_nnz_max = int(np.diff(M.indptr).max()) if M.nnz else 0
        QM = (Qbar @ M).tocsr()
        M = (QM @ Qbar.T).tocsr()
        qm_row_nnz_max = int(np.diff(QM.indptr).max()) if QM.nnz else 0
        M.eliminate_zeros()
        fro_end = math.sqrt((M.data ** 2).sum())
        # exact loss of this stage's retirements (R12) and peeling of the retired rows/columns
        R = np.asarray(retired_pos, dtype=np.int64)
        keep = np.ones(size, dtype=bool)
        keep[R] = False
        Sv = np.flatnonzero(keep)
        MR = M[R]
        m_rs = MR[:, Sv]
        m_rr = MR[:, R].tolil()
        m_rr.setdiag(0.0)                       # only e' != e enters the residual
        m_rr = m_rr.tocsr()
        stage_loss = 2.0 * float((m_rs.data ** 2).sum()) + float((m_rr.data ** 2).sum())
        loss += stage_loss
        hdiag_check = float(np.max(np.abs(M.diagonal()[R] - hdiag[S[R]]))) if R.size else 0.0
        stages.append(dict(stage=p, size=size, rotations=t, cluster_sizes=sizes,
                           cluster_rotations=r_u, offsets=offsets, active=S.copy(),
                           retired=S[R].copy(), nnz_start=nnz_start, fro_start=fro_start,
                           row_nnz_max=row_nnz_max, qm_row_nnz_max=qm_row_nnz_max,
                           full_row_nnz_max=int(np.diff(M.indptr).max()) if M.nnz else 0,
                           fro_end=fro_end, loss=stage_loss, hdiag_check=hdiag_check))
        M = M[Sv][:, Sv].tocsr()
        S = S[Sv]

    hcore = M.toarray()
    return Factorization(n=n, k=k, rotations=rotations, stages=stages, hdiag=hdiag,
                         core_ids=S.copy(), hcore=hcore, loss=loss, loss_literal=loss_literal,
                         retired_order=np.asarray(retired_order, dtype=np.int64))


# --------------------------------------------------------------------------- matrix-free use

def apply_U(fac: Factorization, X: np.ndarray) -> np.ndarray:
    """U X with U = Q_L ... Q_1: the rotations in the order they were found (Sec. 2.4)."""
    Z = np.array(X, dtype=np.float64, copy=True)
    for r in fac.rotations:
        Z[r.ids] = r.O @ Z[r.ids]
    return Z


def apply_Ut(fac: Factorization, X: np.ndarray) -> np.ndarray:
    """U^T X: transposed rotations in reverse order."""
    Z = np.array(X, dtype=np.float64, copy=True)
    for r in reversed(fac.rotations):
        Z[r.ids] = r.O.T @ Z[r.ids]
    return Z


def _apply_H(fac: Factorization, Z: np.ndarray, inverse: bool = False) -> np.ndarray:
    W = np.zeros_like(Z)
    core = fac.core_ids
    mask = np.ones(fac.n, dtype=bool)
    mask[core] = False
    if inverse:
        if np.any(fac.hdiag[mask] == 0.0):
            raise ZeroDivisionError("zero diagonal entry in H")
        W[mask] = Z[mask] / fac.hdiag[mask, None]
        chol = np.linalg.cholesky(fac.hcore)          # raises LinAlgError if not SPD
        y = np.linalg.solve(chol, Z[core])
        W[core] = np.linalg.solve(chol.T, y)
    else:
        W[mask] = Z[mask] * fac.hdiag[mask, None]
        W[core] = fac.hcore @ Z[core]
    return W


def apply(fac: Factorization, X: np.ndarray) -> np.ndarray:
    """Matrix-free product  A~ X = U^T H U X  (Sec. 2.4)."""
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    X2 = X[:, None] if squeeze else X
    Y = apply_Ut(fac, _apply_H(fac, apply_U(fac, X2)))
    return Y[:, 0] if squeeze else Y


def apply_inverse(fac: Factorization, X: np.ndarray) -> np.ndarray:
    """A~^{-1} X = U^T H^{-1} U X: reciprocal diagonal and inverted core (Sec. 2.4)."""
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    X2 = X[:, None] if squeeze else X
    Y = apply_Ut(fac, _apply_H(fac, apply_U(fac, X2), inverse=True))
    return Y[:, 0] if squeeze else Y


def apply_inverse_sqrt(fac: Factorization, X: np.ndarray) -> np.ndarray:
    """A~^{-1/2} X = U^T H^{-1/2} U X (Sec. 4, the xi = 1/2 power used for split-symmetric
    preconditioning): U is orthogonal, so A~^{-1/2} = U^T H^{-1/2} U with H^{-1/2} the retired
    diagonal to the power -1/2 and the core's inverse square root V diag(lambda^{-1/2}) V^T from
    LAPACK's symmetric eigendecomposition.  Requires H positive definite."""
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    X2 = X[:, None] if squeeze else X
    Z = apply_U(fac, X2)
    W = np.zeros_like(Z)
    core = fac.core_ids
    mask = np.ones(fac.n, dtype=bool)
    mask[core] = False
    if np.any(fac.hdiag[mask] <= 0.0):
        raise ValueError("H has a retired diagonal entry that is not positive")
    W[mask] = Z[mask] / np.sqrt(fac.hdiag[mask, None])
    if len(core):
        lam, V = np.linalg.eigh(0.5 * (fac.hcore + fac.hcore.T))
        if np.any(lam <= 0.0):
            raise ValueError("the core of H is not positive definite")
        W[core] = (V * (1.0 / np.sqrt(lam))) @ (V.T @ Z[core])
    Y = apply_Ut(fac, W)
    return Y[:, 0] if squeeze else Y


def dense_U(fac: Factorization) -> np.ndarray:
    return apply_U(fac, np.eye(fac.n))


def dense_H(fac: Factorization) -> np.ndarray:
    H = np.diag(fac.hdiag.copy())
    H[np.ix_(fac.core_ids, fac.core_ids)] = fac.hcore
    return H


def dense_reconstruction(fac: Factorization) -> np.ndarray:
    U = dense_U(fac)
    return U.T @ dense_H(fac) @ U


# --------------------------------------------------------------------------- adjoint

def rot3_generators():
    """G_01, G_02, G_12 (R15): G_pq = E_qp - E_pq, the generator of rotations in the (p, q)
    plane of a 3-point rotation's slots."""
    gens = []
    for p, q in ((0, 1), (0, 2), (1, 2)):
        G = np.zeros((3, 3))
        G[q, p], G[p, q] = 1.0, -1.0
        gens.append(G)
    return gens


def rot3_param_matrix(w) -> np.ndarray:
    """W(w) = w_0 G_01 + w_1 G_02 + w_2 G_12 (skew-symmetric)."""
    return sum(wm * G for wm, G in zip(w, rot3_generators()))


def rot3_param_jacobian(w) -> np.ndarray:
    """3x3 matrix B(w) with  d expm(W(w)) = W(B(w) dw) expm(W(w)): the left-trivialized
    derivative of the matrix exponential, dexp_W(X) = sum_{k>=0} ad_W^k(X) / (k+1)! with
    ad_W(X) = W X - X W, applied to each generator and read back in the generator basis."""
    W = rot3_param_matrix(w)
    gens = rot3_generators()
    B = np.zeros((3, 3))
    for m, G in enumerate(gens):
        term, total = G.copy(), G.copy()
        for k in range(1, 40):
            term = (W @ term - term @ W) / (k + 1)
            total = total + term
            if np.abs(term).max() < 1e-18:
                break
        # coordinates of the skew matrix `total` in (G_01, G_02, G_12): entries (1,0), (2,0), (2,1)
        B[:, m] = [total[1, 0], total[2, 0], total[2, 1]]
    return B


def with_params3(fac: Factorization, theta, hdiag=None, hcore=None) -> Factorization:
    """Copy of a k = 3 factorization with O_t = expm(W(theta_t)) O_t (R15): ``fac`` holds the
    rotations at theta = 0.  Steps with 2 indices use theta_t[0] as their Givens angle offset in
    the (0, 1) plane."""
    import scipy.linalg
    theta = np.asarray(theta, dtype=np.float64)
    rots = []
    for r, w in zip(fac.rotations, theta):
        if len(r.ids) == 2:
            c, sn = math.cos(w[0]), math.sin(w[0])
            O = np.array([[c, -sn], [sn, c]]) @ r.O
        else:
            O = scipy.linalg.expm(rot3_param_matrix(w)) @ r.O
        rots.append(dataclasses.replace(r, O=O))
    return dataclasses.replace(fac, rotations=rots,
                               hdiag=fac.hdiag if hdiag is None else hdiag,
                               hcore=fac.hcore if hcore is None else hcore)


def backward(fac: Factorization, X: np.ndarray, Ybar: np.ndarray, theta=None):
    """Adjoint of Y = U^T H U X with respect to X, H and the Givens angles.

    The angle of rotation t is theta_t with O_t = [[cos, -sin], [sin, cos]], so
    dO_t/dtheta_t = J O_t with J = [[0, -1], [1, 0]].  With a = U x and b = U ybar, and the
    adjoint states g_a = (Q_T..Q_{t+1})^T H a and g_b = (Q_T..Q_{t+1})^T H^T b, the angle
    gradient is  sum_rhs <g_a[T], J zy_t[T]> + <g_b[T], J zx_t[T]>,  where zx_t and zy_t are x and
    ybar after rotations 1..t.  States are recovered by undoing rotations, not stored.
    For k = 3 (R15) the plane generators G_01, G_02, G_12 take J's place, giving the derivatives
    l_t along exp(eps G_m) O_t; the gradient in the parameters w_t of O_t = expm(W(w_t)) O0_t is
    the chain rule through the derivative of the matrix exponential (``rot3_param_jacobian``),
    which is the identity at w = 0.  ``theta`` are the current parameters (k = 3: [R][3]; None
    means zero).
    Returns (xbar, hdiag_bar, hcore_bar, theta_bar); theta_bar is [R] for k = 2, [R][3] for k = 3.
    """
    X = np.asarray(X, dtype=np.float64)
    Yb = np.asarray(Ybar, dtype=np.float64)
    if X.ndim == 1:
        X, Yb = X[:, None], Yb[:, None]
    a = apply_U(fac, X)
    b = apply_U(fac, Yb)
    core = fac.core_ids
    mask = np.ones(fac.n, dtype=bool)
    mask[core] = False
    hdiag_bar = np.zeros(fac.n)
    hdiag_bar[mask] = (b[mask] * a[mask]).sum(axis=1)
    hcore_bar = b[core] @ a[core].T
    ga = _apply_H(fac, a)
    gb = _apply_H(dataclasses.replace(fac, hcore=fac.hcore.T), b)
    zx, zy = a.copy(), b.copy()
    R = len(fac.rotations)
    theta_bar = np.zeros(R) if fac.k == 2 else np.zeros((R, 3))
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    gens = rot3_generators()
    for t in range(R - 1, -1, -1):
        r = fac.rotations[t]
        ids = r.ids
        if len(ids) == 2:
            lt = float((ga[ids] * (J @ zy[ids])).sum() + (gb[ids] * (J @ zx[ids])).sum())
            if fac.k == 2:
                theta_bar[t] = lt
            else:  # a 2-point step inside a k = 3 factorization: its (0, 1) plane only
                theta_bar[t, 0] = lt
        else:
            l3 = np.array([float((ga[ids] * (G @ zy[ids])).sum() + (gb[ids] * (G @ zx[ids])).sum())
                           for G in gens])
            w = np.zeros(3) if theta is None else np.asarray(theta, dtype=np.float64)[t]
            theta_bar[t] = rot3_param_jacobian(w).T @ l3
        Ot = r.O.T
        zx[ids] = Ot @ zx[ids]
        zy[ids] = Ot @ zy[ids]
        ga[ids] = Ot @ ga[ids]
        gb[ids] = Ot @ gb[ids]
    return gb, hdiag_bar, hcore_bar, theta_bar


def angles(fac: Factorization) -> np.ndarray:
    """Givens angles theta_t = atan2(sin, cos) of each k = 2 rotation."""
    return np.array([math.atan2(r.O[1, 0], r.O[0, 0]) for r in fac.rotations])


def with_angles(fac: Factorization, theta: np.ndarray, hdiag=None, hcore=None) -> Factorization:
    """Copy of a k = 2 factorization with new angles (and optionally new H)."""
    rots = []
    for r, th in zip(fac.rotations, theta):
        c, s = math.cos(th), math.sin(th)
        rots.append(dataclasses.replace(r, O=np.array([[c, -s], [s, c]])))
    return dataclasses.replace(fac, rotations=rots,
                               hdiag=fac.hdiag if hdiag is None else hdiag,
                               hcore=fac.hcore if hcore is None else hcore)
