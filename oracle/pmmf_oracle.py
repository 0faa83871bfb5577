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
  R13 Decision margins (not part of the factorization), each a gap relative to the values it
      separates: partners (s_q - s_{q+1}) / s_q below each chosen rank q of the sorted scores;
      the rotation |tau| at the k = 2 root switch, the relative gap of the two best traces for
      k = 3, and for both the relative eigengap of G[T,T]; the elimination
      (off2_(2) - off2_(1)) / off2_(2).  A decision is a near-tie, where every choice is correct,
      if its margin is at most TIE = 1e-5 or if its absolute gap is within the FP32 error bounds
      of the two values compared: a method that stores the matrix, the Gram, the diagonal block
      and the rotations in FP32 cannot order values closer than that.  The bounds come from a
      first-order running error analysis of such a method (see KAPPA below), carried beside the
      FP64 values.  Replay adopts another implementation's choice at a near-tie and reports any
      other adopted choice as a divergence.
  R15 Angles of a 3-point rotation (the paper parametrizes only Givens rotations by an angle):
      O(w) = expm(w_0 G_01 + w_1 G_02 + w_2 G_12) O0, with O0 the rotation the search found and
      G_pq = E_qp - E_pq the generator of the (p, q) plane in slot order (G_01 extends the Givens
      J = [[0, -1], [1, 0]]); w = 0 at the start.
  R17 Several eliminations per rotation (optional; Sec. 2 allows more than one wavelet per
      k-point rotation): a rotation retires its `elims` slots with the smallest off-diagonal
      norms, smallest first (ties to the later slot), elims <= k - 1; a cluster still retires
      its r_u indices, so it takes ceil(r_u / elims) rotations, the last one retiring what is
      left.  Seeds are drawn per rotation (step s of the hash is the rotation's index).
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

def rotation_k2(g: np.ndarray, other_root: bool = False):
    """2x2 rotation O = [[c, -s], [s, c]] with O g O^T diagonal and |theta| <= pi/4.

    The symmetric Schur decomposition of a 2x2 block (Golub & Van Loan, Alg. 8.4.1), with the
    smaller-magnitude root of t^2 + 2 tau t - 1 = 0.  Returns (O, |tau|); |tau| -> 0 is where the
    choice of root switches sign.  ``other_root`` takes the other root t' = -1/t (|theta| >= pi/4),
    which diagonalizes g as well; replay adopts it where |tau| is a near-tie.
    """
    a, b, d = float(g[0, 0]), float(g[0, 1]), float(g[1, 1])
    if b == 0.0:
        return np.eye(2), math.inf
    tau = (d - a) / (2.0 * b)
    sgn = 1.0 if tau >= 0.0 else -1.0
    t = sgn / (abs(tau) + math.hypot(1.0, tau))
    if other_root:
        t = -1.0 / t
    c = 1.0 / math.sqrt(1.0 + t * t)
    s = t * c
    return np.array([[c, -s], [s, c]]), abs(tau)


def _relative_eigengap(lam_desc: np.ndarray) -> float:
    """Smallest gap between consecutive eigenvalues over the largest magnitude (0 if g = 0)."""
    scale = float(np.abs(lam_desc).max())
    if scale == 0.0:
        return 0.0
    return float(min(lam_desc[r] - lam_desc[r + 1] for r in range(len(lam_desc) - 1))) / scale


def rotation_k3(g: np.ndarray, prefer: Optional[np.ndarray] = None,
                with_trace_margin: bool = False):
    """k x k orthogonal O whose rows are eigenvectors of g, arranged closest to the identity.

    Rows are eigenvectors in descending eigenvalue order (LAPACK), then permuted and signed to
    maximize trace(O) with nonnegative diagonal; ties go to the lexicographically smallest
    permutation.  Returns (O, margin) with margin the smaller of the relative gap between the best
    and second-best trace and the relative eigengap (an eigenvector is determined only when its
    eigenvalue is simple).  ``prefer`` (replay at a near-tie only): among the permuted and signed
    arrangements take the one closest to ``prefer`` instead of the largest trace.
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
    trace_margin = (best - others[0]) / best if best > 0 else 0.0
    margin = min(trace_margin, _relative_eigengap(w[::-1]))

    def arrange(pm):
        O = np.empty((kk, kk))
        for r in range(kk):
            row = base[pm[r]]
            O[r] = row if row[r] >= 0.0 else -row
        return O

    if prefer is not None:
        perm = min(itertools.permutations(range(kk)),
                   key=lambda pm: (float(np.abs(arrange(pm) - prefer).max()), pm))
    if with_trace_margin:
        return arrange(perm), margin, trace_margin, best
    return arrange(perm), margin


def _nearest_orthogonal(O: np.ndarray) -> np.ndarray:
    """Orthogonal polar factor of O (closest orthogonal matrix in the Frobenius norm)."""
    u, _, vt = np.linalg.svd(np.asarray(O, dtype=np.float64))
    return u @ vt


# --------------------------------------------------------------------------- decision margins

TIE = 1e-5  # a decision whose margin (R13) is at most this is a near-tie: every choice is correct
# FP32 error bounds of the compared values (R13), by a first-order running error analysis of an
# FP32 implementation of the same steps.  A stage starts from running magnitudes: the same
# computation carried out on absolute values (|A| for the input, |Qbar| for each stage's two-sided
# rotation, |slab|^T |slab| for a Gram), and a Gram or diagonal-block entry starts within KAPPA
# U32 of its magnitude.  Each rotation then forms rows and columns T again from k terms with a
# rounded O: the new error is |O| times the old one, plus (k + 1) U32 |O| |G| for the rounding, plus
# |dO| |G| where dO bounds how far the eigenvectors of an FP32 G[T,T] lie from the exact ones.
U32 = 2.0 ** -24
KAPPA = 16.0
# FP32 keeps nothing below its smallest normal number 2^-126 (GPU code flushes subnormals), so a
# stored value errs by at least that much
TINY32 = 2.0 ** -126


def near_tie(rel: float, gap: float, err: float) -> bool:
    """R13: relative margin at most TIE, or an absolute gap within ``err``, the sum of the FP32
    error bounds of the two values compared."""
    return rel <= TIE or gap <= err


def score_error(g_ij: float, err_ij: float, g_jj: float, err_jj: float) -> float:
    """FP32 error bound of the score |G_ij| / sqrt(G_jj) from the error bounds of its two Gram
    entries (first-order perturbation of the quotient)."""
    if g_jj <= 0.0:
        return err_ij
    sc = abs(g_ij) / math.sqrt(g_jj)
    return err_ij / math.sqrt(g_jj) + sc * err_jj / (2.0 * g_jj)


def partner_decision(scores_desc: np.ndarray, kk: int, err_desc: np.ndarray):
    """R13 for the partner choice: (margin, tie).  The margin is the smallest relative gap
    (s_q - s_{q+1}) / s_q below a chosen rank q of the sorted scores (it fixes both the set and the
    slot order; 0 where the compared scores are zero, inf where no further candidate exists);
    the choice is a near-tie if some such gap is a near-tie, ``err_desc`` being the scores' FP32
    error bounds in the same order."""
    m, tie = math.inf, False
    for q in range(kk - 1):
        if q + 1 >= len(scores_desc):
            break
        hi, lo = float(scores_desc[q]), float(scores_desc[q + 1])
        rel = (hi - lo) / hi if hi > 0 else 0.0
        m = min(m, rel)
        tie = tie or near_tie(rel, hi - lo, float(err_desc[q]) + float(err_desc[q + 1]))
    return m, tie


def elimination_decision(off2, err):
    """R13 for the elimination: (off2_(2) - off2_(1)) / off2_(2) over the two smallest values;
    ``err`` are the FP32 error bounds of off2_t = G_tt - D_tt^2 in slot order."""
    order = sorted(range(len(off2)), key=lambda t: float(off2[t]))
    v1, v2 = float(off2[order[0]]), float(off2[order[1]])
    rel = (v2 - v1) / v2 if v2 > 0 else 0.0
    return rel, near_tie(rel, v2 - v1, float(err[order[0]]) + float(err[order[1]]))


def rotation_decision(gTT: np.ndarray, errTT: np.ndarray):
    """R13 for the rotation: (margin, tie, relative eigengap, eigenvector error bound).

    G[T,T] known to within ``errTT`` entrywise errs by at most E = ||errTT||_F in the 2-norm,
    which moves each eigenvalue by at most E (Weyl) and each eigenvector by at most E / gap
    (Davis-Kahan).  k = 2: the root switch |tau|, fixed by the sign of G_jj - G_ii (a near-tie
    within the error bounds of the two diagonal entries), and the eigengap (a near-tie within
    2E).  k = 3: the relative gap of the two best traces (each trace moves by at most 3 E / gap)
    and the eigengap."""
    lam = np.linalg.eigvalsh(gTT)[::-1]
    scale = float(np.abs(lam).max())
    eig = _relative_eigengap(lam)
    gap_abs = eig * scale
    E = float(np.sqrt((np.asarray(errTT) ** 2).sum()))
    tie_eig = near_tie(eig, gap_abs, 2.0 * E)
    vec_err = E / gap_abs if gap_abs > 0 else math.inf
    if gTT.shape[0] == 2:
        _, tau = rotation_k2(gTT)
        a, d = float(gTT[0, 0]), float(gTT[1, 1])
        err_ad = float(errTT[0, 0]) + float(errTT[1, 1])
        tie_root = near_tie(tau, abs(d - a), err_ad) if gTT[0, 1] != 0.0 else False
        return min(tau, eig), tie_root or tie_eig, eig, vec_err
    _, m, tr, best = rotation_k3(gTT, with_trace_margin=True)   # m = min(trace margin, eigengap)
    tie_tr = near_tie(tr, tr * best, 2.0 * 3.0 * vec_err)
    return m, tie_tr or tie_eig, eig, vec_err


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
    margin: float            # smallest decision margin of the step (R13)
    margins: tuple = ()      # (partner, rotation, elimination) relative margins (R13)
    eig_gap: float = math.inf  # relative eigengap of G[T,T] (sets how well O is determined)
    o_err: float = 0.0       # bound on how far an FP32 G[T,T] moves the rows of O (R13)
    near_ties: tuple = ()    # (partner, rotation, elimination): near-tie under R13
    adopted: tuple = ()      # replay: decisions taken from the replayed log instead of the rule


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
    divergences: list = dataclasses.field(default_factory=list)
    # replay: (rotation index, decision, margin) for every adopted decision whose margin > TIE

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


def _search_cluster(slab, D, gids, r_u, k, seed, p, u, replay=None, on_step=None, ctx=None,
                    slab_abs=None, D_abs=None, elims=1):
    """Algorithm 2 on one cluster: greedy steps on its Gram and diagonal block until r_u indices
    are retired, ``elims`` per rotation (R17; the last step may retire fewer).

    ``slab`` is the column slab M[S_{p-1}, B_u] (sparse), ``D`` the diagonal block, ``gids`` the
    global ids of the cluster's columns.  ``replay`` (ids [r_u][k], retired [r_u], O [r_u][k][k]:
    another implementation's log of this cluster, global ids) makes the step take that log's choice
    wherever it differs from the rule's; every such decision is reported with its margin (R13).
    ``slab_abs`` and ``D_abs`` are the running magnitudes of the slab and the block (R13): they
    set the initial FP32 error bounds of the Gram and the block, which are carried through the
    rotations beside them, only to bound the error of each compared value.
    Returns the rotations, the accumulated Q_u (sparse), the retired local positions in step order,
    their H entries and the literal loss terms."""

    def gram(sl):                                        # local Gram, Sec. 2.1
        if sl.nnz >= 0.1 * sl.shape[0] * sl.shape[1]:    # (filled-in late stages: BLAS product)
            dense = sl.toarray()
            return dense.T @ dense
        return (sl.T @ sl).toarray()

    def dense(x):
        return x.toarray() if sp.issparse(x) else np.array(x, dtype=np.float64)

    G = gram(slab)
    D = dense(D)
    # FP32 error bounds of the Gram and the diagonal block (R13)
    ErrG = KAPPA * U32 * gram(abs(slab) if slab_abs is None else slab_abs) + TINY32
    ErrD = KAPPA * U32 * (np.abs(D) if D_abs is None else dense(D_abs)) + TINY32
    c = G.shape[0]
    Qu = np.eye(c)
    active = np.ones(c, dtype=bool)                      # I = [c]
    rots, retired, hd, literal = [], [], [], []
    ent, s = 0, 0                                        # log entries (one per retiree), steps
    while ent < r_u:
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
        T = [i] + [int(j) for j in order[:kk - 1]]

        def err(j):                                      # FP32 error bound of score j (R13)
            return score_error(G[i, j], ErrG[i, j], G[j, j], ErrG[j, j])

        score_err = np.array([err(j) for j in order[:kk]])
        m_part, tie_part = partner_decision(score[order[:kk]], kk, score_err)
        adopted = []
        rp_s = replay is not None and bool(replay["use"][ent])
        if rp_s:
            g_ids = np.minimum(np.searchsorted(gids, replay["ids"][ent][:kk]), c - 1)
            g_T = [int(x) for x in g_ids]
            if not np.array_equal(gids[g_ids], replay["ids"][ent][:kk]):
                adopted.append(("partners", False, m_part))   # not a tuple of this cluster
            elif g_T != T:
                # the other log's tuple is correct if its seed is this seed and each of its
                # partners scores within the tie margin of the same rank's best score
                valid = g_T[0] == i and len(set(g_T)) == kk and all(active[j] for j in g_T)
                ok = valid and all(
                    near_tie(abs(score[g_T[q + 1]] - score[order[q]]) / score[order[q]]
                             if score[order[q]] > 0 else 0.0,
                             abs(score[g_T[q + 1]] - score[order[q]]),
                             err(g_T[q + 1]) + err(order[q]))
                    for q in range(kk - 1))
                adopted.append(("partners", ok, m_part))
                if valid:
                    T = g_T
        # rotation that diagonalizes the k x k Gram block (R6)
        gTT = G[np.ix_(T, T)]
        O = rotation_k2(gTT)[0] if kk == 2 else rotation_k3(gTT)[0]
        m_rot, tie_rot, eig_gap, vec_err = rotation_decision(gTT, ErrG[np.ix_(T, T)])
        if rp_s:
            g_O = np.asarray(replay["O"][ent][:kk, :kk], dtype=np.float64)
            alt = O
            if np.abs(O - g_O).max() > 1e-3:
                if kk == 2:
                    alt = rotation_k2(gTT, other_root=True)[0]
                else:
                    alt = rotation_k3(gTT, prefer=g_O)[0]
            # a different root / arrangement of the eigenvectors is a decision (R6, R13)
            if np.abs(alt - g_O).max() < np.abs(O - g_O).max():
                adopted.append(("rotation", tie_rot, m_rot))
                O = alt
                if tie_rot and np.abs(O - g_O).max() > 1e-3:
                    O = _nearest_orthogonal(g_O)      # a multiple eigenvalue: any basis is right
        # G <- O G O^T and the same for the diagonal block and the accumulated Q (Alg. 2), with
        # the error bounds carried beside them (R13): |O| err + dO |X| + (k + 1) u |O| |X|
        Oabs = np.abs(O)
        dO = min(vec_err, 2.0)
        for X, Err in ((G, ErrG), (D, ErrD)):
            Xa = np.abs(X[T, :])
            Err[T, :] = (Oabs @ Err[T, :] + dO * Xa.sum(axis=0)[None, :]
                         + (kk + 1) * U32 * (Oabs @ Xa) + TINY32)
            X[T, :] = O @ X[T, :]
            Xa = np.abs(X[:, T])
            Err[:, T] = (Err[:, T] @ Oabs.T + dO * Xa.sum(axis=1)[:, None]
                         + (kk + 1) * U32 * (Xa @ Oabs.T) + TINY32)
            X[:, T] = X[:, T] @ O.T
        Qu[T, :] = O @ Qu[T, :]
        # eliminate the slot with the smallest off-diagonal norm, ties to the later (R5); with
        # several eliminations per rotation (R17) the next smallest of the remaining slots, and so
        # on, each logged as its own entry on T (the later ones with the identity block)
        off2 = [max(0.0, G[tt, tt] - D[tt, tt] ** 2) for tt in T]
        off2_err = [ErrG[tt, tt] + 2.0 * abs(D[tt, tt]) * ErrD[tt, tt] for tt in T]
        left = list(range(kk))
        first_e = None
        for q in range(min(elims, kk - 1, r_u - ent)):
            e_slot = left[0]
            for sl in left[1:]:
                if off2[sl] <= off2[e_slot]:
                    e_slot = sl
            m_elim, tie_elim = elimination_decision([off2[sl] for sl in left],
                                                    [off2_err[sl] for sl in left])
            adopted_e = list(adopted) if q == 0 else []
            if replay is not None and bool(replay["use"][ent]):
                g_e = int(np.searchsorted(gids, replay["retired"][ent]))
                if q > 0 and not np.array_equal(replay["ids"][ent][:kk], gids[np.asarray(T)]):
                    adopted_e.append(("partners", False, math.inf))  # not this step's tuple
                if g_e != T[e_slot] and g_e in [T[sl] for sl in left]:
                    adopted_e.append(("elimination", tie_elim, m_elim))
                    e_slot = T.index(g_e)
                elif g_e != T[e_slot]:
                    adopted_e.append(("elimination", False, m_elim))
            left.remove(e_slot)
            e = T[e_slot]
            first_e = e if first_e is None else first_e
            active[e] = False
            retired.append(e)
            hd.append(float(D[e, e]))
            literal.append(2.0 * off2[e_slot])
            if q == 0:
                rots.append(Rotation(stage=p, cluster=u, step=s, ids=gids[np.asarray(T)].copy(),
                                     O=O.copy(), retired=int(gids[e]), seed_pos=i,
                                     margin=float(min(m_part, m_rot, m_elim)),
                                     margins=(m_part, m_rot, m_elim), eig_gap=eig_gap,
                                     o_err=vec_err, near_ties=(tie_part, tie_rot, tie_elim),
                                     adopted=tuple(adopted_e)))
            else:
                rots.append(Rotation(stage=p, cluster=u, step=s, ids=gids[np.asarray(T)].copy(),
                                     O=np.eye(kk), retired=int(gids[e]), seed_pos=i,
                                     margin=float(m_elim), margins=(math.inf, math.inf, m_elim),
                                     near_ties=(False, False, tie_elim),
                                     adopted=tuple(adopted_e)))
            ent += 1
        if on_step is not None:
            on_step(dict(stage=p, cluster=u, step=s, G=G, D=D, T=list(T), O=O, e=first_e,
                         active=active.copy(), ranked=[int(j) for j in order[:kk]],
                         score_err=score_err, off2_err=off2_err, **(ctx or {})))
        s += 1
    Qs = sp.csr_matrix(Qu)
    Qs.eliminate_zeros()
    return dict(rots=rots, Q=Qs, retired=retired, hd=hd, literal=literal)


# state of the stage being computed, read by the per-cluster tasks (a forked worker inherits it)
_STAGE: dict = {}


def _stage_map(fn, items, workers: int):
    """[fn(x) for x in items], in ``workers`` forked processes when workers > 1."""
    if workers <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    import concurrent.futures
    import multiprocessing
    with concurrent.futures.ProcessPoolExecutor(
            max_workers=min(workers, len(items)),
            mp_context=multiprocessing.get_context("fork")) as pool:
        return list(pool.map(fn, items))


def _cluster_task(u: int):
    """Algorithm 2 on cluster u of the current stage."""
    st = _STAGE
    off, c = int(st["offsets"][u]), int(st["sizes"][u])
    rp = None
    if st["replay"] is not None:
        r0 = st["r_base"] + sum(st["r_u"][:u])
        r1 = r0 + st["r_u"][u]
        use = st["replay"].get("rot_use")
        rp = dict(ids=st["replay"]["rot_ids"][r0:r1], retired=st["replay"]["rot_retired"][r0:r1],
                  O=st["replay"]["rot_o"][r0:r1],
                  use=np.ones(r1 - r0, dtype=bool) if use is None else use[r0:r1])
    ctx = dict(offset=off, S=st["S"]) if st["on_step"] is not None else None
    return _search_cluster(st["Mc"][:, off:off + c],           # rows: all of S_{p-1} (R4)
                           st["M"][off:off + c, off:off + c],  # [[A]]_{u,u}
                           st["S"][off:off + c].copy(), st["r_u"][u], st["k"], st["seed"],
                           st["p"], u, rp, st["on_step"], ctx,
                           st["Mabs_c"][:, off:off + c], st["Mabs"][off:off + c, off:off + c],
                           st["elims"])


def _rotate_rows_task(u: int):
    """Block rows B_u of A_p = Qbar A_{p-1} Qbar^T, Q_u [[A_{p-1}]]_{u,:} Qbar^T (Alg. 1), then
    their part of the exact loss (R12) and of the peeled matrix: the rows of B_u that survive,
    restricted to the surviving columns."""
    st = _STAGE
    off, c = int(st["offsets"][u]), int(st["sizes"][u])
    QM_u = (st["Q"][u] @ st["M"][off:off + c]).tocsr()
    rows = (QM_u @ st["QbarT"]).tocsr()
    rows.eliminate_zeros()
    keep, R = st["keep"], st["R"]
    local_keep = keep[off:off + c]
    mine = R[(R >= off) & (R < off + c)] - off             # this block's retired rows
    MR = rows[mine]
    m_rs = MR[:, st["Sv"]]
    m_rr = MR[:, R].tocoo()
    m_rr_off = m_rr.data[mine[m_rr.row] + off != R[m_rr.col]]   # only e' != e enters
    stats = dict(sq_rs=float((m_rs.data ** 2).sum()), sq_rr=float((m_rr_off ** 2).sum()),
                 diag_R=np.asarray(rows[mine, mine + off]).ravel() if mine.size else np.zeros(0),
                 qm_row_nnz_max=int(np.diff(QM_u.indptr).max()) if QM_u.nnz else 0,
                 row_nnz_max=int(np.diff(rows.indptr).max()) if rows.nnz else 0,
                 fro2=float((rows.data ** 2).sum()), mine=mine + off)
    # running magnitudes of the same rows (R13): |Q_u| |A_{p-1}|_mag[B_u, :] |Qbar|^T
    mag = ((abs(st["Q"][u]) @ st["Mabs"][off:off + c]) @ st["QbarT_abs"]).tocsr()
    surv = np.flatnonzero(local_keep)
    return stats, rows[surv][:, st["Sv"]].tocsr(), mag[surv][:, st["Sv"]].tocsr()


def factor(A, k: int = 2, eta: float = 0.5, core: int = 64, cluster=(0, 0), seed: int = 0,
           even_clusters: bool = False, cut_clusters: bool = False,
           on_step: Optional[Callable[[dict], None]] = None, replay: Optional[dict] = None,
           workers: int = 1, elims: int = 1) -> Factorization:
    """pMMF factorization A ~ U^T H U (Eq. 1 / Eq. 4) by Algorithm 1 with Algorithm 2 inside.

    ``A`` is symmetric (a CSR from ``workloads``, a SciPy sparse matrix or a dense array).
    ``on_step`` (tests only) receives the cluster's state after every rotation.
    ``replay`` (tests only): a rotation log of another implementation in (stage, cluster, step)
    order, a dict with ``rot_ids`` [R][k] and ``rot_retired`` [R] (global ids) and ``rot_o``
    [R][k][k], optionally ``rot_use`` [R] (False: that step follows the rule); where the log's
    choice differs from the rule's, the step takes it and records the decision with its margin,
    and ``Factorization.divergences`` lists those that are not near-ties (R13).
    ``workers`` > 1 runs the clusters of a stage (their searches, and their block rows of the
    two-sided rotation) in that many forked processes: clusters are independent (Sec. 2.3), and
    the result does not depend on it.
    ``elims`` (R17): indices retired per rotation, 1 <= elims <= k - 1.  The log keeps one entry
    per retired index: a rotation's later eliminations follow it as entries on the same tuple with
    the identity block.
    """
    if k not in (2, 3):
        raise ValueError("k must be 2 or 3")
    if not (1 <= elims <= k - 1):
        raise ValueError("elims must lie in [1, k - 1]")
    M = _as_csr64(A)
    n = M.shape[0]
    if (abs(M - M.T) > 0).nnz:
        raise ValueError("matrix is not symmetric")
    if on_step is not None:
        workers = 1
    lo, hi = cluster
    schedule = stage_schedule(n, core, eta)
    S = np.arange(n)                    # global ids of the active positions, ascending
    Mabs = abs(M)                       # running magnitude of the active matrix (R13)
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
        _STAGE.clear()
        _STAGE.update(M=M, Mc=M.tocsc(), Mabs=Mabs, Mabs_c=Mabs.tocsc(), S=S, offsets=offsets,
                      sizes=sizes, r_u=r_u, k=k, elims=elims,
                      seed=seed, p=p, replay=replay, r_base=len(rotations), on_step=on_step)
        results = _stage_map(_cluster_task, list(range(len(sizes))), workers)
        retired_pos = []                # compact positions retired in this stage, in order
        for u, res in enumerate(results):
            off = int(offsets[u])
            for rot, e, h, lit in zip(res["rots"], res["retired"], res["hd"], res["literal"]):
                gid_e = int(S[off + e])
                hdiag[gid_e] = h
                loss_literal += lit
                retired_pos.append(off + e)
                retired_order.append(gid_e)
                rotations.append(rot)

        # rotate the whole (blocked) matrix from both sides with the stage's rotations (Alg. 1):
        # block rows [[A_p]]_{u,:} = Q_u [[A_{p-1}]]_{u,:} Qbar^T with Qbar = diag(Q_1, ..., Q_m);
        # then the exact loss of this stage's retirements (R12) and the peeling of their rows and
        # columns
        R = np.asarray(retired_pos, dtype=np.int64)
        keep = np.ones(size, dtype=bool)
        keep[R] = False
        Sv = np.flatnonzero(keep)
        Q = [res["Q"] for res in results]
        QbarT = sp.block_diag(Q, format="csr").T.tocsr()
        _STAGE.update(Q=Q, QbarT=QbarT, QbarT_abs=abs(QbarT), keep=keep, R=R, Sv=Sv)
        blocks = _stage_map(_rotate_rows_task, list(range(len(sizes))), workers)
        _STAGE.clear()
        row_nnz_max = int(np.diff(M.indptr).max()) if M.nnz else 0
        stage_loss = sum(2.0 * st["sq_rs"] + st["sq_rr"] for st, _, _ in blocks)
        loss += stage_loss
        fro_end = math.sqrt(sum(st["fro2"] for st, _, _ in blocks))
        diag_R = np.zeros(size)
        for st, _, _ in blocks:
            diag_R[st["mine"]] = st["diag_R"]
        hdiag_check = float(np.max(np.abs(diag_R[R] - hdiag[S[R]]))) if R.size else 0.0
        stages.append(dict(stage=p, size=size, rotations=t, cluster_sizes=sizes,
                           cluster_rotations=r_u, offsets=offsets, active=S.copy(),
                           retired=S[R].copy(), nnz_start=nnz_start, fro_start=fro_start,
                           row_nnz_max=row_nnz_max,
                           qm_row_nnz_max=max(st["qm_row_nnz_max"] for st, _, _ in blocks),
                           full_row_nnz_max=max(st["row_nnz_max"] for st, _, _ in blocks),
                           fro_end=fro_end, loss=stage_loss, hdiag_check=hdiag_check))
        M = sp.vstack([blk for _, blk, _ in blocks], format="csr")
        Mabs = sp.vstack([mag for _, _, mag in blocks], format="csr")
        S = S[Sv]

    divergences = [(t, what, m) for t, r in enumerate(rotations)
                   for what, ok, m in r.adopted if not ok]
    hcore = M.toarray()
    return Factorization(n=n, k=k, rotations=rotations, stages=stages, hdiag=hdiag,
                         core_ids=S.copy(), hcore=hcore, loss=loss, loss_literal=loss_literal,
                         retired_order=np.asarray(retired_order, dtype=np.int64),
                         divergences=divergences)


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
