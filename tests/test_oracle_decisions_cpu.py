"""Pins for the oracle's decision rules, margins and replay (R13), all on the CPU.

* Margins and near-tie tests against hand-computed values.
* The seeded cluster sizes against hand arithmetic with the hash replaced by chosen values.
* Replay: an oracle log replays to itself; a planted near-tie choice is adopted silently; a
  planted choice that is not a tie is reported.
* The FP32 resolution floor RHO: an FP32 model of the path (matrix, Gram, diagonal block and
  rotations stored in FP32, the decisions of the FP64 run) stays within half the floor in every
  compared quantity, so a gap beyond the floor is resolved by FP32 arithmetic.
* Exhaustive pair search on n <= 16: the greedy step's loss increment against the best of all
  pairs and both eliminations from the same state.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.pmmf_oracle as om
import workloads


# --------------------------------------------------------------------------- margins by hand

def test_partner_margin_hand_values():
    e = np.zeros(3)
    m, tie = oracle.partner_decision(np.array([0.5, 0.4, 0.1]), 2, e)
    assert m == pytest.approx(0.2) and not tie            # (0.5 - 0.4) / 0.5
    m, tie = oracle.partner_decision(np.array([0.5, 0.4, 0.1]), 3, e)
    assert m == pytest.approx(0.2) and not tie            # min(0.2, (0.4 - 0.1) / 0.4)
    m, tie = oracle.partner_decision(np.array([1.0, 1.0 - 5e-6, 0.2]), 2, e)
    assert m == pytest.approx(5e-6) and tie               # relative gap at most 1e-5
    m, tie = oracle.partner_decision(np.array([2e-7, 1e-7]), 2, np.array([6e-8, 5e-8]))
    assert m == pytest.approx(0.5) and tie                # gap 1e-7 within the errors 6e-8 + 5e-8
    m, tie = oracle.partner_decision(np.array([2e-7, 1e-7]), 2, np.array([4e-8, 5e-8]))
    assert not tie                                        # gap 1e-7 beyond 4e-8 + 5e-8
    m, tie = oracle.partner_decision(np.array([0.5, 0.4, 0.4 - 1e-9]), 3, e)
    assert tie                                            # ranks 2 and 3 tie: the slot order
    m, tie = oracle.partner_decision(np.array([0.0, 0.0]), 2, e)
    assert m == 0.0 and tie                               # all scores zero
    m, tie = oracle.partner_decision(np.array([0.7]), 2, e)
    assert m == math.inf and not tie                      # a single candidate: no choice


def test_score_error_bound_by_hand():
    # s = |g| / sqrt(h) with |dg| <= eg, |dh| <= eh: |ds| <= eg / sqrt(h) + s eh / (2 h)
    assert oracle.score_error(-3.0, 5e-6, 4.0, 6e-6) == pytest.approx(5e-6 / 2.0 + 1.5 * 6e-6 / 8.0)
    assert oracle.score_error(1.0, 2e-6, 0.0, 1e-6) == pytest.approx(2e-6)


def test_elimination_margin_hand_values():
    m, tie = oracle.elimination_decision([3.0, 1.0], [0.0, 0.0])
    assert m == pytest.approx(2.0 / 3.0) and not tie
    m, tie = oracle.elimination_decision([1.0, 1.0 + 1e-6, 4.0], [0.0, 0.0, 0.0])
    assert m == pytest.approx(1e-6 / (1.0 + 1e-6)) and tie
    # the two smallest are slots 1 and 0: the error bounds of those two count, not slot 2's
    m, tie = oracle.elimination_decision([2e-6, 1e-6, 5.0], [6e-7, 5e-7, 1.0])
    assert m == pytest.approx(0.5) and tie                # gap 1e-6 within 6e-7 + 5e-7
    m, tie = oracle.elimination_decision([2e-6, 1e-6, 5.0], [4e-7, 5e-7, 1.0])
    assert not tie


def test_rotation_margin_hand_values():
    z2, z3 = np.zeros((2, 2)), np.zeros((3, 3))
    # tau = (G_jj - G_ii) / (2 G_ij) = 0: the root switch itself
    m, tie, eig, _ = oracle.rotation_decision(np.array([[1.0, 0.5], [0.5, 1.0]]), z2)
    assert m == 0.0 and tie
    # tau = -1; eigenvalues 1.5 +- sqrt(0.5): relative eigengap 2 sqrt(0.5) / (1.5 + sqrt(0.5))
    g = np.array([[2.0, 0.5], [0.5, 1.0]])
    m, tie, eig, verr = oracle.rotation_decision(g, z2)
    gap = 2 * math.sqrt(0.5) / (1.5 + math.sqrt(0.5))
    assert eig == pytest.approx(gap) and m == pytest.approx(gap) and not tie and verr == 0.0
    # the same block known to within 1e-4 entrywise: E = ||err||_F = 2e-4, eigenvectors move by at
    # most E / gap (Davis-Kahan), gap = 2 sqrt(0.5)
    _, tie, _, verr = oracle.rotation_decision(g, np.full((2, 2), 1e-4))
    assert verr == pytest.approx(2e-4 / (2 * math.sqrt(0.5)), rel=1e-9) and not tie
    # an eigengap within 2E: the eigenvectors are undetermined
    assert oracle.rotation_decision(g, np.full((2, 2), 0.4))[1]
    # G_jj - G_ii = 1e-4 (tau = 1e-4): resolved with exact entries, undetermined once the error
    # bounds of the two diagonal entries add up to more than that
    g = np.array([[1.0, 0.5], [0.5, 1.0 + 1e-4]])
    assert oracle.rotation_decision(g, z2)[1] is False
    assert oracle.rotation_decision(g, np.array([[6e-5, 0.0], [0.0, 6e-5]]))[1]
    # k = 3, diag(3, 2, 1): O = I; eigengap 1/3; the best other trace is 1 (a transposition)
    m, tie, eig, _ = oracle.rotation_decision(np.diag([3.0, 2.0, 1.0]), z3)
    assert eig == pytest.approx(1.0 / 3.0) and m == pytest.approx(1.0 / 3.0) and not tie
    # a double eigenvalue leaves the eigenvectors undetermined
    m, tie, eig, _ = oracle.rotation_decision(np.diag([2.0, 2.0, 1.0]), z3)
    assert eig == 0.0 and tie


# --------------------------------------------------------------------------- cluster sizes

def test_cluster_sizes_by_hand_with_chosen_hash_values(monkeypatch):
    """Sizes are lo + floor(h (hi - lo + 1) / 2^64) from the tag-2 hash of (seed, p, q, 0), each
    clipped so at least lo indices remain, the last cluster taking the rest."""
    calls = []
    values = [0, 1 << 63, (1 << 64) - 1, 3 << 62]

    def fake(seed, *vals):
        calls.append((seed,) + vals)
        return values[len(calls) - 1]

    monkeypatch.setattr(om, "chain_hash", fake)
    # lo = 10, hi = 25 (16 sizes): h = 0 -> 10; 2^63 -> 10 + 8 = 18; 2^64 - 1 -> 10 + 15 = 25;
    # then 100 - 53 = 47 > 25 remain: h = 3 * 2^62 -> 10 + 12 = 22, 25 remain -> last cluster
    assert om.cluster_sizes(100, 10, 25, seed=77, p=3) == [10, 18, 25, 22, 25]
    assert calls == [(77, 2, 3, 0, 0), (77, 2, 3, 1, 0), (77, 2, 3, 2, 0), (77, 2, 3, 3, 0)]
    # 40 > hi: h = 2^64 - 1 gives 25, the last cluster takes the remaining 15
    calls.clear()
    values[:] = [(1 << 64) - 1]
    assert om.cluster_sizes(40, 10, 25, seed=1, p=1) == [25, 15]
    calls.clear()
    values[:] = [(1 << 64) - 1]
    assert om.cluster_sizes(33, 10, 25, seed=1, p=2) == [23, 10]   # 25 clipped to 33 - lo
    assert om.cluster_sizes(25, 10, 25, seed=1, p=2) == [25]       # at most hi: one cluster


def test_cluster_sizes_reach_both_ends_of_the_range():
    seen = set()
    for seed in range(60):
        for p in range(1, 6):
            seen.update(oracle.cluster_sizes(10_000, 10, 20, seed, p)[:-1])
    assert seen == set(range(10, 21))


# --------------------------------------------------------------------------- replay

def _log(fac):
    k = fac.k
    R = len(fac.rotations)
    return dict(rot_ids=np.array([r.ids for r in fac.rotations], dtype=np.int64).reshape(R, k),
                rot_retired=np.array([r.retired for r in fac.rotations], dtype=np.int64),
                rot_o=np.array([r.O for r in fac.rotations], dtype=np.float32).reshape(R, k, k))


@pytest.mark.parametrize("case", ["k2", "k3"])
def test_replay_of_own_log_adopts_nothing(case):
    if case == "k2":
        A, prm = workloads.small_grid((14, 14), seed=3), dict(k=2, core=20, cluster=(16, 48), seed=2)
    else:
        A = workloads.knn_points_matrix(300, 2, 8, 0.01, 4)
        prm = dict(k=3, core=30, cluster=(24, 80), seed=1)
    free = oracle.factor(A, **prm)
    rep = oracle.factor(A, replay=_log(free), workers=2, **prm)
    assert not rep.divergences
    assert all(not r.adopted for r in rep.rotations)
    assert rep.loss == free.loss
    np.testing.assert_array_equal(rep.retired_order, free.retired_order)
    np.testing.assert_array_equal(rep.hcore, free.hcore)


def _find_step(fac, pred):
    for t, r in enumerate(fac.rotations):
        if pred(r):
            return t
    raise AssertionError("no such step")


def test_replay_reports_a_planted_non_tie_elimination_and_partner():
    A = workloads.small_grid((14, 14), seed=3)
    prm = dict(k=2, core=20, cluster=(16, 48), seed=2)
    free = oracle.factor(A, **prm)
    t = _find_step(free, lambda r: r.margins[2] > 0.1 and r.margins[0] > 0.1 and r.stage == 1)
    lg = _log(free)
    r = free.rotations[t]
    other = int(r.ids[0]) if r.retired == int(r.ids[1]) else int(r.ids[1])
    lg["rot_retired"][t] = other
    rep = oracle.factor(A, replay=lg, **prm)
    assert rep.divergences[0][:2] == (t, "elimination")
    assert rep.retired_order[t] == other                  # the log's choice is taken
    # a partner far below the best
    lg = _log(free)
    st = free.stages[0]
    u, off = r.cluster, int(st["offsets"][r.cluster])
    cl_ids = st["active"][off:off + st["cluster_sizes"][u]]
    bad = [int(g) for g in cl_ids if g not in r.ids and g not in free.retired_order[:t]][-1]
    lg["rot_ids"][t, 1] = bad
    rep = oracle.factor(A, replay=lg, **prm)
    assert rep.divergences[0][:2] == (t, "partners")


def test_replay_adopts_a_near_tie_silently_and_stays_valid():
    """A path graph with equal weights is symmetric under reflection, so many eliminations compare
    equal off-diagonal norms: replaying the other choice at such a step is a tie."""
    n = 64
    a = np.diag(np.full(n, 2.0)) - np.eye(n, k=1) - np.eye(n, k=-1)
    A = workloads.csr_from_dense(a)
    prm = dict(k=2, core=8, cluster=(0, 0), seed=3)
    free = oracle.factor(A, **prm)
    t = _find_step(free, lambda r: r.near_ties[2] and r.margins[2] <= oracle.TIE)
    # the other side of the tie at step t, then the rule's own continuation from there
    lg = _log(free)
    r = free.rotations[t]
    lg["rot_retired"][t] = int(r.ids[0]) if r.retired == int(r.ids[1]) else int(r.ids[1])
    lg["rot_use"] = np.arange(len(free.rotations)) <= t
    alt = oracle.factor(A, replay=lg, **prm)
    assert alt.retired_order[t] != free.retired_order[t]
    rep = oracle.factor(A, replay=_log(alt), **prm)
    assert not rep.divergences
    assert [(t2, w, ok) for t2, r2 in enumerate(rep.rotations) for w, ok, _ in r2.adopted] == \
        [(t, "elimination", True)]
    # the replayed factorization is still exact in its own accounting (three-way identity)
    U = oracle.dense_U(rep)
    H = np.diag(rep.hdiag)
    H[np.ix_(rep.core_ids, rep.core_ids)] = rep.hcore
    dense = float(((a - U.T @ H @ U) ** 2).sum())
    assert abs(rep.loss - dense) <= 1e-10 * float((a ** 2).sum())


# --------------------------------------------------------------------------- FP32 floor

def _fp32_model_errors(A, params):
    """FP32 errors of the values each decision compares, against the oracle's bounds for them.

    The oracle's decision sequence is re-run twice, with the matrix, each cluster's Gram and
    diagonal block and the rotations stored in FP64 and in FP32 (NumPy arithmetic in that type,
    so each operation rounds as an FP32 implementation's would).  Per step this gives, for the
    oracle's ranked candidates, |score_32 - score_64| / bound and, for the slots,
    |off2_32 - off2_64| / bound, the bounds being the oracle's own (R13)."""
    steps = []

    def on_step(d):
        steps.append(dict(stage=d["stage"], cluster=d["cluster"], T=list(d["T"]), e=d["e"],
                          O=d["O"].copy(), ranked=list(d["ranked"]),
                          score_err=np.array(d["score_err"]), off2_err=np.array(d["off2_err"])))

    fac = oracle.factor(A, on_step=on_step, **params)
    dts = (np.float64, np.float32)
    Ms = [A.to_scipy(np.float64).astype(dt) for dt in dts]
    ratios_s, ratios_o = [], []
    it = iter(steps)
    for st in fac.stages:
        Qs = [[] for _ in dts]
        for u, c in enumerate(st["cluster_sizes"]):
            off = int(st["offsets"][u])
            state = []
            for M, dt in zip(Ms, dts):
                slab = M[:, off:off + c].toarray()
                state.append([slab.T @ slab, M[off:off + c, off:off + c].toarray(),
                              np.eye(c, dtype=dt)])
            for _ in range(st["cluster_rotations"][u]):
                d = next(it)
                T, i = d["T"], d["T"][0]
                sc = []
                for G, _, _ in state:
                    sc.append(np.array([abs(float(G[i, j])) / math.sqrt(float(G[j, j]))
                                        if G[j, j] > 0 else 0.0 for j in d["ranked"]]))
                ratios_s.extend(np.abs(sc[1] - sc[0]) / np.maximum(d["score_err"], 1e-300))
                offs = []
                for (G, D, Q), dt in zip(state, dts):
                    O = d["O"].astype(dt)
                    G[T, :] = O @ G[T, :]
                    G[:, T] = G[:, T] @ O.T
                    D[T, :] = O @ D[T, :]
                    D[:, T] = D[:, T] @ O.T
                    Q[T, :] = O @ Q[T, :]
                    offs.append(np.array([float(G[x, x]) - float(D[x, x]) ** 2 for x in T]))
                ratios_o.extend(np.abs(offs[1] - offs[0]) / np.maximum(d["off2_err"], 1e-300))
            for q in range(len(dts)):
                Qs[q].append(sp.csr_matrix(state[q][2]))
        keep = np.isin(st["active"], st["retired"], invert=True)
        for q, dt in enumerate(dts):
            Qb = sp.block_diag(Qs[q], format="csr").astype(dt)
            Mn = (Qb @ Ms[q] @ Qb.T).tocsr()
            Ms[q] = Mn[keep][:, keep].tocsr()
    return np.array(ratios_s), np.array(ratios_o)


PRECISION_CASES = [
    ("knn2d_n512", lambda: workloads.make_matrix("knn2d_n512"),
     workloads.WORKLOADS["knn2d_n512"]["params"]),
    ("grid32x32_lognormal_clusters", lambda: workloads.small_grid((32, 32), seed=1),
     dict(k=2, eta=0.5, core=64, cluster=(64, 256), seed=0)),
    ("knn2d_n700_k3_clusters", lambda: workloads.knn_points_matrix(700, 2, 8, 0.01, 4),
     dict(k=3, eta=0.5, core=50, cluster=(40, 120), seed=1)),
    ("knn3d_n1000_k3_single", lambda: workloads.knn_points_matrix(1000, 3, 10, 0.01, 2),
     dict(k=3, eta=0.5, core=64, cluster=(0, 0), seed=0)),
]


@pytest.mark.parametrize("name,make,params", PRECISION_CASES, ids=[c[0] for c in PRECISION_CASES])
def test_fp32_errors_of_compared_values_stay_within_half_the_bound(name, make, params):
    """The oracle's FP32 error bounds (its running error analysis, R13) cover twice the error an
    FP32 run of the same decisions makes, so a gap beyond the sum of two bounds is resolved by
    FP32 arithmetic and a divergence there is a real one."""
    rs, ro = _fp32_model_errors(make(), dict(params))
    print(f"{name}: largest FP32 error over its bound: scores {rs.max():.3f}, off2 {ro.max():.3f}")
    assert rs.max() <= 0.5 and ro.max() <= 0.5


# --------------------------------------------------------------------------- exhaustive pairs

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_greedy_step_against_exhaustive_pair_search(seed):
    """Plain MMF (one cluster) with Givens rotations on n = 16: at every step, from the state the
    greedy step starts from, every active pair (i, j) with its diagonalizing rotation and either
    elimination gives a loss increment 2 off2_e; the greedy choice is one of them (its recorded
    literal term is recomputed exactly), so the best of all is a lower bound."""
    n = 16
    A = workloads.random_symmetric(n, 0.4, 40 + seed)
    Ad = A.to_dense()
    state = {"M": Ad.copy(), "stage": 0, "rows": None}
    ratios, greedy_sum = [], [0.0]

    def on_step(d):
        if d["stage"] != state["stage"]:
            state["stage"] = d["stage"]
            state["rows"] = d["S"].copy()
        S = state["rows"]
        M = state["M"]
        act = d["active"].copy()
        act[d["e"]] = True                                 # active set before this step
        live = [q for q in range(len(S)) if act[q]]
        best = math.inf
        for a_, b_ in [(a_, b_) for a_ in live for b_ in live if a_ < b_]:
            ids = S[[a_, b_]]
            slab = M[np.ix_(S, ids)]
            O, _ = oracle.rotation_k2(slab.T @ slab)
            Q = np.eye(n)
            Q[np.ix_(ids, ids)] = O
            M1 = Q @ M @ Q.T
            for e in ids:
                col = M1[np.ix_(S, [e])].ravel()
                best = min(best, 2.0 * (float(col @ col) - M1[e, e] ** 2))
        ids = S[d["T"]]
        Q = np.eye(n)
        Q[np.ix_(ids, ids)] = d["O"]
        state["M"] = Q @ M @ Q.T
        e = S[d["e"]]
        col = state["M"][np.ix_(S, [e])].ravel()
        greedy = 2.0 * (float(col @ col) - state["M"][e, e] ** 2)
        assert best <= greedy + 1e-12 * max(1.0, greedy)
        greedy_sum[0] += greedy
        ratios.append((greedy + 1e-300) / (best + 1e-300) if greedy > 1e-14 else 1.0)

    fac = oracle.factor(A, k=2, core=4, seed=seed, on_step=on_step)
    assert len(ratios) == len(fac.rotations) == n - 4
    # the oracle's own literal terms are these increments, formed from its incremental Gram
    assert greedy_sum[0] == pytest.approx(fac.loss_literal, rel=1e-10, abs=1e-12)
    print(f"greedy / exhaustive increment: median {np.median(ratios):.3f}, max {max(ratios):.3f}")
    assert min(ratios) >= 1.0 - 1e-9


# --------------------------------------------------------------------------- several eliminations

def _dense_U(fac):
    U = np.eye(fac.n)
    for r in fac.rotations:
        Q = np.eye(fac.n)
        Q[np.ix_(r.ids, r.ids)] = r.O
        U = Q @ U
    return U


@pytest.mark.parametrize("cluster", [(0, 0), (12, 30)])
def test_two_eliminations_per_rotation_by_brute_force_and_three_way_loss(cluster):
    """k = 3 with two indices retired per rotation (R17) on n = 48: every step's two retirees are
    the two slots with the smallest off-diagonal norms recomputed from the dense current matrix,
    the cluster takes ceil(r_u / 2) rotations, and the exact loss, ||A||^2 - ||H||^2 and the dense
    residual from the log agree."""
    n = 48
    A = workloads.random_symmetric(n, 0.2, 31)
    Ad = A.to_dense()
    state = {"M": Ad.copy(), "stage": 0, "rows": None}
    steps = []

    def on_step(d):
        if d["stage"] != state["stage"]:
            state["stage"] = d["stage"]
            state["rows"] = d["S"].copy()
        S, off = state["rows"], d["offset"]
        c = d["G"].shape[0]
        cols = S[off:off + c]
        ids = cols[np.asarray(d["T"])]
        Q = np.eye(n)
        Q[np.ix_(ids, ids)] = d["O"]
        state["M"] = Q @ state["M"] @ Q.T
        M1 = state["M"]
        off2 = [float(np.sum(M1[np.ix_(S, [g])] ** 2) - M1[g, g] ** 2) for g in ids]
        steps.append((d["stage"], d["cluster"], list(ids), off2))

    fac = oracle.factor(A, k=3, core=8, cluster=cluster, seed=4, elims=2, on_step=on_step)
    assert len(fac.rotations) == n - 8                     # one log entry per retired index
    # entries of a step: the rotation, then the identity block on the same tuple
    real = [r for r in fac.rotations if not np.array_equal(r.O, np.eye(3))]
    assert len(real) == len(steps)
    it = iter(fac.rotations)
    for (p, u, ids, off2) in steps:
        r1 = next(it)
        assert list(r1.ids) == ids
        order = sorted(range(3), key=lambda t: (off2[t], -t))   # smallest first, ties: later slot
        assert r1.retired == ids[order[0]]
        st = fac.stages[p - 1]
        # a second entry unless this was the cluster's last, odd retirement
        nxt = fac.rotations.index(r1) + 1
        if nxt < len(fac.rotations) and list(fac.rotations[nxt].ids) == ids:
            r2 = fac.rotations[nxt]
            np.testing.assert_array_equal(r2.O, np.eye(3))
            rest = [t for t in range(3) if t != order[0]]
            second = min(rest, key=lambda t: (off2[t], -t))
            assert r2.retired == ids[second]
            next(it)
    for st in fac.stages:
        for ru, c in zip(st["cluster_rotations"], st["cluster_sizes"]):
            assert ru <= c - 2
    U = _dense_U(fac)
    H = np.diag(fac.hdiag)
    H[np.ix_(fac.core_ids, fac.core_ids)] = fac.hcore
    dense = float(((Ad - U.T @ H @ U) ** 2).sum())
    scale = float((Ad ** 2).sum())
    assert abs(fac.loss - dense) <= 1e-10 * scale
    assert abs(fac.loss - (scale - float((H ** 2).sum()))) <= 1e-10 * scale
    np.testing.assert_allclose(U @ U.T, np.eye(n), atol=1e-12)


def test_several_eliminations_bounds_and_default():
    A = workloads.random_symmetric(30, 0.2, 3)
    with pytest.raises(ValueError):
        oracle.factor(A, k=2, core=6, elims=2)
    a = oracle.factor(A, k=3, core=6, elims=1)
    b = oracle.factor(A, k=3, core=6)
    assert a.loss == b.loss
    np.testing.assert_array_equal(a.retired_order, b.retired_order)
