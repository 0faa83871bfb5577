"""Pins for the FP64 oracle: checks against what the paper and the mathematics fix.

None of these re-types the oracle's formulas.  They compare it with published test vectors, hand
computations, LAPACK, brute force over all choices on tiny inputs, dense matrix products built
here from the rotation log, closed-form invariants, and special cases whose answer is known.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import oracle.pmmf_oracle as om
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MASK = (1 << 64) - 1


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --------------------------------------------------------------------------- RNG

def test_mix64_matches_published_splitmix64_outputs():
    expect = [int(r[0]) for r in _golden_rows("splitmix64_seed1234567.txt")]
    state = 1234567
    got = []
    for _ in range(5):
        state = (state + om.GOLDEN64) & MASK
        got.append(oracle.mix64(state))
    assert got == expect


def test_chain_hash_is_a_splitmix_step_per_value():
    # one value v = 0 from x = seed is exactly the first SplitMix64 output of state seed
    assert oracle.chain_hash(1234567, 0) == 6457827717110365317


def test_mulhi_maps_to_range():
    assert oracle.mulhi(0, 7) == 0
    assert oracle.mulhi(MASK, 7) == 6
    assert oracle.mulhi(1 << 63, 10) == 5
    assert oracle.mulhi(1 << 62, 8) == 2
    rng = np.random.default_rng(0)
    for _ in range(200):
        x = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        n = int(rng.integers(1, 5000))
        assert 0 <= oracle.mulhi(x, n) < n
        assert oracle.mulhi(x, n) == (x * n) // (1 << 64)


# --------------------------------------------------------------------------- schedule

def test_stage_schedule_hand_examples():
    assert oracle.stage_schedule(512, 64, 0.5) == [(512, 256), (256, 128), (128, 64)]
    # 100 -> 50 -> 25 -> 13 (t = floor(12.5)) -> 10 (t = |S| - core = 3)
    assert oracle.stage_schedule(100, 10, 0.5) == [(100, 50), (50, 25), (25, 12), (13, 3)]
    assert oracle.stage_schedule(64, 64, 0.5) == []
    with pytest.raises(ValueError):
        oracle.stage_schedule(10, 9, 0.05)  # floor(0.05 * 10) = 0 cannot make progress


def test_allocate_rotations_largest_remainder_by_hand():
    # t = 5 over sizes (3, 3, 4): shares 1.5, 1.5, 2.0 -> floors (1, 1, 2), one leftover to the
    # largest remainder; clusters 0 and 1 tie, the lower index wins
    assert oracle.allocate_rotations(5, [3, 3, 4]) == [2, 1, 2]
    assert oracle.allocate_rotations(7, [5, 5]) == [4, 3]
    assert oracle.allocate_rotations(0, [5, 5]) == [0, 0]


@pytest.mark.parametrize("total,lo,hi", [(65536, 256, 2048), (1000, 10, 40), (95, 10, 20),
                                         (41, 10, 40), (5, 10, 40)])
def test_cluster_sizes_bounds(total, lo, hi):
    for p in range(1, 4):
        s = oracle.cluster_sizes(total, lo, hi, seed=3, p=p)
        assert sum(s) == total
        for c in s[:-1]:
            assert lo <= c <= hi
        assert s[-1] <= hi
        if total >= lo:
            assert s[-1] >= lo
        r = oracle.allocate_rotations(total // 2, s)
        assert sum(r) == total // 2
        for c, ru in zip(s, r):
            share = (total // 2) * c / total
            assert math.floor(share) <= ru <= math.ceil(share)


# --------------------------------------------------------------------------- rotations

def test_rotation_k2_hand_value():
    row = [float(x) for x in _golden_rows("givens_2x2_tau0.txt")[0]]
    g = np.array([[row[0], row[1]], [row[1], row[2]]])
    O, _ = oracle.rotation_k2(g)
    np.testing.assert_allclose(O, [[row[3], -row[4]], [row[4], row[3]]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(O @ g @ O.T, np.diag([row[5], row[6]]), atol=1e-14)


def test_rotation_k2_is_the_eigenbasis_closest_to_identity():
    rng = np.random.default_rng(1)
    for _ in range(300):
        a = rng.standard_normal((2, 5)) * rng.uniform(0.01, 10)
        g = a @ a.T
        O, _ = oracle.rotation_k2(g)
        np.testing.assert_allclose(O @ O.T, np.eye(2), atol=1e-14)
        d = O @ g @ O.T
        assert abs(d[0, 1]) <= 1e-13 * np.abs(g).max()
        assert abs(math.atan2(O[1, 0], O[0, 0])) <= math.pi / 4 + 1e-12
        # rows are LAPACK eigenvectors up to order and sign
        w, v = np.linalg.eigh(g)
        assert np.allclose(np.abs(O @ v), np.eye(2)[::-1], atol=1e-9) or \
            np.allclose(np.abs(O @ v), np.eye(2), atol=1e-9)
        # the k-point rule (max trace, nonnegative diagonal) reduces to the same rotation
        O3, _ = oracle.rotation_k3(g)
        np.testing.assert_allclose(O3, O, atol=1e-12)


def test_rotation_k2_zero_coupling_is_identity():
    O, _ = oracle.rotation_k2(np.array([[3.0, 0.0], [0.0, 1.0]]))
    assert np.array_equal(O, np.eye(2))


def test_rotation_k3_maximizes_trace_over_all_signed_permutations():
    rng = np.random.default_rng(2)
    for _ in range(100):
        a = rng.standard_normal((3, 6))
        g = a @ a.T
        O, _ = oracle.rotation_k3(g)
        np.testing.assert_allclose(O @ O.T, np.eye(3), atol=1e-13)
        d = O @ g @ O.T
        assert np.abs(d - np.diag(np.diag(d))).max() <= 1e-12 * np.abs(g).max()
        assert np.all(np.diag(O) >= 0)
        w, v = np.linalg.eigh(g)
        best = -1.0
        for perm in itertools.permutations(range(3)):
            for signs in itertools.product([1, -1], repeat=3):
                cand = np.array([signs[r] * v[:, perm[r]] for r in range(3)])
                best = max(best, float(np.trace(cand)))
        assert np.trace(O) >= best - 1e-12


# --------------------------------------------------------------------------- factorization

def _dense_rotation(n, ids, O):
    Q = np.eye(n)
    Q[np.ix_(ids, ids)] = O
    return Q


def _dense_U_from_log(fac):
    U = np.eye(fac.n)
    for r in fac.rotations:
        U = _dense_rotation(fac.n, r.ids, r.O) @ U
    return U


def _dense_H(fac):
    H = np.diag(fac.hdiag)
    H[np.ix_(fac.core_ids, fac.core_ids)] = fac.hcore
    return H


CASES = [
    ("rand48_k2_single", lambda: workloads.random_symmetric(48, 0.15, 5), dict(k=2, core=8)),
    ("rand48_k3_single", lambda: workloads.random_symmetric(48, 0.15, 6), dict(k=3, core=8)),
    ("grid8x8_k2_clusters", lambda: workloads.small_grid((8, 8), seed=7),
     dict(k=2, core=6, cluster=(6, 16))),
    ("knn64_k3_clusters", lambda: workloads.knn_points_matrix(64, 2, 5, 0.05, 8),
     dict(k=3, core=10, cluster=(8, 20), seed=4)),
    ("grid6x7_eta03", lambda: workloads.small_grid((6, 7), seed=9),
     dict(k=2, core=5, eta=0.3, cluster=(4, 12), seed=11)),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def small_case(request):
    name, make, params = request.param
    A = make()
    fac = oracle.factor(A, **params)
    return A.to_dense(), fac, params


def test_loss_three_way_identity(small_case):
    Ad, fac, _ = small_case
    U = _dense_U_from_log(fac)
    H = _dense_H(fac)
    dense = float(((Ad - U.T @ H @ U) ** 2).sum())
    fro_gap = float((Ad ** 2).sum() - (H ** 2).sum())
    scale = float((Ad ** 2).sum())
    assert abs(fac.loss - dense) <= 1e-10 * scale
    assert abs(fac.loss - fro_gap) <= 1e-10 * scale
    assert fac.loss_literal >= fac.loss - 1e-12 * scale


def test_trace_and_frobenius_preserved(small_case):
    Ad, fac, _ = small_case
    H = _dense_H(fac)
    assert abs(np.trace(H) - np.trace(Ad)) <= 1e-11 * np.abs(Ad).sum()
    for st in fac.stages:
        assert abs(st["fro_start"] - st["fro_end"]) <= 1e-12 * st["fro_start"]
        assert st["hdiag_check"] <= 1e-12 * np.abs(Ad).max()


def test_rotations_orthogonal_and_active_sets_nested(small_case):
    Ad, fac, params = small_case
    n = fac.n
    seen = set()
    for r in fac.rotations:
        k = len(r.ids)
        np.testing.assert_allclose(r.O @ r.O.T, np.eye(k), atol=1e-14)
        assert len(set(r.ids.tolist())) == k
        assert r.retired in r.ids
        # Q_l is the identity off the active set: no rotation touches a retired index
        assert not (set(r.ids.tolist()) & seen)
        seen.add(r.retired)
    sizes = [st["size"] for st in fac.stages]
    sched = oracle.stage_schedule(n, params["core"], params.get("eta", 0.5))
    assert sizes == [s for s, _ in sched]
    assert len(seen) == n - params["core"]
    assert sorted(seen | set(fac.core_ids.tolist())) == list(range(n))
    assert np.all(fac.hdiag[fac.core_ids] == 0)


def test_stage_rotations_block_diagonal(small_case):
    """Every stage Q_p is block diagonal in that stage's clusters (Def. 1)."""
    Ad, fac, _ = small_case
    n = fac.n
    for st in fac.stages:
        p = st["stage"]
        label = -np.ones(n, dtype=int)
        for u in range(len(st["cluster_sizes"])):
            label[st["active"][st["offsets"][u]:st["offsets"][u + 1]]] = u
        Q = np.eye(n)
        for r in fac.rotations:
            if r.stage == p:
                assert len(set(label[r.ids].tolist())) == 1
                assert label[r.ids[0]] == r.cluster
                Q = _dense_rotation(n, r.ids, r.O) @ Q
        same = label[:, None] == label[None, :]
        same |= np.eye(n, dtype=bool)
        assert np.abs(Q[~same]).max(initial=0.0) == 0.0


def test_deterministic(small_case):
    Ad, fac, params = small_case
    fac2 = oracle.factor(workloads.csr_from_dense(Ad), **params)
    assert [r.ids.tolist() for r in fac.rotations] == [r.ids.tolist() for r in fac2.rotations]
    assert fac.loss == fac2.loss


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("cluster", [(0, 0), (4, 8)])
def test_gram_recursion_and_greedy_choices_by_brute_force(k, cluster):
    """n <= 16: every step's Gram and diagonal block equal a recomputation from the dense current
    matrix, and the chosen tuple / eliminated index are the brute-force optimum of the rules."""
    n = 16
    A = workloads.random_symmetric(n, 0.35, 21 + k)
    Ad = A.to_dense()
    state = {"M": Ad.copy(), "stage": 0, "rows": None}
    checks = []

    def on_step(d):
        if d["stage"] != state["stage"]:
            state["stage"] = d["stage"]
            state["rows"] = d["S"].copy()                 # S_{p-1}, global ids
        S = state["rows"]
        off = d["offset"]
        G, D, T, O, e = d["G"], d["D"], d["T"], d["O"], d["e"]
        c = G.shape[0]
        cols = S[off:off + c]
        M = state["M"]
        pre_M = M.copy()
        # apply this rotation to the dense current matrix from both sides
        ids = cols[np.asarray(T)]
        Q = _dense_rotation(n, ids, O)
        state["M"] = Q @ M @ Q.T
        M1 = state["M"]
        slab = M1[np.ix_(S, cols)]
        np.testing.assert_allclose(G, slab.T @ slab, atol=1e-12 * max(1.0, np.abs(G).max()))
        np.testing.assert_allclose(D, M1[np.ix_(cols, cols)], atol=1e-12)
        # brute force over the choices the rules allow, from the state before the rotation
        slab0 = pre_M[np.ix_(S, cols)]
        G0 = slab0.T @ slab0
        active_before = d["active"].copy()
        active_before[e] = True
        i = T[0]
        cand = [j for j in range(c) if active_before[j] and j != i]
        sc = {j: (abs(G0[i, j]) / math.sqrt(G0[j, j]) if G0[j, j] > 0 else 0.0) for j in cand}
        want = sorted(cand, key=lambda j: (-sc[j], j))[:len(T) - 1]
        assert T[1:] == want
        off2 = [np.sum(M1[np.ix_(S, [cols[t]])] ** 2) - M1[cols[t], cols[t]] ** 2 for t in T]
        best = min(off2)
        later = max(sl for sl in range(len(T)) if off2[sl] <= best + 1e-12 * max(1.0, best))
        assert T.index(e) == later
        checks.append(1)

    fac = oracle.factor(A, k=k, core=4, cluster=cluster, seed=5, on_step=on_step)
    assert len(checks) == len(fac.rotations) == n - 4


def test_special_case_diagonal_matrix_has_zero_loss():
    rng = np.random.default_rng(3)
    A = workloads.csr_from_dense(np.diag(rng.uniform(1, 5, 40)))
    fac = oracle.factor(A, k=2, core=5, cluster=(4, 10))
    assert fac.loss == 0.0
    for r in fac.rotations:
        assert np.array_equal(r.O, np.eye(2))


@pytest.mark.parametrize("k", [2, 3])
def test_special_case_pair_blocks_single_cluster_zero_loss(k):
    A, _ = workloads.block_diag_pairs(64, seed=4)
    fac = oracle.factor(A, k=k, core=8, seed=2)
    assert fac.loss <= 1e-24 * (A.to_dense() ** 2).sum() + 1e-20


def test_special_case_pair_blocks_clusters_one_stage_zero_loss():
    # adjacent pairs, even cluster sizes, one stage (core = n / 2): no pair straddles a cluster
    n = 96
    A, _ = workloads.block_diag_pairs(n, seed=5, permute=False)
    fac = oracle.factor(A, k=2, core=n // 2, cluster=(6, 16), seed=3, even_clusters=True)
    assert fac.num_stages == 1
    assert fac.loss <= 1e-20 * (A.to_dense() ** 2).sum() + 1e-20


def test_special_case_core_equals_n_keeps_A():
    A = workloads.random_symmetric(20, 0.3, 9)
    fac = oracle.factor(A, k=2, core=20)
    assert fac.rotations == [] and fac.loss == 0.0
    np.testing.assert_array_equal(fac.hcore, A.to_dense())


def test_rejects_nonsymmetric_and_bad_params():
    a = np.arange(16.0).reshape(4, 4)
    with pytest.raises(ValueError):
        oracle.factor(a, core=2)
    A = workloads.random_symmetric(10, 0.5, 1)
    with pytest.raises(ValueError):
        oracle.factor(A, k=4, core=2)
    with pytest.raises(ValueError):
        oracle.factor(A, core=2, cluster=(4, 6))
    with pytest.raises(ValueError):
        oracle.factor(A, core=0)


# --------------------------------------------------------------------------- matrix-free use

def test_apply_matches_dense_product_from_the_log(small_case):
    Ad, fac, _ = small_case
    U = _dense_U_from_log(fac)
    H = _dense_H(fac)
    X = np.random.default_rng(4).standard_normal((fac.n, 3))
    np.testing.assert_allclose(oracle.apply(fac, X), U.T @ H @ U @ X, atol=1e-11 * np.abs(Ad).max())
    np.testing.assert_allclose(oracle.apply_U(fac, X), U @ X, atol=1e-13)
    np.testing.assert_allclose(oracle.apply_Ut(fac, X), U.T @ X, atol=1e-13)


def test_apply_is_symmetric_and_inverse_inverts():
    A = workloads.small_grid((7, 9), sigma=0.7, shift=0.5, seed=12)   # SPD
    fac = oracle.factor(A, k=2, core=9, cluster=(6, 20), seed=1)
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(fac.n), rng.standard_normal(fac.n)
    assert abs(x @ oracle.apply(fac, y) - y @ oracle.apply(fac, x)) <= 1e-12 * np.abs(x).sum()
    Xb = rng.standard_normal((fac.n, 4))
    np.testing.assert_allclose(oracle.apply_inverse(fac, oracle.apply(fac, Xb)), Xb, atol=1e-10)
    U = _dense_U_from_log(fac)
    Atil = U.T @ _dense_H(fac) @ U
    np.testing.assert_allclose(oracle.apply_inverse(fac, Xb), np.linalg.solve(Atil, Xb),
                               rtol=1e-9, atol=1e-11)


def test_inverse_square_root_pins():
    """A~^{-1/2} (Sec. 4, xi = 1/2) against independent routes: its square is the Cholesky-based
    A~^{-1}, it is symmetric, A~^{-1/2} A~ A~^{-1/2} = I, and it equals SciPy's inverse of the
    dense matrix square root of A~ rebuilt from the log."""
    import scipy.linalg as sla
    A = workloads.small_grid((7, 9), sigma=0.7, shift=0.5, seed=12)   # SPD
    fac = oracle.factor(A, k=2, core=9, cluster=(6, 20), seed=1)
    rng = np.random.default_rng(8)
    Xb = rng.standard_normal((fac.n, 4))
    S = lambda Z: oracle.apply_inverse_sqrt(fac, Z)  # noqa: E731
    np.testing.assert_allclose(S(S(Xb)), oracle.apply_inverse(fac, Xb), rtol=1e-9, atol=1e-11)
    x, y = rng.standard_normal(fac.n), rng.standard_normal(fac.n)
    assert abs(x @ S(y) - y @ S(x)) <= 1e-12 * np.abs(x).sum() * np.abs(y).max()
    np.testing.assert_allclose(S(oracle.apply(fac, S(Xb))), Xb, atol=1e-10)
    U = _dense_U_from_log(fac)
    Atil = U.T @ _dense_H(fac) @ U
    ref = np.linalg.solve(np.real(sla.sqrtm(Atil)), Xb)
    np.testing.assert_allclose(S(Xb), ref, rtol=1e-8, atol=1e-10)
    # an indefinite H is refused
    bad = om.with_angles(fac, om.angles(fac), hcore=-np.eye(len(fac.core_ids)))
    with pytest.raises(ValueError):
        oracle.apply_inverse_sqrt(bad, Xb)


# --------------------------------------------------------------------------- adjoint

def _objective(fac, X, W):
    return float((W * oracle.apply(fac, X)).sum())


def test_backward_matches_central_finite_differences():
    A = workloads.small_grid((5, 6), seed=13)
    fac = oracle.factor(A, k=2, core=6, cluster=(4, 10), seed=2)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((fac.n, 3))
    W = rng.standard_normal((fac.n, 3))
    xbar, hdbar, hcbar, thbar = oracle.backward(fac, X, W)
    th = om.angles(fac)
    h = 1e-6
    for t in range(len(th)):
        e = np.zeros_like(th)
        e[t] = h
        fd = (_objective(om.with_angles(fac, th + e), X, W)
              - _objective(om.with_angles(fac, th - e), X, W)) / (2 * h)
        assert abs(fd - thbar[t]) <= 1e-6 * max(1.0, abs(fd))
    retired = np.setdiff1d(np.arange(fac.n), fac.core_ids)
    for e_id in retired[:8]:
        hd = fac.hdiag.copy()
        hd[e_id] += h
        hm = fac.hdiag.copy()
        hm[e_id] -= h
        fd = (_objective(om.with_angles(fac, th, hdiag=hd), X, W)
              - _objective(om.with_angles(fac, th, hdiag=hm), X, W)) / (2 * h)
        assert abs(fd - hdbar[e_id]) <= 1e-6 * max(1.0, abs(fd))
    for (a, b) in [(0, 0), (1, 3), (4, 2), (5, 5)]:
        hp = fac.hcore.copy()
        hp[a, b] += h
        hm = fac.hcore.copy()
        hm[a, b] -= h
        fd = (_objective(om.with_angles(fac, th, hcore=hp), X, W)
              - _objective(om.with_angles(fac, th, hcore=hm), X, W)) / (2 * h)
        assert abs(fd - hcbar[a, b]) <= 1e-6 * max(1.0, abs(fd))
    d = rng.standard_normal(X.shape)
    fd = _objective(fac, X + d, W) - _objective(fac, X, W)          # linear in X: exact
    assert abs(fd - float((xbar * d).sum())) <= 1e-10 * max(1.0, abs(fd))


@pytest.mark.parametrize("scale", [0.0, 0.3])
def test_backward_k3_angle_gradient_matches_central_finite_differences(scale):
    # R15: 3-point rotations O_t(w) = expm(W(w_t)) O0_t; the gradient in w at w = 0 and at a
    # random w (where the derivative of the exponential map is not the identity)
    A = workloads.small_grid((5, 6), seed=13)
    fac0 = oracle.factor(A, k=3, core=6, cluster=(4, 10), seed=2)
    rng = np.random.default_rng(7)
    R = len(fac0.rotations)
    w0 = scale * rng.standard_normal((R, 3))
    X = rng.standard_normal((fac0.n, 3))
    W = rng.standard_normal((fac0.n, 3))
    fac = om.with_params3(fac0, w0)
    _, _, _, thbar = oracle.backward(fac, X, W, theta=w0)
    assert thbar.shape == (R, 3)
    h = 1e-6
    for t in range(R):
        for m in range(3):
            e = np.zeros_like(w0)
            e[t, m] = h
            fd = (_objective(om.with_params3(fac0, w0 + e), X, W)
                  - _objective(om.with_params3(fac0, w0 - e), X, W)) / (2 * h)
            assert abs(fd - thbar[t, m]) <= 1e-6 * max(1.0, abs(fd)), (t, m, fd, thbar[t, m])


def test_rot3_parametrization_pins():
    # G_01 is the Givens generator in slots (0, 1); W(w) is skew; expm(W) is a rotation; B(0) = I
    G = om.rot3_generators()
    assert np.array_equal(G[0][:2, :2], np.array([[0.0, -1.0], [1.0, 0.0]]))
    w = np.array([0.4, -1.1, 0.7])
    Wm = om.rot3_param_matrix(w)
    assert np.array_equal(Wm, -Wm.T)
    import scipy.linalg
    Q = scipy.linalg.expm(Wm)
    assert np.allclose(Q @ Q.T, np.eye(3), atol=1e-14) and abs(np.linalg.det(Q) - 1) < 1e-14
    assert np.array_equal(om.rot3_param_jacobian(np.zeros(3)), np.eye(3))
    # a rotation about a single plane: the exponential map is linear along it (B w = w)
    assert np.allclose(om.rot3_param_jacobian(np.array([0.0, 0.9, 0.0])) @ [0, 1, 0], [0, 1, 0])


def test_backward_matches_torch_autograd_fp64():
    torch = pytest.importorskip("torch")
    A = workloads.small_grid((6, 6), seed=14)
    fac = oracle.factor(A, k=2, core=6, cluster=(4, 12), seed=3)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((fac.n, 2))
    W = rng.standard_normal((fac.n, 2))
    xbar, hdbar, hcbar, thbar = oracle.backward(fac, X, W)

    th = torch.tensor(om.angles(fac), dtype=torch.float64, requires_grad=True)
    hd = torch.tensor(fac.hdiag, dtype=torch.float64, requires_grad=True)
    hc = torch.tensor(fac.hcore, dtype=torch.float64, requires_grad=True)
    xt = torch.tensor(X, dtype=torch.float64, requires_grad=True)
    core = torch.tensor(fac.core_ids)
    mask = torch.ones(fac.n, dtype=torch.bool)
    mask[core] = False
    rows = [xt[i] for i in range(fac.n)]
    for t, r in enumerate(fac.rotations):          # z <- Q_t z, one Givens at a time
        i, j = int(r.ids[0]), int(r.ids[1])
        c, s = torch.cos(th[t]), torch.sin(th[t])
        rows[i], rows[j] = c * rows[i] - s * rows[j], s * rows[i] + c * rows[j]
    z = torch.stack(rows)
    w = torch.where(mask[:, None], hd[:, None] * z, torch.zeros_like(z))
    w = w.index_put((core,), hc @ z[core])
    rows = [w[i] for i in range(fac.n)]
    for t in range(len(fac.rotations) - 1, -1, -1):   # y <- Q_t^T y in reverse
        r = fac.rotations[t]
        i, j = int(r.ids[0]), int(r.ids[1])
        c, s = torch.cos(th[t]), torch.sin(th[t])
        rows[i], rows[j] = c * rows[i] + s * rows[j], -s * rows[i] + c * rows[j]
    y = torch.stack(rows)
    (y * torch.tensor(W)).sum().backward()
    np.testing.assert_allclose(thbar, th.grad.numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(xbar, xt.grad.numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(hdbar[mask.numpy()], hd.grad.numpy()[mask.numpy()], atol=1e-10)
    np.testing.assert_allclose(hcbar, hc.grad.numpy(), atol=1e-10)

