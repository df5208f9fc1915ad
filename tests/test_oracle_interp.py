"""Pins of the oracle's classical, extended+i and hybrid interpolations
(Section 2, Interpolation; Alg. extintset) against facts fixed outside the
oracle: the interpolatory sets the paper states for Fig. intset, hand-worked
values on a four-point chain, linear interpolation on the 1D Laplacian,
exact interpolation of constants on rows with zero sum, the covering
property Alg. extintset guarantees, and the two-grid iteration matrix."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB
from tests.helpers import dense, from_dense, rows_sorted

GOLD = os.path.join(os.path.dirname(__file__), "golden")
VARIANTS = {"classical": O.INTERP_CLASSICAL, "exti": O.INTERP_EXTI, "hybrid": O.INTERP_HYBRID}


def _interp_dense(A, cf, variant):
    s, _ = O.strength(A)
    P = O.interp(A, s, np.asarray(cf, np.int8), variant)
    assert rows_sorted(P)
    return dense(P)


# ----------------------------------------------------------------- Fig. intset
def _fig_intset():
    nodes, edges, sets = {}, [], {}
    with open(os.path.join(GOLD, "fig_intset.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "node":
                nodes[t[1]] = t[4]
            elif t[0] == "edge":
                edges.append((t[1], t[2]))
            elif t[0] == "set":
                sets[t[1]] = set(t[2:])
    names = list(nodes)
    idx = {nm: k for k, nm in enumerate(names)}
    n = len(names)
    M = np.zeros((n, n))
    for a, b in edges:
        M[idx[a], idx[b]] = M[idx[b], idx[a]] = -1.0
    M[np.arange(n), np.arange(n)] = -M.sum(1) + 1.0   # graph Laplacian + I: SPD, every edge strong
    cf = np.array([1 if nodes[nm] == "C" else -1 for nm in names], np.int8)
    return names, idx, from_dense(M), cf, sets


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_fig_intset_sets(variant):
    names, idx, A, cf, sets = _fig_intset()
    D = _interp_dense(A, cf, VARIANTS[variant])
    coarse = [nm for nm in names if cf[idx[nm]] == 1]     # coarse numbering keeps the fine order
    got = {coarse[c] for c in np.nonzero(D[idx["i"]])[0]}
    assert got == sets[variant]


def test_fig_intset_nested_and_covering():
    """C_i^S is inside the hybrid set, which is inside the extended set, and
    after Alg. extintset every strong F neighbour of i with a strong C
    neighbour has one in the hybrid set."""
    names, idx, A, cf, sets = _fig_intset()
    assert sets["classical"] <= sets["hybrid"] <= sets["exti"]
    Ad = dense(A)
    coarse = [nm for nm in names if cf[idx[nm]] == 1]
    for nm in names:
        if cf[idx[nm]] != -1 or Ad[idx["i"], idx[nm]] == 0:
            continue
        mine = {coarse.index(c) for c in sets["hybrid"]}
        theirs = {coarse.index(c) for c in coarse if Ad[idx[nm], idx[c]] != 0}
        assert not theirs or mine & theirs


# ----------------------------------------------------------------- hand-worked values
# Four points 0 - 1 - 2 - 3 with C = {0, 3}, F = {1, 2}:
#     [ 2   -1   0.5  0 ]
#     [-1    3  -1    0 ]
#     [ 0.5 -1   3   -1 ]
#     [ 0    0  -1    2 ]
# theta = 0.25: S_1 = {0, 2}, S_2 = {1, 3} (the positive coupling a_20 is not
# strong).  The sign filter drops a_20 from row 2 (abar_20 = 0), and a_13 is
# not stored (abar_13 = 0).
#
# classical, row 1: C_1^S = {0}; k = 2 has abar_20 = 0, so 2 is in F_1^{S*}
#   and lumped: d = 3 - 1 = 2, w_10 = -a_10 / d = 1/2.
# classical, row 2: C_2^S = {3}; k = 1 has abar_13 = 0 (lumped), 0 is weak:
#   d = 3 + 0.5 - 1 = 2.5, w_23 = 1/2.5 = 0.4.
# extended+i, row 1: set {0, 3}; k = 2: D = abar_20 + abar_21 + abar_23 = -2;
#   num_0 = -1 + (-1)(0)/(-2) = -1, num_3 = 0 + (-1)(-1)/(-2) = -1/2,
#   a~_11 = 3 + (-1)(-1)/(-2) = 2.5: w_10 = 0.4, w_13 = 0.2.
# extended+i, row 2: set {0, 3} (0 enters through C_1^S and is a weak
#   neighbour, so a_20 stays in the numerator); k = 1: D = abar_10 + abar_12
#   (+ abar_13 = 0) = -2; num_0 = 0.5 + (-1)(-1)/(-2) = 0, num_3 = -1,
#   a~_22 = 3 + (-1)(-1)/(-2) = 2.5: w_20 = 0 (kept as a structural entry),
#   w_23 = 0.4.
# hybrid: in both rows the only strong F neighbour has no strong connection
#   to C_i^S and a single strong C neighbour, which is added: same sets and
#   weights as extended+i.
CHAIN = [[2, -1, 0.5, 0], [-1, 3, -1, 0], [0.5, -1, 3, -1], [0, 0, -1, 2]]
CHAIN_CF = [1, -1, -1, 1]
CHAIN_P = {
    "classical": [[1, 0], [0.5, 0], [0, 0.4], [0, 1]],
    "exti": [[1, 0], [0.4, 0.2], [0.0, 0.4], [0, 1]],
    "hybrid": [[1, 0], [0.4, 0.2], [0.0, 0.4], [0, 1]],
}
CHAIN_NNZ = {"classical": [1, 1, 1, 1], "exti": [1, 2, 2, 1], "hybrid": [1, 2, 2, 1]}


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_chain_hand_values(variant):
    A = from_dense(CHAIN)
    s, _ = O.strength(A)
    # stored entries row by row: (0,0) (0,1) (0,2) | (1,0) (1,1) (1,2) | (2,0) (2,1) (2,2) (2,3) | (3,2) (3,3)
    assert s.tolist() == [0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 1, 0]
    P = O.interp(A, s, np.array(CHAIN_CF, np.int8), VARIANTS[variant])
    assert np.diff(P[2]).tolist() == CHAIN_NNZ[variant]
    np.testing.assert_allclose(dense(P), np.array(CHAIN_P[variant]), rtol=1e-15, atol=0)


@pytest.mark.parametrize("variant,w", [("classical", [1.0]), ("exti", [2 / 3, 1 / 3]),
                                       ("hybrid", [2 / 3, 1 / 3])])
def test_laplacian_1d_linear(variant, w):
    """1D Laplacian (2, -1) with C F F C F F C ...: extended+i reproduces
    linear interpolation between the two C points around an F pair; the
    classical formula sees one C point and lumps the other F point."""
    n = 3 * 6 + 1
    M = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    cf = np.where(np.arange(n) % 3 == 0, 1, -1)
    D = _interp_dense(from_dense(M), cf, VARIANTS[variant])
    for i in range(1, n - 1):
        if cf[i] == 1:
            continue
        near, far = (i // 3, i // 3 + 1) if i % 3 == 1 else (i // 3 + 1, i // 3)
        row = D[i]
        assert row[near] == pytest.approx(w[0], rel=1e-15)
        if len(w) > 1:
            assert row[far] == pytest.approx(w[1], rel=1e-15)
            assert np.count_nonzero(row) == 2
        else:
            assert np.count_nonzero(row) == 1


# ----------------------------------------------------------------- invariants on PMIS splits
def _int_laplacian(shape, rng):
    """Graph Laplacian of a 2D/3D grid with random integer edge weights
    1..9; boundary rows get +1 on the diagonal.  Interior rows sum to
    exactly zero in floating point."""
    nd = len(shape)
    n = int(np.prod(shape))
    M = np.zeros((n, n))
    ids = np.arange(n).reshape(shape[::-1])
    for ax in range(nd):
        a = np.take(ids, range(0, ids.shape[ax] - 1), axis=ax).ravel()
        b = np.take(ids, range(1, ids.shape[ax]), axis=ax).ravel()
        wts = rng.integers(1, 10, size=a.size).astype(float)
        M[a, b] -= wts
        M[b, a] -= wts
    M[np.arange(n), np.arange(n)] = -M.sum(1)
    interior = np.ones(ids.shape, bool)
    for ax in range(nd):
        sl = [slice(None)] * nd
        sl[ax] = 0
        interior[tuple(sl)] = False
        sl[ax] = -1
        interior[tuple(sl)] = False
    M[np.arange(n), np.arange(n)] += (~interior.ravel()).astype(float)
    return M, interior.ravel()


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("shape", [(14, 13), (7, 6, 6)])
def test_constants_interpolated_exactly(variant, shape):
    rng = np.random.default_rng(11)
    M, interior = _int_laplacian(shape, rng)
    A = from_dense(M)
    s, cnt = O.strength(A)
    cf, _ = O.pmis(A, s, cnt, 0, 0)
    P = O.interp(A, s, cf, VARIANTS[variant])
    D = dense(P)
    C = np.where(cf == 1)[0]
    assert np.array_equal(D[C], np.eye(len(C)))
    checked = 0
    for i in np.where((cf == -1) & interior)[0]:
        if np.count_nonzero(D[i]):
            assert abs(D[i].sum() - 1.0) < 1e-13
            assert np.all(D[i][D[i] != 0] > 0)       # M-matrix: positive weights
            checked += 1
    assert checked > 10


@pytest.mark.parametrize("gen", ["p2", "ln3", "an3", "el"])
def test_sets_nested_and_hybrid_covers(gen):
    """Per F row: C_i^S <= hybrid set <= extended set, the extended set is
    C_i^S plus the strong C neighbours of the strong F neighbours, and the
    hybrid set leaves no strong F neighbour with a strong C neighbour
    uncovered."""
    A = {"p2": lambda: PB.poisson2d(16), "ln3": lambda: PB.lognormal3d(7, 2.0),
         "an3": lambda: PB.aniso3d(7), "el": lambda: PB.elasticity3d(2)}[gen]()
    s, cnt = O.strength(A)
    cf, _ = O.pmis(A, s, cnt, 0, 0)
    n = A.n
    S = np.zeros((n, n), bool)
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    S[rows[s == 1], A.col_idx[s == 1]] = True
    Cf = np.where(cf == 1)[0]
    sets = {}
    for name, var in VARIANTS.items():
        D = dense(O.interp(A, s, cf, var))
        sets[name] = [set(Cf[np.nonzero(D[i])[0]]) if cf[i] == -1 else None for i in range(n)]
    isC = cf == 1
    for i in np.where(cf == -1)[0]:
        cs = set(np.where(S[i] & isC)[0])
        fs = np.where(S[i] & ~isC)[0]
        ext = set(cs)
        for k in fs:
            ext |= set(np.where(S[k] & isC)[0])
        assert sets["classical"][i] == cs
        assert sets["exti"][i] == ext
        hy = sets["hybrid"][i]
        assert cs <= hy <= ext
        for k in fs:
            ck = set(np.where(S[k] & isC)[0])
            assert not ck or ck & hy


# ----------------------------------------------------------------- hierarchies
def _M_recursive(Al, Ps, omegas, l):
    if l == len(Ps):
        return np.linalg.inv(Al)
    P = Ps[l]
    Mc = _M_recursive(P.T @ Al @ P, Ps, omegas, l + 1)
    n = Al.shape[0]
    S = np.eye(n) - omegas[l] * Al / np.diag(Al)[:, None]
    E = S @ (np.eye(n) - P @ Mc @ P.T @ Al) @ S
    return (np.eye(n) - E) @ np.linalg.inv(Al)


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("gen", ["ln2", "el"])
def test_vcycle_matches_iteration_matrix(variant, gen):
    A = {"ln2": lambda: PB.lognormal2d(11, 2.0), "el": lambda: PB.elasticity3d(2)}[gen]()
    h = O.Hierarchy(A, max_coarse=12, interp=VARIANTS[variant])
    assert h.nlev >= 2
    Ps = [dense(h.P(l)) for l in range(h.nlev - 1)]
    om = [h.omega(l) for l in range(h.nlev - 1)]
    M = _M_recursive(dense(A), Ps, om, 0)
    Mo = np.stack([h.vcycle(e) for e in np.eye(A.n)], axis=1)
    np.testing.assert_allclose(Mo, M, rtol=0, atol=1e-12 * np.abs(M).max())


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_pcg_converges_and_exti_beats_direct(variant):
    A = PB.lognormal3d(12, 2.0)
    b = PB.rhs(A.n)
    xs = np.linalg.solve(dense(A), b)
    its = {}
    for name, var in (("direct", O.INTERP_DIRECT), (variant, VARIANTS[variant])):
        h = O.Hierarchy(A, max_coarse=40, interp=var)
        r = h.solve(b, 1e-8)
        assert r.status == O.OK
        assert np.linalg.norm(b - dense(A) @ r.x) < 1e-8 * np.linalg.norm(b) * 1.0001
        assert np.linalg.norm(r.x - xs) <= 1e-5 * np.linalg.norm(xs)
        its[name] = r.iters
    if variant == "exti":
        assert its["exti"] < its["direct"]


def test_hybrid_tie_takes_smallest_index():
    """Alg. extintset leaves ties between candidates of equal degree open;
    the reading here takes the smallest index.  Graph 0-1, 1-2, 2-3, 2-4
    with C = {0, 3, 4}: row 1 has C_1^S = {0} and the F neighbour 2, whose
    strong C neighbours 3 and 4 both cover it."""
    n = 5
    M = np.zeros((n, n))
    for a, b in [(0, 1), (1, 2), (2, 3), (2, 4)]:
        M[a, b] = M[b, a] = -1.0
    M[np.arange(n), np.arange(n)] = -M.sum(1) + 1.0
    cf = [1, -1, -1, 1, 1]
    A = from_dense(M)
    want = {"classical": [0], "exti": [0, 1, 2], "hybrid": [0, 1]}   # coarse numbering of 0, 3, 4
    for name, var in VARIANTS.items():
        D = _interp_dense(A, cf, var)
        assert np.nonzero(D[1])[0].tolist() == want[name]
