"""Pins of the oracle's BAMG prolongation (Section 2, Interpolation, eq.
minBAMG and Alg. BAMG) and of the orthonormal test-space basis: exact
linear interpolation on the 1D Laplacian, piecewise-constant rows for a
constant test space, exact reproduction of a linear test space on a 2D grid,
a hand-worked greedy basis choice, the adaptive distance, the two-grid
iteration matrix, and fewer PCG iterations than direct interpolation with
rigid body modes on elasticity."""
import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB
from tests.helpers import dense, from_dense, rows_sorted


def _lap1d(n):
    return from_dense(2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))


# ----------------------------------------------------------------- basis
def test_orthonormalize_basis():
    rng = np.random.default_rng(3)
    V = rng.standard_normal((200, 5))
    Q = O.orthonormalize(V)
    np.testing.assert_allclose(Q.T @ Q, np.eye(5), atol=1e-13)
    # same span: V = Q (Q^T V), and Q^T V is upper triangular (Cholesky-QR)
    Rm = Q.T @ V
    np.testing.assert_allclose(Q @ Rm, V, atol=1e-12)
    assert np.abs(np.tril(Rm, -1)).max() < 1e-12


def test_orthonormalize_rejects_dependent_columns():
    V = np.ones((50, 2))
    with pytest.raises(O.OracleError) as e:
        O.orthonormalize(V)
    assert e.value.status == O.E_ARG


# ----------------------------------------------------------------- closed forms
def test_linear_test_space_1d_is_linear_interpolation():
    """C F F C ... with V = [1, x]: at distance 1 an F point sees one C
    point and cannot reproduce x, so the distance grows to 2, where the two
    C points around the F pair give (2/3, 1/3)."""
    n = 19
    A = _lap1d(n)
    s, _ = O.strength(A)
    cf = np.where(np.arange(n) % 3 == 0, 1, -1).astype(np.int8)
    V = O.orthonormalize(np.stack([np.ones(n), np.arange(n) / n], 1))
    D = dense(O.bamg(A, s, cf, V))
    for i in range(1, n - 1):
        if cf[i] == 1:
            continue
        near, far = (i // 3, i // 3 + 1) if i % 3 == 1 else (i // 3 + 1, i // 3)
        assert D[i, near] == pytest.approx(2 / 3, rel=1e-14)
        assert D[i, far] == pytest.approx(1 / 3, rel=1e-14)
        assert np.count_nonzero(D[i]) == 2
    # distance 1 only: one C point, one entry
    D1 = dense(O.bamg(A, s, cf, V, lmax=1))
    assert all(np.count_nonzero(D1[i]) == 1 for i in range(n) if cf[i] == -1 and 0 < i < n - 1)


def test_constant_test_space_gives_first_strong_c_neighbour():
    """nt = 1, V = 1/sqrt(n): every candidate row has the same norm, so the
    basis is the smallest-index C point at distance 1 and its weight 1."""
    A = PB.poisson2d(12)
    s, cnt = O.strength(A)
    cf, _ = O.pmis(A, s, cnt, 0, 0)
    V = O.orthonormalize(np.ones((A.n, 1)))
    P = O.bamg(A, s, cf, V)
    D = dense(P)
    Cidx = np.where(cf == 1)[0]
    for i in np.where(cf == -1)[0]:
        row = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        st = s[A.row_ptr[i]:A.row_ptr[i + 1]] == 1
        near = [c for c in row[st] if cf[c] == 1 and c != i]
        if not near:
            continue
        assert np.nonzero(D[i])[0].tolist() == [int(np.searchsorted(Cidx, min(near)))]
        assert D[i][D[i] != 0][0] == pytest.approx(1.0, rel=1e-15)


def test_linear_test_space_2d_reproduced():
    """V = [1, x, y] on a 2D 5-point grid: every F row whose basis has three
    points reproduces the test space exactly, so P V_C = V on that row."""
    g = 14
    A = PB.poisson2d(g)
    s, cnt = O.strength(A)
    cf, _ = O.pmis(A, s, cnt, 0, 0)
    x = (np.arange(A.n) % g) / g
    y = (np.arange(A.n) // g) / g
    V = O.orthonormalize(np.stack([np.ones(A.n), x, y], 1))
    P = O.bamg(A, s, cf, V)
    assert rows_sorted(P)
    D = dense(P)
    VC = V[cf == 1]
    full = 0
    for i in np.where(cf == -1)[0]:
        if np.count_nonzero(D[i]) == 3:
            np.testing.assert_allclose(D[i] @ VC, V[i], atol=1e-12)
            full += 1
    assert full > 20
    np.testing.assert_array_equal(D[cf == 1], np.eye(int(np.sum(cf == 1))))


def test_greedy_basis_hand_example():
    """F point 0 with strong C neighbours 1, 2, 3 and test rows
    phi_1 = (1, 0), phi_2 = (0, 2), phi_3 = (1, 1), phi_0 = (1, 1).  The
    largest row is phi_2; after removing its direction phi_1 and phi_3 both
    leave (1, 0), a tie taken by the smaller index 1.  So the basis is
    {1, 2} and phi_0 = 1 phi_1 + 0.5 phi_2, although phi_3 equals phi_0."""
    M = np.array([[3.0, -1, -1, -1], [-1, 3, 0, 0], [-1, 0, 3, 0], [-1, 0, 0, 3]])
    A = from_dense(M)
    s, _ = O.strength(A)
    cf = np.array([-1, 1, 1, 1], np.int8)
    V = np.array([[1.0, 1.0], [1.0, 0.0], [0.0, 2.0], [1.0, 1.0]])
    D = dense(O.bamg(A, s, cf, V, lmax=1))
    np.testing.assert_allclose(D[0], [1.0, 0.5, 0.0], rtol=1e-15, atol=0)


def test_adaptive_distance():
    """A threshold nothing can meet runs every row to lmax; thresholds that
    always hold stop every row at lmin."""
    A = PB.elasticity3d(3)
    s, cnt = O.strength(A)
    cf, _ = O.pmis(A, s, cnt, 0, 0)
    V = O.orthonormalize(PB.elasticity_rigid_modes(3))
    at1 = O.bamg(A, s, cf, V, lmin=1, lmax=1)
    lazy = O.bamg(A, s, cf, V, lmin=1, lmax=2, eps=1e300, mu=1e300)
    eager = O.bamg(A, s, cf, V, lmin=1, lmax=2, eps=-1.0, mu=-1.0)
    at2 = O.bamg(A, s, cf, V, lmin=2, lmax=2)
    for a, b in ((lazy, at1), (eager, at2)):
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4])
    assert not np.array_equal(at1[2], at2[2])


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


def test_bamg_vcycle_matches_iteration_matrix():
    A = PB.elasticity3d(2)
    h = O.Hierarchy(A, V=PB.elasticity_rigid_modes(2), max_coarse=20, interp=O.INTERP_BAMG)
    assert h.nlev >= 2
    Ps = [dense(h.P(l)) for l in range(h.nlev - 1)]
    om = [h.omega(l) for l in range(h.nlev - 1)]
    M = _M_recursive(dense(A), Ps, om, 0)
    Mo = np.stack([h.vcycle(e) for e in np.eye(A.n)], axis=1)
    np.testing.assert_allclose(Mo, M, rtol=0, atol=1e-12 * np.abs(M).max())


def test_bamg_rigid_modes_beat_direct_on_elasticity():
    A = PB.elasticity3d(6)
    b = PB.rhs(A.n)
    xs = np.linalg.solve(dense(A), b)
    rd = O.Hierarchy(A).solve(b, 1e-8)
    hb = O.Hierarchy(A, V=PB.elasticity_rigid_modes(6), interp=O.INTERP_BAMG)
    rb = hb.solve(b, 1e-8)
    assert rb.status == O.OK and rd.status == O.OK
    assert np.linalg.norm(rb.x - xs) <= 1e-5 * np.linalg.norm(xs)
    assert rb.iters < 0.7 * rd.iters, (rb.iters, rd.iters)


def test_bamg_needs_a_test_space():
    A = PB.poisson2d(8)
    with pytest.raises(O.OracleError) as e:
        O.Hierarchy(A, interp=O.INTERP_BAMG)
    assert e.value.status == O.E_ARG


def test_distance_follows_strong_connections():
    """0 -weak- 1 -strong- 2 with C = {0, 2}: the distance-1 candidate of
    the F point 1 is 2 only (its coupling to 0 is below theta)."""
    M = np.array([[2.0, -0.1, 0.0], [-0.1, 2.0, -1.0], [0.0, -1.0, 2.0]])
    A = from_dense(M)
    s, _ = O.strength(A)
    cf = np.array([1, -1, 1], np.int8)
    V = np.ones((3, 1)) / np.sqrt(3.0)
    D = dense(O.bamg(A, s, cf, V, lmax=1))
    np.testing.assert_array_equal(D[1], [0.0, 1.0])


def test_coarse_test_space_is_injected():
    """Level 1 of a BAMG hierarchy is built with the level-0 orthonormal test
    space restricted to the C points."""
    A = PB.elasticity3d(4)
    V = PB.elasticity_rigid_modes(4)
    h = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=30)
    assert h.nlev >= 3
    V1 = O.orthonormalize(V)[h.cf(0) == 1]
    P1 = O.bamg(h.A(1), h.strong(1), h.cf(1), V1)
    hp = h.P(1)
    assert all(np.array_equal(a, b) for a, b in zip(P1[2:], hp[2:]))


# ----------------------------------------------------------------- prolongation smoothing and filtering
def _int_laplacian_2d(g, rng):
    """Grid Laplacian with integer weights 1..9; boundary rows get +1 on the
    diagonal, so interior rows sum to exactly zero."""
    n = g * g
    M = np.zeros((n, n))
    ids = np.arange(n).reshape(g, g)
    for a, b in ((ids[:, :-1], ids[:, 1:]), (ids[:-1, :], ids[1:, :])):
        w = rng.integers(1, 10, size=a.size).astype(float)
        M[a.ravel(), b.ravel()] -= w
        M[b.ravel(), a.ravel()] -= w
    M[np.arange(n), np.arange(n)] = -M.sum(1)
    interior = np.zeros((g, g), bool)
    interior[1:-1, 1:-1] = True
    M[np.arange(n), np.arange(n)] += (~interior.ravel()).astype(float)
    return M, interior.ravel()


def test_psmooth_keeps_constants_on_zero_sum_rows():
    """P 1 = 1 and A 1 = 0 on a row give (P - w D^-1 A P) 1 = 1 there."""
    M, interior = _int_laplacian_2d(12, np.random.default_rng(5))
    A = from_dense(M)
    s, cnt = O.strength(A)
    cf, _ = O.pmis(A, s, cnt, 0, 0)
    P = O.interp_direct(A, s, cf)
    D = dense(P)
    ok = np.isclose(D.sum(1), 1.0, rtol=0, atol=1e-14)          # rows interpolating constants exactly
    n, _, rp, ci, _ = A
    nb = np.array([ok[ci[rp[i]:rp[i + 1]]].all() for i in range(n)])
    Ps = dense(O.psmooth(A, 1.0 / np.diag(M), 2.0 / 3.0, P))
    rows = interior & nb
    assert rows.sum() > 20
    np.testing.assert_allclose(Ps[rows].sum(1), 1.0, rtol=0, atol=1e-13)
    # omega = 0 leaves P unchanged (the pattern may grow by explicit zeros)
    np.testing.assert_array_equal(dense(O.psmooth(A, 1.0 / np.diag(M), 0.0, P)), D)


def test_pfilter_hand_example():
    """Row (0.5, -0.3, 0.15, 0.05), rho = 0.8: the two largest reach 0.8 of
    the absolute sum 1.0 and are kept; the dropped 0.2 of action on the unit
    vector is split evenly by the minimum-norm correction: (0.6, -0.2)."""
    P = (1, 4, np.array([0, 4], np.int32), np.array([0, 1, 2, 3], np.int32), np.array([0.5, -0.3, 0.15, 0.05]))
    F = O.pfilter(P, 0.8, np.ones(4))
    assert F[3].tolist() == [0, 1]
    np.testing.assert_allclose(F[4], [0.6, -0.2], rtol=1e-11)
    # rho = 1 keeps everything unchanged
    F1 = O.pfilter(P, 1.0, np.ones(4))
    assert F1[3].tolist() == [0, 1, 2, 3] and np.array_equal(F1[4], P[4])


def test_pfilter_compensates_the_test_space():
    """The filtered P keeps P's action on the coarse test space (eq. action),
    up to the ridge term, wherever the kept columns span it."""
    A = PB.elasticity3d(4)
    V = PB.elasticity_rigid_modes(4)
    s, cnt = O.strength(A)
    cf, _ = O.pmis(A, s, cnt, 0, 0)
    Q = O.orthonormalize(V)
    P = O.bamg(A, s, cf, Q)
    Ps = O.psmooth(A, 1.0 / np.diag(dense(A)), 0.6, P)
    W = Q[cf == 1]
    F = O.pfilter(Ps, 0.7, W)
    Dp, Df = dense(Ps), dense(F)
    assert F[3].size < 0.8 * Ps[3].size
    checked = 0
    for i in range(A.n):
        kept = np.nonzero(Df[i])[0]
        if len(kept) < W.shape[1] or np.linalg.matrix_rank(W[kept]) < W.shape[1]:
            continue
        np.testing.assert_allclose(Df[i] @ W, Dp[i] @ W, atol=1e-8 * np.abs(Dp[i] @ W).max() + 1e-12)
        # the kept entries are the largest ones
        drop = np.setdiff1d(np.nonzero(Dp[i])[0], kept)
        if len(drop):
            assert np.abs(Dp[i][drop]).max() <= np.abs(Dp[i][kept]).min()
        checked += 1
    assert checked > 20


def test_smoothed_bamg_hierarchy():
    A = PB.elasticity3d(2)
    h = O.Hierarchy(A, V=PB.elasticity_rigid_modes(2), max_coarse=20, interp=O.INTERP_BAMG, psmooth=1, pfilter=0.8)
    Ps = [dense(h.P(l)) for l in range(h.nlev - 1)]
    om = [h.omega(l) for l in range(h.nlev - 1)]
    M = _M_recursive(dense(A), Ps, om, 0)
    Mo = np.stack([h.vcycle(e) for e in np.eye(A.n)], axis=1)
    np.testing.assert_allclose(Mo, M, rtol=0, atol=1e-12 * np.abs(M).max())
    A = PB.elasticity3d(10)
    b = PB.rhs(A.n)
    V = PB.elasticity_rigid_modes(10)
    r0 = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG).solve(b, 1e-8)
    r1 = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, psmooth=1).solve(b, 1e-8)
    assert r1.status == O.OK and r1.iters < r0.iters
