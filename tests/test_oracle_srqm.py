"""Pins of the oracle's test-space refinement by simultaneous Rayleigh
quotient minimisation (Section 2, Unveiling the operator near kernel, eq.
eigP) and of its dense symmetric eigensolver.  The checks come from outside
the oracle: LAPACK's eigenvalues, a Rayleigh-Ritz step written with SciPy's
generalized eigensolver, the Rayleigh-Ritz properties (orthonormal output,
a trace that never grows, convergence to the lowest eigenvectors), exact
invariant subspaces that must stop the iteration, and the hierarchy's
handling of the option."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from paper_2102_07417_amd import problems as PB
from tests.helpers import dense


def _rr_step(Ad, V, Minv, drop_tol=1e-12):
    """One preconditioned Rayleigh-Ritz step, written out independently:
    W = M^{-1}(A V - V V^T A V); the nt lowest Ritz vectors of span[V, W]
    (columns of W that add no direction are left out first)."""
    X = Ad @ V
    W = Minv @ (X - V @ (V.T @ X))
    keep = [W[:, b] for b in range(W.shape[1])
            if np.linalg.norm(W[:, b] - V @ (V.T @ W[:, b])) > np.sqrt(drop_tol) * np.linalg.norm(W[:, b]) and
            np.linalg.norm(W[:, b]) > 1e-6 * np.sqrt(drop_tol)]
    S = np.hstack([V] + [w[:, None] for w in keep])
    lam, Y = sl.eigh(S.T @ Ad @ S, S.T @ S)
    return S @ Y[:, :V.shape[1]], lam[:V.shape[1]]


def _proj(V):
    Q, _ = np.linalg.qr(V)
    return Q @ Q.T


def _case():
    A = PB.lognormal3d(6, 1.0)
    Ad = dense(A)
    rng = np.random.default_rng(3)
    V0 = O.orthonormalize(rng.standard_normal((A.n, 3)))
    return A, Ad, V0


# ----------------------------------------------------------------- eigensolver
@pytest.mark.parametrize("m", [1, 2, 5, 12, 16])
def test_symeig_matches_lapack(m):
    rng = np.random.default_rng(m)
    B = rng.standard_normal((m, m))
    Cm = B + B.T
    lam, Q = O.symeig(Cm)
    ref = np.linalg.eigvalsh(Cm)
    np.testing.assert_allclose(np.sort(lam), ref, rtol=0, atol=1e-13 * max(1.0, np.abs(ref).max()))
    np.testing.assert_allclose(Cm @ Q, Q * lam, atol=1e-12 * max(1.0, np.abs(ref).max()))
    np.testing.assert_allclose(Q.T @ Q, np.eye(m), atol=1e-13)


def test_symeig_diagonal_and_repeated():
    d = np.array([3.0, -1.0, 2.0, 0.5])
    lam, Q = O.symeig(np.diag(d))
    assert np.array_equal(lam, d) and np.array_equal(Q, np.eye(4))  # nothing to rotate
    # identity plus a rank-one term: eigenvalue 1 five times and 1 + |u|^2
    u = np.arange(1.0, 7.0)
    lam, Q = O.symeig(np.eye(6) + np.outer(u, u))
    np.testing.assert_allclose(np.sort(lam), [1, 1, 1, 1, 1, 1 + u @ u], atol=1e-12 * (u @ u))
    k = int(np.argmax(lam))
    np.testing.assert_allclose(np.abs(Q[:, k]), u / np.linalg.norm(u), atol=1e-12)


def test_symeig_two_by_two_closed_form():
    a, b, c = 2.0, 0.75, -1.0
    lam, Q = O.symeig(np.array([[a, b], [b, c]]))
    mid, rad = (a + c) / 2, np.hypot((a - c) / 2, b)
    np.testing.assert_allclose(np.sort(lam), [mid - rad, mid + rad], atol=1e-15)


# ----------------------------------------------------------------- one step
def test_one_step_is_rayleigh_ritz_jacobi():
    A, Ad, V0 = _case()
    dinv = 1.0 / np.diag(Ad)
    V1, done = O.srqm(A, V0, 1, dinv=dinv)
    Vr, lam = _rr_step(Ad, V0, np.diag(dinv))
    assert done == 1
    np.testing.assert_allclose(_proj(V1), _proj(Vr), atol=1e-10)
    np.testing.assert_allclose(np.trace(V1.T @ Ad @ V1), lam.sum(), rtol=1e-12)
    np.testing.assert_allclose(V1.T @ V1, np.eye(3), atol=1e-12)


def test_one_step_is_rayleigh_ritz_fsai():
    A, Ad, V0 = _case()
    st, G = O.fsai(A)
    assert st == O.OK
    Gd = dense(G)
    V1, done = O.srqm(A, V0, 1, G=G)
    Vr, lam = _rr_step(Ad, V0, Gd.T @ Gd)
    assert done == 1
    np.testing.assert_allclose(_proj(V1), _proj(Vr), atol=1e-10)
    np.testing.assert_allclose(np.trace(V1.T @ Ad @ V1), lam.sum(), rtol=1e-12)


def test_ritz_vectors_are_the_lowest_not_the_highest():
    """The kept Ritz vectors minimise the Rayleigh quotient: the trace after
    one step is at most that of any nt-dimensional part of span[V, W]."""
    A, Ad, V0 = _case()
    dinv = 1.0 / np.diag(Ad)
    V1, _ = O.srqm(A, V0, 1, dinv=dinv)
    assert np.trace(V1.T @ Ad @ V1) < np.trace(V0.T @ Ad @ V0)


# ----------------------------------------------------------------- iteration
def test_trace_never_grows_and_converges():
    A, Ad, V0 = _case()
    dinv = 1.0 / np.diag(Ad)
    tr = [np.trace(V0.T @ Ad @ V0)]
    V = V0
    for _ in range(15):
        V, done = O.srqm(A, V, 1, dinv=dinv)
        assert done == 1
        tr.append(np.trace(V.T @ Ad @ V))
    assert all(b <= a * (1 + 1e-14) for a, b in zip(tr, tr[1:]))
    # k steps in one call are k single steps
    Vk, done = O.srqm(A, V0, 15, dinv=dinv)
    assert done == 15 and np.array_equal(Vk, V)


def test_converges_to_lowest_eigenvectors():
    A, Ad, V0 = _case()
    st, G = O.fsai(A)
    ev, EV = np.linalg.eigh(Ad)
    V, done = O.srqm(A, V0, 150, G=G)
    cos = np.linalg.svd(EV[:, :3].T @ np.linalg.qr(V)[0], compute_uv=False)
    assert cos.min() > 0.999
    np.testing.assert_allclose(np.trace(V.T @ Ad @ V), ev[:3].sum(), rtol=1e-5)


def test_invariant_subspace_stops_at_once():
    A, Ad, _ = _case()
    ev, EV = np.linalg.eigh(Ad)
    Ve = np.ascontiguousarray(EV[:, [0, 4, 9]])
    V, done = O.srqm(A, Ve, 5, dinv=1.0 / np.diag(Ad))
    assert done == 0 and np.array_equal(V, Ve)


def test_exact_column_is_left_out_of_the_subspace():
    """One exact eigenvector in V: its residual vanishes, the matching column
    of W is left out, and the step is Rayleigh-Ritz over the other columns."""
    A, Ad, _ = _case()
    ev, EV = np.linalg.eigh(Ad)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(A.n)
    r = r - EV[:, 0] * (EV[:, 0] @ r)
    V0 = np.stack([EV[:, 0], r / np.linalg.norm(r)], 1)
    dinv = 1.0 / np.diag(Ad)
    V1, done = O.srqm(A, V0, 1, dinv=dinv)
    Vr, lam = _rr_step(Ad, V0, np.diag(dinv))
    assert done == 1
    np.testing.assert_allclose(_proj(V1), _proj(Vr), atol=1e-9)
    np.testing.assert_allclose(np.abs(V1[:, 0] @ EV[:, 0]), 1.0, atol=1e-12)


def test_rejects_bad_arguments():
    A, Ad, V0 = _case()
    with pytest.raises(O.OracleError):
        O.srqm(A, V0, -1, dinv=1.0 / np.diag(Ad))
    with pytest.raises(O.OracleError):
        O.srqm(A, np.zeros((A.n, 9)), 1, dinv=1.0 / np.diag(Ad))


# ----------------------------------------------------------------- hierarchy
def test_hierarchy_option():
    A = PB.elasticity3d(4)
    V = PB.elasticity_rigid_modes(4)
    h0 = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=40)
    hz = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=40, srqm_iters=0)
    assert np.array_equal(h0.P(0)[4], hz.P(0)[4])
    h3 = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=40, srqm_iters=3)
    p0, p3 = h0.P(0), h3.P(0)
    assert np.array_equal(h0.cf(0), h3.cf(0))  # the split does not use the test space
    assert not (np.array_equal(p0[3], p3[3]) and np.array_equal(p0[4], p3[4]))
    b = PB.rhs(A.n)
    r = h3.solve(b, 1e-8, max_iter=2000)
    assert r.status == O.OK and r.true_relres < 1e-8
    with pytest.raises(O.OracleError) as e:
        O.Hierarchy(A, max_coarse=40, srqm_iters=2)  # needs the BAMG test space
    assert e.value.status == O.E_ARG
    with pytest.raises(O.OracleError):
        O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, srqm_iters=101)


def test_refined_random_space_beats_the_random_one():
    """From a random start, a few steps give a BAMG hierarchy that converges
    in fewer PCG iterations (the near kernel is uncovered)."""
    A = PB.elasticity3d(4)
    V = np.random.default_rng(11).standard_normal((A.n, 6))
    b = PB.rhs(A.n)
    it = {}
    for k in (0, 8):
        h = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=40, srqm_iters=k)
        r = h.solve(b, 1e-8, max_iter=3000)
        assert r.status == O.OK
        it[k] = r.iters
    assert it[8] < it[0], it
