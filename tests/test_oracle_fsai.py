"""Pins of the oracle's FSAI smoother (M^{-1} = G^T G, G lower triangular;
Section 2, eq. smo), checked against what the mathematics fixes: closed
forms, brute-force local systems, invariants of G A G^T, omega against the
spectral condition and against the power method written with dense
algebra, and the V-cycle against the two-grid iteration matrix with
S = I - omega G^T G A."""
import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB

from helpers import dense, from_dense


def _G(A):
    st, G = O.fsai(A)
    assert st == O.OK
    return G


def test_fsai_diagonal_closed_form():
    d = np.array([4.0, 0.25, 9.0, 2.0, 1e-3])
    A = from_dense(np.diag(d))
    G = dense(_G(A))
    np.testing.assert_allclose(np.diag(G), 1.0 / np.sqrt(d), rtol=1e-15)
    assert np.count_nonzero(G - np.diag(np.diag(G))) == 0


def test_fsai_full_pattern_is_inverse_cholesky_factor():
    """With the whole lower triangle as pattern, G A G^T = I and G = L^{-1}."""
    rng = np.random.default_rng(11)
    for n in (3, 8, 17):
        B = rng.standard_normal((n, n))
        Ad = B @ B.T + n * np.eye(n)
        G = dense(_G(from_dense(Ad)))
        np.testing.assert_allclose(G @ Ad @ G.T, np.eye(n), atol=1e-12)
        L = np.linalg.cholesky(Ad)
        np.testing.assert_allclose(G, np.linalg.inv(L), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("gen", ["p2", "ln2", "ln3", "el"])
def test_fsai_pattern_unit_diagonal_and_local_systems(gen):
    A = {"p2": lambda: PB.poisson2d(7), "ln2": lambda: PB.lognormal2d(6, 2.0),
         "ln3": lambda: PB.lognormal3d(4, 2.0), "el": lambda: PB.elasticity3d(2)}[gen]()
    G = _G(A)
    Ad, Gd = dense(A), dense(G)
    # pattern: exactly the stored entries of A on or below the diagonal
    for i in range(A.n):
        cols = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert list(G[3][G[2][i]:G[2][i + 1]]) == [c for c in cols if c <= i]
    # G A G^T has a unit diagonal
    np.testing.assert_allclose(np.diag(Gd @ Ad @ Gd.T), 1.0, rtol=0, atol=1e-13)
    # brute force: each row solves its local system A(P_i, P_i) g = e_last, scaled
    for i in range(A.n):
        P = [c for c in A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]] if c <= i]
        g = np.linalg.solve(Ad[np.ix_(P, P)], np.eye(len(P))[-1])
        np.testing.assert_allclose(Gd[i, P], g / np.sqrt(g[-1]), rtol=1e-12, atol=1e-14)


_OMEGA_CASES = {"p2": lambda: PB.poisson2d(9), "ln2": lambda: PB.lognormal2d(9, 2.0),
                "ln3": lambda: PB.lognormal3d(5, 2.0), "el": lambda: PB.elasticity3d(2),
                "an3": lambda: PB.aniso3d(5, 1e-3)}


def _splitmix64(seed, c):
    """Draw c of splitmix64 seeded with `seed` (the published algorithm,
    written here again; its outputs are pinned in test_oracle.py)."""
    m = (1 << 64) - 1
    z = (seed + (c + 1) * 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


@pytest.mark.parametrize("gen", list(_OMEGA_CASES))
def test_fsai_omega_spectral_condition(gen):
    """omega = (4/3) / rho_hat with rho_hat a Rayleigh quotient of G A G^T,
    so omega rho(G^T G A) >= 4/3; fifteen power steps from a random start
    bring rho_hat within 17 % of rho here, so omega rho < 1.6 < 2."""
    A = _OMEGA_CASES[gen]()
    G = _G(A)
    w = O.fsai_omega(A, G, 7, 0)
    Gd, Ad = dense(G), dense(A)
    M = Gd @ Ad @ Gd.T
    lam = np.linalg.eigvalsh(M).max()
    assert w * lam >= 4.0 / 3.0 * (1 - 1e-12)
    assert w * lam < 1.6
    # rho(G^T G A) = rho(G A G^T)
    assert abs(np.abs(np.linalg.eigvals(Gd.T @ Gd @ Ad)).max() - lam) <= 1e-10 * lam


@pytest.mark.parametrize("gen", list(_OMEGA_CASES))
@pytest.mark.parametrize("seed,level", [(7, 0), (2021, 3)])
def test_fsai_omega_matches_dense_power_method(gen, seed, level):
    """The same fifteen power steps written with dense numpy algebra on the
    formed M = G A G^T, from the start vector drawn with splitmix64 written
    here again: the Rayleigh quotient and so omega agree to rounding."""
    A = _OMEGA_CASES[gen]()
    G = _G(A)
    Gd, Ad = dense(G), dense(A)
    M = Gd @ Ad @ Gd.T
    n = M.shape[0]
    v = np.array([2.0 * ((_splitmix64(seed + 1, (level << 40) + i) >> 11) * 2.0 ** -53) - 1.0 for i in range(n)])
    for _ in range(15):
        w = M @ v
        rq = (v @ w) / (v @ v)
        v = w / np.linalg.norm(w)
    assert O.fsai_omega(A, G, seed, level) == pytest.approx((4.0 / 3.0) / rq, rel=1e-12)


def test_fsai_omega_is_four_thirds_when_the_factor_is_exact():
    """G A G^T = I (diagonal A, or the whole lower triangle as pattern):
    every Rayleigh quotient is 1, so omega = 4/3."""
    A = from_dense(np.diag([4.0, 0.25, 9.0, 2.0, 1e-3, 7.0]))
    assert O.fsai_omega(A, _G(A), 3, 1) == pytest.approx(4.0 / 3.0, rel=1e-14)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((12, 12))
    A = from_dense(B @ B.T + 12 * np.eye(12))
    assert O.fsai_omega(A, _G(A), 3, 0) == pytest.approx(4.0 / 3.0, rel=1e-12)


def _M_fsai(Al, Ps, Gs, omegas, l, nu1, nu2):
    """M_l = (I - E_l) A_l^{-1}, E_l = S^nu2 (I - P M_{l+1} P^T A_l) S^nu1 with
    S = I - omega G^T G A_l (eq. twoGridOp, eq. smoother, eq. smo)."""
    if l == len(Ps):
        return np.linalg.inv(Al)
    P = Ps[l]
    Mc = _M_fsai(P.T @ Al @ P, Ps, Gs, omegas, l + 1, nu1, nu2)
    n = Al.shape[0]
    S = np.eye(n) - omegas[l] * Gs[l].T @ Gs[l] @ Al
    E = np.linalg.matrix_power(S, nu2) @ (np.eye(n) - P @ Mc @ P.T @ Al) @ np.linalg.matrix_power(S, nu1)
    return (np.eye(n) - E) @ np.linalg.inv(Al)


@pytest.mark.parametrize("gen,mc,nu", [("p2", 40, 1), ("ln2", 15, 1), ("p2", 20, 2), ("el", 30, 1)])
def test_fsai_vcycle_matches_iteration_matrix(gen, mc, nu):
    A = {"p2": lambda: PB.poisson2d(12), "ln2": lambda: PB.lognormal2d(11, 2.0),
         "el": lambda: PB.elasticity3d(2)}[gen]()
    h = O.Hierarchy(A, max_coarse=mc, nu_pre=nu, nu_post=nu, smoother=O.SMOOTH_FSAI)
    assert h.nlev >= 2
    Ps = [dense(h.P(l)) for l in range(h.nlev - 1)]
    Gs = [dense(h.G(l)) for l in range(h.nlev - 1)]
    om = [h.omega(l) for l in range(h.nlev - 1)]
    # each level's G is the FSAI factor of that level's operator
    for l in range(h.nlev - 1):
        np.testing.assert_array_equal(Gs[l], dense(_G(h.A(l))))
    M = _M_fsai(dense(A), Ps, Gs, om, 0, nu, nu)
    Mo = np.stack([h.vcycle(e) for e in np.eye(A.n)], axis=1)
    np.testing.assert_allclose(Mo, M, rtol=0, atol=1e-12 * np.abs(M).max())
    # symmetric positive definite preconditioner
    np.testing.assert_allclose(Mo, Mo.T, rtol=0, atol=1e-12 * np.abs(Mo).max())
    assert np.linalg.eigvalsh((Mo + Mo.T) / 2).min() > 0


@pytest.mark.parametrize("gen", ["ln3", "el", "an3"])
def test_fsai_pcg_converges_to_dense_solution(gen):
    A = {"ln3": lambda: PB.lognormal3d(9, 2.0), "el": lambda: PB.elasticity3d(3),
         "an3": lambda: PB.aniso3d(9)}[gen]()
    h = O.Hierarchy(A, max_coarse=30, max_iter=2000, smoother=O.SMOOTH_FSAI)
    b = PB.rhs(A.n)
    r = h.solve(b, 1e-8, max_iter=2000)
    assert r.status == O.OK
    Ad = dense(A)
    assert np.linalg.norm(b - Ad @ r.x) / np.linalg.norm(b) < 1.5e-8
    assert r.hist[-1] < 1e-8 * np.linalg.norm(b) <= r.hist[-2]


# ----------------------------------------------------------------- FSAI where the rows fit, Jacobi elsewhere
def _lower_max(Al):
    n, _, rp, ci, _ = Al
    rows = np.repeat(np.arange(n), np.diff(rp))
    return int(np.bincount(rows[ci <= rows], minlength=n).max())


def test_fsai_jacobi_with_short_rows_is_fsai():
    A = PB.lognormal3d(9, 2.0)
    hf = O.Hierarchy(A, max_coarse=30, smoother=O.SMOOTH_FSAI)
    hm = O.Hierarchy(A, max_coarse=30, smoother=O.SMOOTH_FSAI_JACOBI)
    assert hf.nlev == hm.nlev >= 3
    for l in range(hm.nlev - 1):
        assert _lower_max(hm.A(l)) <= 192
        np.testing.assert_array_equal(hm.G(l)[4], hf.G(l)[4])
        assert hm.omega(l) == hf.omega(l)
    y = np.random.default_rng(4).standard_normal(A.n)
    assert np.array_equal(hm.vcycle(y), hf.vcycle(y))


def test_fsai_jacobi_with_long_rows_is_jacobi():
    """Every row of a radius-10 stencil has 221 entries on or below the
    diagonal: that level keeps the Jacobi smoother and weight."""
    from helpers import wide_stencil_2d
    A = wide_stencil_2d(24, 10)
    hj = O.Hierarchy(A, max_coarse=40)
    hm = O.Hierarchy(A, max_coarse=40, smoother=O.SMOOTH_FSAI_JACOBI)
    assert _lower_max(hm.A(0)) > 192 and not hm.has_G(0)
    assert hm.omega(0) == hj.omega(0)
    for l in range(hm.nlev - 1):
        assert hm.has_G(l) == (_lower_max(hm.A(l)) <= 192)
        if not hm.has_G(l):
            assert hm.omega(l) == hj.omega(l)
    if not any(hm.has_G(l) for l in range(hm.nlev - 1)):
        y = np.random.default_rng(4).standard_normal(A[0])
        assert np.array_equal(hm.vcycle(y), hj.vcycle(y))


def _M_levels(Al, Ps, Minvs, omegas, l):
    """Iteration-matrix recursion with each level's own smoother
    S_l = I - omega_l Minv_l A_l (G^T G on FSAI levels, D^{-1} on Jacobi ones)."""
    if l == len(Ps):
        return np.linalg.inv(Al)
    P = Ps[l]
    Mc = _M_levels(P.T @ Al @ P, Ps, Minvs, omegas, l + 1)
    n = Al.shape[0]
    S = np.eye(n) - omegas[l] * Minvs[l] @ Al
    E = S @ (np.eye(n) - P @ Mc @ P.T @ Al) @ S
    return (np.eye(n) - E) @ np.linalg.inv(Al)


def test_fsai_jacobi_mixed_levels_vcycle_matches_iteration_matrix():
    """BAMG on 8^3 elasticity: level 1 has rows with 212 entries on or below
    the diagonal (Jacobi), levels 0 and 2 smooth with FSAI."""
    A, V = PB.elasticity3d(8), PB.elasticity_rigid_modes(8)
    h = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=40, smoother=O.SMOOTH_FSAI_JACOBI)
    kinds = [h.has_G(l) for l in range(h.nlev - 1)]
    assert kinds[0] and not all(kinds), kinds
    Ps, Minvs, om = [], [], []
    for l in range(h.nlev - 1):
        Ps.append(dense(h.P(l)))
        Ad = dense(h.A(l))
        if kinds[l]:
            Gd = dense(h.G(l))
            np.testing.assert_array_equal(Gd, dense(_G(h.A(l))))
            Minvs.append(Gd.T @ Gd)
        else:
            Minvs.append(np.diag(1.0 / np.diag(Ad)))
        om.append(h.omega(l))
    M = _M_levels(dense(A), Ps, Minvs, om, 0)
    Mo = np.stack([h.vcycle(e) for e in np.eye(A.n)], axis=1)
    np.testing.assert_allclose(Mo, M, rtol=0, atol=1e-12 * np.abs(M).max())
    np.testing.assert_allclose(Mo, Mo.T, rtol=0, atol=1e-12 * np.abs(Mo).max())
    b = PB.rhs(A.n)
    rj = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=40).solve(b, 1e-8, max_iter=2000)
    rm = h.solve(b, 1e-8, max_iter=2000)
    assert rm.status == O.OK and rm.iters < rj.iters
