"""Pins of the CPU oracle against facts fixed outside it: published test
vectors, hand-worked examples, closed forms, dense linear algebra from
numpy, invariants of the definitions and the paper's two-grid formula."""
import os

import numpy as np
import pytest
import yaml

import oracle as O
from paper_2102_07417_amd import problems as PB
from tests.helpers import dense, from_dense, pattern, rows_sorted

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _hand():
    with open(os.path.join(GOLD, "hand_examples.yaml")) as f:
        return yaml.safe_load(f)


# ----------------------------------------------------------------- RNG
def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(os.path.join(GOLD, "splitmix64.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 7
    for seed, k, out in rows:
        assert O.splitmix64(int(seed), int(k)) == int(out)


def test_pmis_rand_layout():
    # draw (level << 40) + i of the seeded generator, top 53 bits
    for seed, lev, i in [(0, 0, 0), (0, 0, 5), (7, 3, 123456), (2**63 + 5, 24, 2**31 - 1)]:
        assert O.pmis_rand(seed, lev, i) == O.splitmix64(seed, (lev << 40) + i) >> 11
        assert O.pmis_rand(seed, lev, i) < 2**53


# ----------------------------------------------------------------- validation
def test_validate_accepts_generators():
    for A in [PB.poisson2d(7), PB.lognormal3d(4), PB.aniso3d(4), PB.elasticity3d(2)]:
        assert O.validate(A) == O.OK


def _bad(kind):
    n, _, rp, ci, v = from_dense(PB.poisson2d(3).to_dense())
    rp, ci, v = rp.copy(), ci.copy(), v.copy()
    if kind == "rp0":
        rp[0] = 1
    elif kind == "rp_dec":
        rp[2], rp[3] = rp[3], rp[2]
    elif kind == "col_range":
        ci[-1] = n
    elif kind == "col_order":
        ci[0], ci[1] = ci[1], ci[0]
        v[0], v[1] = v[1], v[0]
    elif kind == "nan":
        v[3] = np.nan
    elif kind == "nodiag":
        d = from_dense(PB.poisson2d(3).to_dense(), keep_zero_diag=False)
        M = dense(d)
        M[4, 4] = 0.0
        return from_dense(M, keep_zero_diag=False), O.E_CSR
    elif kind == "asym":
        v[1] = -1.5
    elif kind == "negdiag":
        v[0] = -4.0
        return (n, n, rp, ci, v), O.E_NOT_SPD
    return (n, n, rp, ci, v), O.E_CSR


@pytest.mark.parametrize("kind", ["rp0", "rp_dec", "col_range", "col_order", "nan", "nodiag", "asym", "negdiag"])
def test_validate_rejects(kind):
    A, code = _bad(kind)
    assert O.validate(A) == code


# ----------------------------------------------------------------- strength
def test_strength_hand_examples():
    for ex in _hand()["strength"]:
        A = from_dense(ex["dense"])
        s, cnt = O.strength(A, 0.25)
        assert s.tolist() == ex["strong_csr_order"], ex["name"]
        assert cnt.tolist() == ex["st_count"], ex["name"]


def test_strength_laplacian_all_strong():
    A = PB.poisson2d(9)
    s, cnt = O.strength(A)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = A.col_idx != rows
    assert np.all(s[off] == 1) and np.all(s[~off] == 0)
    assert np.array_equal(cnt, np.diff(A.row_ptr) - 1)


def test_strength_anisotropic_drops_weak_axis():
    n = 6
    A = PB.aniso3d(n, 1e-3)          # eps = 1e-3 < theta: z couplings are weak
    s, _ = O.strength(A)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    d = np.abs(A.col_idx.astype(np.int64) - rows)
    assert np.all(s[(d == 1) | (d == n)] == 1)
    assert np.all(s[(d == n * n) | (d == 0)] == 0)


def test_strength_threshold_monotone():
    A = PB.lognormal3d(6, 2.0)
    prev = None
    for th in [0.0, 0.1, 0.25, 0.5, 0.9, 1.0]:
        s, _ = O.strength(A, th)
        if prev is not None:
            assert np.all(s <= prev)       # a higher threshold never adds a connection
        prev = s
    s, _ = O.strength(A, 1.0)               # theta = 1: exactly the largest coupling(s) of each row
    for i in range(A.n):
        seg = slice(A.row_ptr[i], A.row_ptr[i + 1])
        cols, vals = A.col_idx[seg], A.val[seg]
        off = cols != i
        m = np.max(-vals[off])
        assert s[seg][off].tolist() == (-vals[off] == m).astype(int).tolist()


# ----------------------------------------------------------------- PMIS
def _check_pmis_invariants(A, s, cnt, cf):
    nr, _, rp, ci, _ = (A.n, A.n, A.row_ptr, A.col_idx, A.val) if hasattr(A, "row_ptr") else A
    assert set(np.unique(cf).tolist()) <= {O.F, O.CPT}
    S = np.zeros((nr, nr), bool)
    rows = np.repeat(np.arange(nr), np.diff(rp))
    S[rows[s == 1], ci[s == 1]] = True
    C = cf == O.CPT
    # Two C points can never depend strongly on each other (whichever was
    # selected first makes the other F); with a symmetric S this means C is
    # independent.  With an asymmetric S a later C point may influence an
    # earlier one.
    assert not np.any((S & S.T)[np.ix_(C, C)])
    if np.array_equal(S, S.T):
        assert not np.any(S[np.ix_(C, C)]), "C points must be independent"
    for i in np.where(cf == O.F)[0]:
        assert cnt[i] == 0 or np.any(S[i] & C), f"F point {i} has no strong C neighbour"
    for i in np.where(cnt == 0)[0]:
        assert cf[i] == O.F


@pytest.mark.parametrize("gen", ["p2", "ln3", "an3", "el"])
def test_pmis_invariants(gen):
    A = {"p2": lambda: PB.poisson2d(12), "ln3": lambda: PB.lognormal3d(6, 2.0),
         "an3": lambda: PB.aniso3d(6), "el": lambda: PB.elasticity3d(2)}[gen]()
    s, cnt = O.strength(A)
    for seed in [0, 1, 99]:
        cf, rounds = O.pmis(A, s, cnt, seed, 0)
        assert rounds >= 1
        _check_pmis_invariants(A, s, cnt, cf)
        # the point with the globally largest measure is always selected first
        u = np.array([O.pmis_rand(seed, 0, i) for i in range(A.n)], dtype=object)
        best = max((i for i in range(A.n) if cnt[i] > 0), key=lambda i: (cnt[i], u[i], i))
        assert cf[best] == O.CPT


def test_pmis_hand_three_points():
    # Strength from the hand example: S_0 = {1,2}, S_1 = {0}, S_2 = {0,1};
    # |S^T| = (2, 2, 1).  Points 0 and 1 tie on |S^T|; the random part decides.
    # If 0 wins it becomes C and both others depend on it -> F; if 1 wins,
    # 0 and 2 depend on 1 -> F.
    A = from_dense([[10, -4, -1], [-4, 10, -0.5], [-1, -0.5, 10]])
    s, cnt = O.strength(A)
    for seed in range(8):
        u0, u1 = O.pmis_rand(seed, 0, 0), O.pmis_rand(seed, 0, 1)
        cf, rounds = O.pmis(A, s, cnt, seed, 0)
        want = [1, -1, -1] if u0 > u1 else [-1, 1, -1]
        assert cf.tolist() == want and rounds == 1


def test_pmis_hand_rounds():
    for ex in _hand()["pmis"]:
        A = from_dense(ex["dense"])
        s, cnt = O.strength(A)
        assert cnt.tolist() == ex["st_count"]
        for seed in range(4):
            cf, rounds = O.pmis(A, s, cnt, seed, 0)
            assert cf.tolist() == ex["cf"] and rounds == ex["rounds"], ex["name"]


def test_pmis_level_changes_draws():
    A = PB.poisson2d(16)
    s, cnt = O.strength(A)
    a, _ = O.pmis(A, s, cnt, 0, 0)
    b, _ = O.pmis(A, s, cnt, 0, 1)
    c, _ = O.pmis(A, s, cnt, 0, 0)
    assert np.array_equal(a, c) and not np.array_equal(a, b)


# ----------------------------------------------------------------- interpolation
def test_interp_hand_lumping():
    ex = [e for e in _hand()["interp_direct"] if e["name"] == "lumping_weak_and_empty_rows"][0]
    A = from_dense(ex["dense"])
    s, _ = O.strength(A)
    P = O.interp_direct(A, s, np.array(ex["cf"], np.int8))
    assert np.diff(P[2]).tolist() == ex["P_row_nnz"]
    np.testing.assert_allclose(dense(P), np.array(ex["P_dense"]), rtol=1e-15, atol=0)


def test_interp_hand_laplacian_columns():
    ex = [e for e in _hand()["interp_direct"] if e["name"] == "laplacian_columns_coarse"][0]
    g = ex["grid"]
    A = PB.poisson2d(g)
    s, _ = O.strength(A)
    ix = np.arange(A.n) % g
    iy = np.arange(A.n) // g
    cf = np.where(ix % 2 == 0, 1, -1).astype(np.int8)
    P = O.interp_direct(A, s, cf)
    D = dense(P)
    for i in range(A.n):
        if cf[i] == 1:
            continue
        nz = D[i][D[i] != 0]
        w = ex["interior_weight"] if 0 < iy[i] < g - 1 else ex["boundary_weight"]
        assert len(nz) == 2 and np.allclose(nz, w, rtol=1e-15, atol=0)


@pytest.mark.parametrize("gen", ["p2", "ln3", "el"])
def test_interp_invariants(gen):
    A = {"p2": lambda: PB.poisson2d(12), "ln3": lambda: PB.lognormal3d(6, 2.0),
         "el": lambda: PB.elasticity3d(2)}[gen]()
    s, cnt = O.strength(A)
    cf, _ = O.pmis(A, s, cnt, 0, 0)
    P = O.interp_direct(A, s, cf)
    nr, nc, rp, ci, v = P
    assert nr == A.n and nc == int(np.sum(cf == 1)) and rows_sorted(P)
    D = dense(P)
    Cidx = np.where(cf == 1)[0]
    assert np.array_equal(D[Cidx], np.eye(nc))            # P = [W; I]
    Ad = dense(A)
    rowsum = Ad.sum(1)
    S = np.zeros_like(Ad, dtype=bool)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    S[rows[s == 1], A.col_idx[s == 1]] = True
    for i in np.where(cf == -1)[0]:
        cols = np.where(D[i] != 0)[0]
        # the interpolatory set is exactly C_i^S, in coarse numbering
        assert np.array_equal(np.sort(np.searchsorted(Cidx, np.where(S[i] & (cf == 1))[0])), cols)
        if len(cols) and abs(rowsum[i]) < 1e-12 * Ad[i, i] and gen != "el":
            assert abs(D[i].sum() - 1.0) < 1e-13                 # constants are interpolated exactly
        if gen != "el":
            assert np.all(D[i][cols] > 0)


# ----------------------------------------------------------------- transpose / SpGEMM / Galerkin
def _rand_int_csr(rng, nr, nc, dens, lo=-3, hi=4):
    M = rng.integers(lo, hi, size=(nr, nc)).astype(float)
    M[rng.random((nr, nc)) > dens] = 0.0
    return M


def test_transpose_matches_dense():
    rng = np.random.default_rng(1)
    M = _rand_int_csr(rng, 13, 7, 0.3)
    T = O.transpose(from_dense(M, keep_zero_diag=False))
    assert T[0] == 7 and T[1] == 13 and rows_sorted(T)
    assert np.array_equal(dense(T), M.T)


def test_spgemm_exact_and_symbolic_pattern():
    rng = np.random.default_rng(2)
    for _ in range(20):
        X = _rand_int_csr(rng, 11, 9, 0.35)
        Y = _rand_int_csr(rng, 9, 8, 0.35)
        Z = O.spgemm(from_dense(X, False), from_dense(Y, False))
        assert rows_sorted(Z)
        assert np.array_equal(dense(Z), X @ Y)                              # exact in FP64
        assert np.array_equal(pattern(Z), (X != 0).astype(int) @ (Y != 0).astype(int) > 0)


def test_spgemm_keeps_cancelled_entries():
    X = np.array([[1.0, 1.0]])
    Y = np.array([[2.0, 5.0], [-2.0, 0.0]])
    Z = O.spgemm(from_dense(X, False), from_dense(Y, False))
    assert Z[3].tolist() == [0, 1] and Z[4].tolist() == [0.0, 5.0]


def test_galerkin_exact_on_integer_operators():
    rng = np.random.default_rng(3)
    A = PB.poisson2d(6)
    for _ in range(5):
        P = _rand_int_csr(rng, A.n, 9, 0.3, -2, 3)
        Ac = O.galerkin(A, from_dense(P, False))
        ref = P.T @ dense(A) @ P
        assert np.array_equal(dense(Ac), ref) and rows_sorted(Ac)
        assert np.array_equal(dense(Ac), dense(Ac).T)


# ----------------------------------------------------------------- smoother weight
def test_omega_closed_form_laplacians():
    for A in [PB.poisson2d(8), PB.poisson3d(5)]:
        assert O.gershgorin_omega(A) == (4.0 / 3.0) / 2.0


@pytest.mark.parametrize("gen", ["ln3", "el", "an3"])
def test_omega_damps(gen):
    A = {"ln3": lambda: PB.lognormal3d(5, 2.0), "el": lambda: PB.elasticity3d(2),
         "an3": lambda: PB.aniso3d(5)}[gen]()
    w = O.gershgorin_omega(A)
    Ad = dense(A)
    ev = np.linalg.eigvals(w * Ad / np.diag(Ad)[:, None]).real
    assert ev.max() < 2.0 and ev.min() > 0.0


# ----------------------------------------------------------------- Cholesky
def test_cholesky_matches_numpy():
    rng = np.random.default_rng(4)
    for n in [1, 2, 7, 40]:
        B = rng.standard_normal((n, n))
        A = B @ B.T + n * np.eye(n)
        st, L = O.cholesky(A)
        assert st == 0
        Ln = np.linalg.cholesky(A)
        np.testing.assert_allclose(L, Ln, rtol=1e-13, atol=1e-13 * np.abs(Ln).max())
        y = rng.standard_normal(n)
        np.testing.assert_allclose(O.chol_solve(L, y), np.linalg.solve(A, y), rtol=1e-11, atol=1e-13)


def test_cholesky_rejects_indefinite():
    st, _ = O.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert st == -2


# ----------------------------------------------------------------- hierarchy
def test_hierarchy_levels_consistent():
    A = PB.poisson2d(40)
    h = O.Hierarchy(A, max_coarse=50)
    assert h.nlev >= 3
    for l in range(h.nlev - 1):
        Al, P, R = h.A(l), h.P(l), h.R(l)
        Ac = h.A(l + 1)
        assert np.array_equal(dense(R), dense(P).T)
        np.testing.assert_allclose(dense(Ac), dense(P).T @ dense(Al) @ dense(P), rtol=1e-12,
                                   atol=1e-13 * np.abs(dense(Al)).max())
        assert np.array_equal(pattern(Ac), (pattern(P).T.astype(int) @ pattern(Al).astype(int)
                                            @ pattern(P).astype(int)) > 0)
        np.testing.assert_allclose(h.dinv(l), 1.0 / np.diag(dense(Al)), rtol=0, atol=0)


def test_single_level_is_direct_solve():
    A = PB.poisson2d(10)                         # n = 100 <= max_coarse
    h = O.Hierarchy(A)
    assert h.nlev == 1
    b = PB.rhs(A.n)
    r = h.solve(b, 1e-8)
    assert r.status == O.OK and r.iters == 1
    np.testing.assert_allclose(dense(A) @ h.vcycle(b), b, rtol=0, atol=1e-12)
    L = h.chol()
    np.testing.assert_allclose(L, np.linalg.cholesky(dense(A)), rtol=1e-13, atol=1e-14)


def test_stalled_coarsening_is_last_level():
    # no negative couplings -> nothing is strong -> every point F -> the
    # level is the last one and solved directly
    n = 300
    M = np.eye(n) * 3 + np.diag(np.full(n - 1, 0.5), 1) + np.diag(np.full(n - 1, 0.5), -1)
    h = O.Hierarchy(from_dense(M), max_coarse=10)
    assert h.nlev == 1


def test_coarsest_too_large():
    n = 9000
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    v = np.ones(n)
    with pytest.raises(O.OracleError) as e:
        O.Hierarchy((n, n, rp, ci, v), max_coarse=10)
    assert e.value.status == O.E_COARSE


# ----------------------------------------------------------------- V-cycle
def _M_recursive(Al, Ps, omegas, l, nu1, nu2):
    """M_l from the two-grid iteration matrix (eq. twoGridOp) applied
    recursively: M_l = (I - E_l) A_l^{-1},
    E_l = S^nu2 (I - P M_{l+1} P^T A_l) S^nu1, S = I - omega D^{-1} A_l;
    on the last level M = A^{-1}.  A_{l+1} is formed here as P^T A_l P."""
    if l == len(Ps):
        return np.linalg.inv(Al)
    P = Ps[l]
    Ac = P.T @ Al @ P
    Mc = _M_recursive(Ac, Ps, omegas, l + 1, nu1, nu2)
    n = Al.shape[0]
    S = np.eye(n) - omegas[l] * Al / np.diag(Al)[:, None]
    E = np.linalg.matrix_power(S, nu2) @ (np.eye(n) - P @ Mc @ P.T @ Al) @ np.linalg.matrix_power(S, nu1)
    return (np.eye(n) - E) @ np.linalg.inv(Al)


@pytest.mark.parametrize("gen,mc,nu", [("p2", 40, 1), ("p2", 10, 1), ("ln2", 15, 1), ("p2", 20, 2),
                                        ("el", 30, 1)])
def test_vcycle_matches_iteration_matrix(gen, mc, nu):
    A = {"p2": lambda: PB.poisson2d(12), "ln2": lambda: PB.lognormal2d(11, 2.0),
         "el": lambda: PB.elasticity3d(2)}[gen]()
    h = O.Hierarchy(A, max_coarse=mc, nu_pre=nu, nu_post=nu)
    assert h.nlev >= 2
    Ps = [dense(h.P(l)) for l in range(h.nlev - 1)]
    om = [h.omega(l) for l in range(h.nlev - 1)]
    M = _M_recursive(dense(A), Ps, om, 0, nu, nu)
    Mo = np.stack([h.vcycle(e) for e in np.eye(A.n)], axis=1)
    np.testing.assert_allclose(Mo, M, rtol=0, atol=1e-12 * np.abs(M).max())


@pytest.mark.parametrize("gen", ["p2", "ln3", "el"])
def test_vcycle_symmetric_positive(gen):
    A = {"p2": lambda: PB.poisson2d(30), "ln3": lambda: PB.lognormal3d(10, 2.0),
         "el": lambda: PB.elasticity3d(4)}[gen]()
    h = O.Hierarchy(A, max_coarse=40)
    rng = np.random.default_rng(5)
    for _ in range(4):
        r1, r2 = rng.standard_normal(A.n), rng.standard_normal(A.n)
        a, b = r1 @ h.vcycle(r2), r2 @ h.vcycle(r1)
        assert abs(a - b) <= 1e-12 * abs(a)
        assert r1 @ h.vcycle(r1) > 0


# ----------------------------------------------------------------- PCG
@pytest.mark.parametrize("gen", ["p2", "ln3", "el", "an3"])
def test_pcg_matches_dense_solve(gen):
    A = {"p2": lambda: PB.poisson2d(30), "ln3": lambda: PB.lognormal3d(9, 2.0),
         "el": lambda: PB.elasticity3d(3), "an3": lambda: PB.aniso3d(9)}[gen]()
    h = O.Hierarchy(A, max_coarse=30, max_iter=2000)
    b = PB.rhs(A.n)
    r = h.solve(b, 1e-8, max_iter=2000)
    assert r.status == O.OK
    Ad = dense(A)
    xs = np.linalg.solve(Ad, b)
    assert np.linalg.norm(b - Ad @ r.x) / np.linalg.norm(b) < 1.5e-8
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(r.x - xs) <= kappa * 1e-8 * np.linalg.norm(xs)
    assert abs(r.true_relres - np.linalg.norm(b - Ad @ r.x) / np.linalg.norm(b)) < 1e-12
    assert r.hist[-1] < 1e-8 * np.linalg.norm(b) <= r.hist[-2]
    assert abs(r.hist[0] - np.linalg.norm(b)) <= 1e-14 * np.linalg.norm(b)


def test_cg_identity_finishes_within_n():
    rng = np.random.default_rng(6)
    for n in [8, 20, 64]:
        B = rng.standard_normal((n, n))
        Ad = B @ B.T / n + np.eye(n)
        h = O.Hierarchy(from_dense(Ad))
        b = rng.standard_normal(n)
        r = h.solve(b, 1e-10, max_iter=5 * n, precond=False)
        assert r.status == O.OK and r.iters <= n
        np.testing.assert_allclose(r.x, np.linalg.solve(Ad, b), rtol=1e-7, atol=1e-9)


def test_pcg_error_energy_norm_monotone():
    A = PB.lognormal2d(20, 2.0)
    h = O.Hierarchy(A, max_coarse=20)
    b = PB.rhs(A.n)
    Ad = dense(A)
    xs = np.linalg.solve(Ad, b)
    errs = []
    for k in range(1, 12):
        r = h.solve(b, 0.0, max_iter=k)            # rtol <= 0: exactly k iterations
        assert r.status == O.MAXIT and r.iters == k
        e = r.x - xs
        errs.append(e @ Ad @ e)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-10) for i in range(len(errs) - 1))


def test_pcg_zero_rhs_and_maxit_and_breakdown():
    A = PB.poisson2d(30)
    h = O.Hierarchy(A, max_coarse=30)
    r = h.solve(np.zeros(A.n), 1e-8)
    assert r.status == O.OK and r.iters == 0 and np.all(r.x == 0)
    r = h.solve(PB.rhs(A.n), 1e-8, max_iter=2)
    assert r.status == O.MAXIT and r.iters == 2 and len(r.hist) == 3
    # symmetric, positive diagonal, indefinite: a Laplacian plus a decoupled
    # 2x2 block [[1, 2], [2, 1]] (eigenvalues 3 and -1).  Its positive
    # couplings are never strong, so its points are F with empty P rows and
    # every coarse level stays SPD; b along the negative eigenvector makes
    # p.Ap < 0 at the first CG step.
    L = dense(PB.poisson2d(12))
    n = L.shape[0] + 2
    M = np.zeros((n, n))
    M[:-2, :-2] = L
    M[-2:, -2:] = [[1.0, 2.0], [2.0, 1.0]]
    hm = O.Hierarchy(from_dense(M), max_coarse=20)
    assert hm.nlev >= 2
    b = np.zeros(n)
    b[-2:] = [1.0, -1.0]
    r = hm.solve(b, 1e-8, precond=False)
    assert r.status == O.E_BREAKDOWN and r.iters == 0
    # the same matrix with no coarsening is caught by the direct factorisation
    with pytest.raises(O.OracleError) as e:
        O.Hierarchy(from_dense(M), max_coarse=1000)
    assert e.value.status == O.E_NOT_SPD
