"""Pins of the oracle's adaptive FSAI factor (Section 2, eq. smo; the
adaptive pattern search of the FSAI package the paper cites), checked
against what the mathematics fixes: the closed form of the factor of the
1D Laplacian on a band, the inverse Cholesky factor once the pattern is
the whole lower triangle, a brute-force greedy search written with dense
numpy algebra, the Kaporin optimality conditions on the final pattern,
monotonicity in the number of steps, the tie rule, the stopping rule, and
the level fallback when a candidate set is too large."""
import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB

from helpers import dense, from_dense, pattern


def _aG(A, steps, step, eps):
    st, G, mc = O.afsai(A, steps, step, eps)
    assert st == O.OK
    return G, mc


def _rows(G):
    n, _, rp, ci, v = G
    return [(list(ci[rp[i]:rp[i + 1]]), v[rp[i]:rp[i + 1]]) for i in range(n)]


def _lap1d(n):
    return from_dense(2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))


def _arrow(n):
    """Diagonal 4 with the last row and column coupled to every point."""
    M = 4.0 * np.eye(n)
    M[-1, :-1] = M[:-1, -1] = -1.0
    M[-1, -1] = 2.0 * n
    return from_dense(M)


def _brute(A, steps, step, eps, follow):
    """The greedy pattern search, written again with dense numpy algebra:
    minimise g^T A g (g_i = 1) on the pattern, add the candidates with the
    largest |(A g)_j|, stop on the step count, on a small decrease of psi,
    or when no candidate has a nonzero gradient component.  Where the last
    places of a step tie to 1e-9 (symmetric stencils tie exactly, and
    rounding then decides), any of the tied candidates is a correct choice:
    those in the pattern `follow` (the oracle's) are taken first, so that the
    comparison checks what is unique and that the rest is a valid choice."""
    Ad, S = dense(A), pattern(A)
    n = Ad.shape[0]
    G = np.zeros((n, n))
    pats, maxcand = [], 0
    for i in range(n):
        P = [i]
        psi_prev, k = 0.0, 0
        while True:
            e = np.zeros(len(P)); e[-1] = 1.0
            y = np.linalg.solve(Ad[np.ix_(P, P)], e)
            psi = 1.0 / y[-1]
            if k == steps or (k > 0 and psi_prev - psi <= eps * psi_prev):
                break
            psi_prev = psi
            cand = sorted({int(j) for c in P for j in np.nonzero(S[c])[0] if j < i and j not in P})
            maxcand = max(maxcand, len(cand))
            z = {}
            for j in cand:  # row j of A against the pattern, one rounding per operation
                s = 0.0
                for c, yc in zip(P, y):
                    if S[j, c]:
                        s = s + float(Ad[j, c]) * float(yc)
                z[j] = s
            order = sorted((j for j in cand if z[j] != 0.0), key=lambda j: (-abs(z[j]), j))
            if not order:
                break
            take = order[:step]
            if len(order) > step:
                zb = abs(z[order[step - 1]])
                tied = [j for j in order if abs(abs(z[j]) - zb) <= 1e-9 * zb]
                sure = [j for j in take if j not in tied]
                need = step - len(sure)
                pref = [j for j in tied if j in follow[i]] + [j for j in tied if j not in follow[i]]
                take = sure + pref[:need]
            P = sorted(P + take)
            k += 1
        G[i, P] = y / np.sqrt(y[-1])
        pats.append(P)
    return G, pats, maxcand


def test_afsai_no_steps_is_diagonal_scaling():
    for A in (PB.lognormal2d(7, 2.0), PB.elasticity3d(2)):
        G, mc = _aG(A, 0, 2, 0.0)
        Gd = dense(G)
        d = np.diag(dense(A))
        np.testing.assert_allclose(np.diag(Gd), 1.0 / np.sqrt(d), rtol=1e-15)
        assert np.count_nonzero(Gd - np.diag(np.diag(Gd))) == 0 and mc == 0


@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_afsai_1d_laplacian_band_closed_form(k):
    """tridiag(-1, 2, -1): one entry per step is the next lower neighbour,
    so after k steps row i holds columns max(0, i-k)..i.  With c = min(i, k)
    the minimiser on that band is g_{i-d} = (c+1-d)/(c+1) and
    psi_i = (c+2)/(c+1) (the Green's function of the band's Dirichlet
    problem), so G(i, i-d) = g_{i-d} / sqrt(psi_i)."""
    n = 15
    G, mc = _aG(_lap1d(n), k, 1, 0.0)
    assert mc == 1
    for i, (cols, vals) in enumerate(_rows(G)):
        c = min(i, k)
        assert cols == list(range(i - c, i + 1))
        d = np.arange(c, -1, -1)
        want = (c + 1 - d) / (c + 1) / np.sqrt((c + 2) / (c + 1))
        np.testing.assert_allclose(vals, want, rtol=1e-13)


@pytest.mark.parametrize("n,steps,step", [(5, 4, 1), (9, 8, 1), (9, 1, 8), (12, 4, 3)])
def test_afsai_full_pattern_is_inverse_cholesky_factor(n, steps, step):
    """Dense SPD: every row reaches the whole lower triangle, so
    G A G^T = I and G = L^{-1} with A = L L^T."""
    rng = np.random.default_rng(n * 7 + step)
    B = rng.standard_normal((n, n))
    Ad = B @ B.T + n * np.eye(n)
    G, mc = _aG(from_dense(Ad), steps, step, 0.0)
    Gd = dense(G)
    assert mc == n - 1
    np.testing.assert_allclose(Gd @ Ad @ Gd.T, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(Gd, np.linalg.inv(np.linalg.cholesky(Ad)), rtol=1e-10, atol=1e-12)


_GENS = {"ln2": lambda: PB.lognormal2d(8, 2.0), "ln3": lambda: PB.lognormal3d(5, 2.0),
         "el": lambda: PB.elasticity3d(2), "an3": lambda: PB.aniso3d(5, 1e-2)}


@pytest.mark.parametrize("gen", sorted(_GENS))
@pytest.mark.parametrize("steps,step,eps", [(3, 1, 0.0), (4, 2, 0.02), (2, 3, 0.0), (6, 2, 0.005)])
def test_afsai_matches_brute_force(gen, steps, step, eps):
    A = _GENS[gen]()
    G, mc = _aG(A, steps, step, eps)
    Gb, pats, mcb = _brute(A, steps, step, eps, [r[0] for r in _rows(G)])
    assert mc == mcb
    for i, (cols, vals) in enumerate(_rows(G)):
        assert cols == pats[i], f"row {i}"
        np.testing.assert_allclose(vals, Gb[i, cols], rtol=1e-11, atol=0)


@pytest.mark.parametrize("gen", sorted(_GENS))
def test_afsai_kaporin_optimality_on_its_pattern(gen):
    """On its final pattern each row is the constrained minimiser: the
    gradient (G A)_ij vanishes for j in P_i other than i, (G A)_ii = 1/G_ii,
    and G A G^T has a unit diagonal; G is lower triangular with at most
    steps * step + 1 entries per row and a positive diagonal."""
    A = _GENS[gen]()
    steps, step = 5, 2
    G, _ = _aG(A, steps, step, 0.01)
    Ad, Gd = dense(A), dense(G)
    GA = Gd @ Ad
    scale = np.abs(GA).max(axis=1)
    for i, (cols, vals) in enumerate(_rows(G)):
        assert cols[-1] == i and all(c < i for c in cols[:-1]) and len(cols) <= steps * step + 1
        assert vals[-1] > 0
        for c in cols[:-1]:
            assert abs(GA[i, c]) <= 1e-13 * scale[i]
        assert abs(GA[i, i] * Gd[i, i] - 1.0) <= 1e-13
    np.testing.assert_allclose(np.diag(Gd @ Ad @ Gd.T), 1.0, rtol=0, atol=1e-13)


def test_afsai_more_steps_never_raise_psi():
    """psi_i = 1 / G_ii^2 is minimised over a growing pattern, so G_ii
    cannot decrease as the step count grows (eps = 0)."""
    A = PB.lognormal3d(5, 2.0)
    prev = None
    for k in range(0, 5):
        d = np.diag(dense(_aG(A, k, 2, 0.0)[0]))
        if prev is not None:
            assert np.all(d >= prev * (1 - 1e-14))
        prev = d


def test_afsai_ties_go_to_the_smaller_index():
    """5-point Poisson: the two lower neighbours of a row tie (|a| = 1).
    With one entry the south one (i - nx, the smaller index) joins:
    local matrix [[4, -1], [-1, 4]], y = (1, 4) / 15, psi = 15 / 4.  With
    two entries per step the pattern is the lower triangle of A, so the
    factor is the static one, bit for bit."""
    nx = 6
    A = PB.poisson2d(nx)
    G, _ = _aG(A, 1, 1, 0.0)
    for i, (cols, vals) in enumerate(_rows(G)):
        if i == 0:
            assert cols == [0]
            continue
        j = i - nx if i >= nx else i - 1
        assert cols == [j, i]
        np.testing.assert_allclose(vals, np.array([0.25, 1.0]) / np.sqrt(3.75), rtol=1e-15)
    G2, _ = _aG(A, 1, 2, 0.0)
    st, Gs = O.fsai(A)
    assert st == O.OK
    for a, b in zip(G2[2:], Gs[2:]):
        np.testing.assert_array_equal(a, b)


def test_afsai_stopping_rule():
    """A tolerance no decrease can meet stops every row after its first
    growth step; eps = 0 keeps growing up to the step count."""
    A = PB.lognormal2d(8, 2.0)
    G1, _ = _aG(A, 1, 2, 0.0)
    Gbig, _ = _aG(A, 5, 2, 1.0)
    for a, b in zip(G1[2:], Gbig[2:]):
        np.testing.assert_array_equal(a, b)
    G5, _ = _aG(A, 5, 2, 0.0)
    assert G5[2][-1] > G1[2][-1]


def test_afsai_level_falls_back_to_jacobi_when_candidates_overflow():
    n = O.AFSAI_MAXCAND + 52
    A = _arrow(n)
    st, G, mc = O.afsai(A, 1, 1, 0.0)
    assert st == O.OK and mc == n - 1 > O.AFSAI_MAXCAND
    h = O.Hierarchy(A, max_coarse=50, smoother=O.SMOOTH_AFSAI, afsai_steps=1, afsai_step=1, afsai_eps=0.0)
    assert not h.has_G(0)
    np.testing.assert_array_equal(h.omega(0), O.gershgorin_omega(A))
    # below the limit the level uses the adaptive factor, bit for bit
    B = PB.lognormal2d(12, 2.0)
    hb = O.Hierarchy(B, max_coarse=20, smoother=O.SMOOTH_AFSAI, afsai_steps=4, afsai_step=2, afsai_eps=0.01)
    Gb, _ = _aG(B, 4, 2, 0.01)
    for a, b in zip(hb.G(0)[2:], Gb[2:]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("kw", [dict(afsai_steps=16, afsai_step=2), dict(afsai_steps=-1),
                                dict(afsai_step=0), dict(afsai_eps=-1e-3), dict(afsai_eps=float("nan"))])
def test_afsai_parameter_errors(kw):
    A = PB.poisson2d(20)
    with pytest.raises(O.OracleError):
        O.Hierarchy(A, smoother=O.SMOOTH_AFSAI, **kw)
    st, G, _ = O.afsai(A, kw.get("afsai_steps", 10), kw.get("afsai_step", 2), kw.get("afsai_eps", 0.01))
    assert st == O.E_ARG and G is None


@pytest.mark.parametrize("gen,mc", [("ln2", 15), ("el", 30)])
def test_afsai_vcycle_matches_iteration_matrix(gen, mc):
    """The V-cycle with the adaptive factor is the two-grid recursion with
    S = I - omega G^T G A (eq. twoGridOp, eq. smoother, eq. smo)."""
    from test_oracle_fsai import _M_fsai
    A = {"ln2": lambda: PB.lognormal2d(11, 2.0), "el": lambda: PB.elasticity3d(2)}[gen]()
    h = O.Hierarchy(A, max_coarse=mc, smoother=O.SMOOTH_AFSAI, afsai_steps=4, afsai_step=2, afsai_eps=0.01)
    assert h.nlev >= 2
    Ps = [dense(h.P(l)) for l in range(h.nlev - 1)]
    Gs = [dense(h.G(l)) for l in range(h.nlev - 1)]
    om = [h.omega(l) for l in range(h.nlev - 1)]
    for l in range(h.nlev - 1):
        np.testing.assert_array_equal(Gs[l], dense(_aG(h.A(l), 4, 2, 0.01)[0]))
        assert O.fsai_omega(h.A(l), h.G(l), h.params.seed, l) == om[l]
    M = _M_fsai(dense(A), Ps, Gs, om, 0, 1, 1)
    Mo = np.stack([h.vcycle(e) for e in np.eye(A.n)], axis=1)
    np.testing.assert_allclose(Mo, M, rtol=0, atol=1e-12 * np.abs(M).max())
    assert np.linalg.eigvalsh((Mo + Mo.T) / 2).min() > 0


def test_afsai_pcg_converges_faster_than_jacobi_on_elasticity():
    A = PB.elasticity3d(4)
    b = PB.rhs(A.n)
    rj = O.Hierarchy(A, max_coarse=30).solve(b, 1e-8)
    ra = O.Hierarchy(A, max_coarse=30, smoother=O.SMOOTH_AFSAI).solve(b, 1e-8)
    assert rj.status == O.OK and ra.status == O.OK
    assert np.linalg.norm(b - dense(A) @ ra.x) / np.linalg.norm(b) < 1.5e-8
    assert ra.iters < rj.iters


def test_afsai_selected_rows_match_all_rows():
    A = PB.elasticity3d(3)
    G, _ = _aG(A, 6, 3, 0.005)
    rows = [0, 1, 5, 17, A.n // 2, A.n - 1]
    for (cols, vals), i in zip(O.afsai_rows(A, rows, 6, 3, 0.005), rows):
        gc, gv = _rows(G)[i]
        assert list(cols) == gc
        np.testing.assert_array_equal(vals, gv)
