"""SRQM refinement of the BAMG test space on the GPU against the CPU oracle,
through the C-ABI (Section 2, near-kernel passage, eq. eigP).  The device
follows the oracle's operations in its order (Gram sums over rows in index
order, the dense Rayleigh-Ritz step and the Jacobi eigensolver in the same
sequence), so the refined space, and every level built from it, must match
bit for bit."""
import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def camg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_07417_amd import camg as C
    C.load()
    return C


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _linear2d(g):
    n = g * g
    return np.stack([np.ones(n), (np.arange(n) % g) / g, (np.arange(n) // g) / g], 1)


def _eigvecs(A, k):
    import scipy.sparse as sp
    Ad = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n)).toarray()
    return np.ascontiguousarray(np.linalg.eigh(Ad)[1][:, :k])


CASES = {
    "elasticity_6_rbm_1": (lambda: PB.elasticity3d(6), lambda A: PB.elasticity_rigid_modes(6), {"srqm_iters": 1}),
    "elasticity_6_rbm_4": (lambda: PB.elasticity3d(6), lambda A: PB.elasticity_rigid_modes(6), {"srqm_iters": 4}),
    "elasticity_4_random_8": (lambda: PB.elasticity3d(4),
                              lambda A: np.random.default_rng(5).standard_normal((A.n, 6)), {"srqm_iters": 8}),
    "elasticity_16_rbm_3": (lambda: PB.elasticity3d(16), lambda A: PB.elasticity_rigid_modes(16),
                            {"srqm_iters": 3}),
    "poisson2d_40_linear_3": (lambda: PB.poisson2d(40), lambda A: _linear2d(40), {"srqm_iters": 3}),
    # FSAI on a 7-point matrix: the local systems' Cholesky factors couple
    # the last unknown only, so the oracle's and the device's substitution
    # orders add the same nonzero terms in the same order and level 0's G
    # (the only one SRQM applies) is the same bit for bit
    "lognormal3d_16_const_fsai_5": (lambda: PB.lognormal3d(16, 2.0), lambda A: np.ones((A.n, 1)),
                                    {"srqm_iters": 5, "smoother": 1}),
    "lognormal3d_16_two_fsai_3": (lambda: PB.lognormal3d(16, 2.0),
                                  lambda A: np.random.default_rng(2).standard_normal((A.n, 2)),
                                  {"srqm_iters": 3, "smoother": 1}),
    "elasticity_6_rbm_3_smoothed_filtered": (lambda: PB.elasticity3d(6), lambda A: PB.elasticity_rigid_modes(6),
                                             {"srqm_iters": 3, "psmooth": 1, "pfilter": 0.7}),
    # an exact invariant subspace: the refinement stops before its first update
    "poisson2d_20_eigvecs": (lambda: PB.poisson2d(20), lambda A: _eigvecs(A, 3), {"srqm_iters": 5}),
}


def _pair(camg, name):
    mkA, mkV, kw = CASES[name]
    A = mkA()
    V = mkV(A)
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), V=_dev(V),
                                interp=camg.INTERP_BAMG, max_coarse=40, **kw)
    o = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=40, **kw)
    return A, V, g, o


def _assert_same(g, o):
    assert g.nlev == o.nlev, (g.nlev, o.nlev)
    for l in range(o.nlev):
        ga, oa = g.A(l), o.A(l)
        assert np.array_equal(ga[2], oa[2]) and np.array_equal(ga[3], oa[3]), f"A_{l} pattern"
        assert np.array_equal(ga[4], oa[4]), f"A_{l} values"
        if l == o.nlev - 1:
            break
        assert np.array_equal(g.cf(l), o.cf(l)), f"cf_{l}"
        gp, op = g.P(l), o.P(l)
        assert np.array_equal(gp[2], op[2]) and np.array_equal(gp[3], op[3]), f"P_{l} pattern"
        assert np.array_equal(gp[4], op[4]), f"P_{l} values"


@pytest.mark.parametrize("name", list(CASES))
def test_srqm_hierarchy_bit_exact(camg, name):
    print(f"[gpu] srqm hierarchy {name}", flush=True)
    A, V, g, o = _pair(camg, name)
    _assert_same(g, o)
    g.close()


def test_srqm_changes_the_prolongation(camg):
    """The option is live on the device: one step moves level 0's P away
    from the one built on the supplied space."""
    A, V = PB.elasticity3d(6), PB.elasticity_rigid_modes(6)
    g0 = camg.Solver(A, V=V, interp=camg.INTERP_BAMG, max_coarse=40)
    g1 = camg.Solver(A, V=V, interp=camg.INTERP_BAMG, max_coarse=40, srqm_iters=1)
    p0, p1 = g0.P(0), g1.P(0)
    assert not (np.array_equal(p0[3], p1[3]) and np.array_equal(p0[4], p1[4]))
    g0.close()
    g1.close()


def test_exact_space_stops_like_no_refinement(camg):
    """An exact invariant subspace is left as it is; only the second
    orthonormalisation of the (already orthonormal) basis moves its entries,
    by rounding."""
    A = PB.poisson2d(20)
    V = _eigvecs(A, 3)
    g0 = camg.Solver(A, V=V, interp=camg.INTERP_BAMG, max_coarse=40)
    g5 = camg.Solver(A, V=V, interp=camg.INTERP_BAMG, max_coarse=40, srqm_iters=5)
    assert g0.nlev == g5.nlev
    for l in range(g0.nlev - 1):
        p0, p5 = g0.P(l), g5.P(l)
        assert np.array_equal(p0[2], p5[2]) and np.array_equal(p0[3], p5[3])
        np.testing.assert_allclose(p5[4], p0[4], rtol=0, atol=1e-11)
    g0.close()
    g5.close()


def test_srqm_solve_parity(camg):
    print("[gpu] srqm solve elasticity_4_random_8", flush=True)
    A, V, g, o = _pair(camg, "elasticity_4_random_8")
    b = PB.rhs(A.n)
    ro = o.solve(b, 1e-8, max_iter=3000)
    r = g.solve(b)
    assert r.status == camg.OK and abs(r.iters - ro.iters) <= 1, (r.iters, ro.iters)
    assert np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    assert r.true_relres < 1e-8 * 1.01
    g.close()
    # host-array set-up gives the same hierarchy and solve
    h = camg.Solver(A, V=V, interp=camg.INTERP_BAMG, max_coarse=40, srqm_iters=8)
    rh = h.solve(b)
    assert rh.iters == r.iters and np.array_equal(rh.x, r.x)
    h.close()
