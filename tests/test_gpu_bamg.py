"""BAMG prolongation on the GPU against the CPU oracle, through the C-ABI
(Section 2, Interpolation, eq. minBAMG, Alg. BAMG).  The set-up performs the
oracle's operations in its order, so every level must match bit for bit;
solves are compared as elsewhere."""
import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB
from tests.helpers import assert_fsai_close

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


CASES = {
    "elasticity_4_rbm": (lambda: PB.elasticity3d(4), lambda: PB.elasticity_rigid_modes(4), {}),
    "elasticity_6_rbm": (lambda: PB.elasticity3d(6), lambda: PB.elasticity_rigid_modes(6), {}),
    "elasticity_6_rbm_l1": (lambda: PB.elasticity3d(6), lambda: PB.elasticity_rigid_modes(6), {"bamg_lmax": 1}),
    "poisson2d_40_linear": (lambda: PB.poisson2d(40), lambda: _linear2d(40), {}),
    "lognormal3d_16_const": (lambda: PB.lognormal3d(16, 2.0), lambda: np.ones((16 ** 3, 1)), {}),
    "elasticity_6_rbm_smoothed": (lambda: PB.elasticity3d(6), lambda: PB.elasticity_rigid_modes(6), {"psmooth": 1}),
    "elasticity_6_rbm_filtered": (lambda: PB.elasticity3d(6), lambda: PB.elasticity_rigid_modes(6),
                                  {"psmooth": 1, "pfilter": 0.7}),
}


def _pair(camg, name, **extra):
    mkA, mkV, kw = CASES[name]
    A, V = mkA(), mkV()
    kw = dict(kw, **extra)
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), V=_dev(V),
                                interp=camg.INTERP_BAMG, max_coarse=40, **kw)
    o = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, max_coarse=40, **kw)
    return A, V, g, o


@pytest.mark.parametrize("name", list(CASES))
def test_bamg_hierarchy_bit_exact(camg, name):
    print(f"[gpu] bamg hierarchy {name}", flush=True)
    A, V, g, o = _pair(camg, name)
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
    g.close()


@pytest.mark.parametrize("name", ["elasticity_6_rbm", "poisson2d_40_linear"])
def test_bamg_solve_parity(camg, name):
    print(f"[gpu] bamg solve {name}", flush=True)
    A, V, g, o = _pair(camg, name)
    b = PB.rhs(A.n)
    ro = o.solve(b, 1e-8, max_iter=3000)
    r = g.solve(b)
    assert r.status == camg.OK and abs(r.iters - ro.iters) <= 1, (r.iters, ro.iters)
    assert np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    assert r.true_relres < 1e-8 * 1.01
    g.close()
    # host-array set-up gives the same hierarchy and solve
    h = camg.Solver(A, V=V, interp=camg.INTERP_BAMG, max_coarse=40, **CASES[name][2])
    rh = h.solve(b)
    assert rh.iters == r.iters and np.array_equal(rh.x, r.x)
    h.close()
    # mixed precision on the BAMG hierarchy
    gm = camg.Solver(A, V=V, interp=camg.INTERP_BAMG, max_coarse=40, precision=camg.MIXED_FP32)
    rm = gm.solve(b)
    assert rm.status == camg.OK and rm.true_relres < 1e-8
    assert np.linalg.norm(rm.x - ro.x) / np.linalg.norm(ro.x) < 1e-6
    gm.close()


def test_bamg_rejects_dependent_test_space(camg):
    A = PB.poisson2d(20)
    with pytest.raises(camg.CamgError) as e:
        camg.Solver(A, V=np.ones((A.n, 2)), interp=camg.INTERP_BAMG)
    assert e.value.status == camg.E_ARG


@pytest.mark.parametrize("name,kw", [("poisson2d_48", {"psmooth": 1, "pfilter": 0.8}),
                                     ("lognormal3d_16", {"psmooth": 1}),
                                     ("lognormal3d_16_f", {"psmooth": 1, "pfilter": 0.8, "interp": 2})])
def test_smoothed_prolongation_without_test_space(camg, name, kw):
    """Smoothing and filtering of the classical prolongations (the filter
    compensates on a unit vector): bit-exact hierarchies and solve parity."""
    print(f"[gpu] smoothed P {name}", flush=True)
    A = PB.poisson2d(48) if name.startswith("poisson") else PB.lognormal3d(16, 2.0)
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), max_coarse=40, **kw)
    o = O.Hierarchy(A, max_coarse=40, **kw)
    assert g.nlev == o.nlev
    for l in range(o.nlev - 1):
        gp, op = g.P(l), o.P(l)
        assert np.array_equal(gp[2], op[2]) and np.array_equal(gp[3], op[3]) and np.array_equal(gp[4], op[4])
        ga, oa = g.A(l + 1), o.A(l + 1)
        assert np.array_equal(ga[3], oa[3]) and np.array_equal(ga[4], oa[4])
    b = PB.rhs(A.n)
    r, ro = g.solve(b), o.solve(b, 1e-8)
    assert r.status == camg.OK and abs(r.iters - ro.iters) <= 1
    assert np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    g.close()


def test_over_filtered_prolongation_fails_like_the_oracle(camg):
    """Filtering to 0.6 of each row can empty a coarse column: the coarse
    operator then has a zero diagonal, which both sides report as not SPD."""
    A = PB.lognormal3d(16, 2.0)
    kw = {"psmooth": 1, "pfilter": 0.6, "interp": 2}
    with pytest.raises(O.OracleError) as eo:
        O.Hierarchy(A, max_coarse=40, **kw)
    with pytest.raises(camg.CamgError) as eg:
        camg.Solver(A, max_coarse=40, **kw)
    assert eo.value.status == O.E_NOT_SPD and eg.value.status == camg.E_NOT_SPD


def test_fsai_where_rows_fit_jacobi_elsewhere(camg):
    """BAMG on 8^3 elasticity with the FSAI_JACOBI smoother: levels 0 and 2
    smooth with FSAI, level 1 (212 entries on or below the diagonal in a
    row) with Jacobi.  Hierarchy and Jacobi weights bit for bit; the FSAI
    factors and their weights to rounding (the local solves substitute in
    different orders); V-cycle, FP64 and mixed solves as elsewhere."""
    print("[gpu] BAMG + FSAI where rows fit", flush=True)
    A, V = PB.elasticity3d(8), PB.elasticity_rigid_modes(8)
    kw = dict(max_coarse=40, smoother=2)
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), V=_dev(V),
                                interp=camg.INTERP_BAMG, **kw)
    o = O.Hierarchy(A, V=V, interp=O.INTERP_BAMG, **kw)
    assert g.nlev == o.nlev
    kinds = [o.has_G(l) for l in range(o.nlev - 1)]
    assert kinds[0] and not all(kinds), kinds
    for l in range(o.nlev):
        ga, oa = g.A(l), o.A(l)
        assert np.array_equal(ga[3], oa[3]) and np.array_equal(ga[4], oa[4]), l
        if l == o.nlev - 1:
            break
        gp, op = g.P(l), o.P(l)
        assert np.array_equal(gp[3], op[3]) and np.array_equal(gp[4], op[4]), l
        if kinds[l]:
            assert_fsai_close(g.G(l), o.G(l), f"_{l}")
            assert abs(g.omega(l) - o.omega(l)) <= 1e-12 * o.omega(l), l
        else:
            assert g.omega(l) == o.omega(l), l
            with pytest.raises(camg.CamgError):
                g.G(l)
    rng = np.random.default_rng(2)
    for _ in range(2):
        y = rng.standard_normal(A.n)
        dz = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        g.vcycle_dev(_dev(y), dz)
        torch.cuda.synchronize()
        zo = o.vcycle(y)
        assert np.linalg.norm(dz.cpu().numpy() - zo) / np.linalg.norm(zo) <= 1e-10
    b = PB.rhs(A.n)
    ro = o.solve(b, 1e-8, max_iter=3000)
    r = g.solve(b)
    assert r.status == camg.OK and abs(r.iters - ro.iters) <= 1, (r.iters, ro.iters)
    assert np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    g.close()
    gm = camg.Solver(A, V=V, interp=camg.INTERP_BAMG, precision=camg.MIXED_FP32, **kw)
    rm = gm.solve(b)
    assert rm.status == camg.OK and rm.true_relres < 1e-8
    assert np.linalg.norm(rm.x - ro.x) / np.linalg.norm(ro.x) < 1e-6
    gm.close()
