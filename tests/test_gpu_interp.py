"""The paper's classical, extended+i and hybrid interpolations on the GPU
against the CPU oracle, through the C-ABI (Section 2, Interpolation;
Alg. extintset).

The set-up kernels add every sum in the oracle's order, so all levels of
the hierarchy (strength, C/F split, P, R, A_l) must match bit for bit; the
V-cycle and PCG are compared as in the direct-interpolation tests."""
import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB
from tests.helpers import hub_graph, wide_stencil_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VARIANTS = ["classical", "exti", "hybrid"]
CASES = {
    "poisson2d_64": lambda: PB.poisson2d(64),
    "poisson2d_ragged_37x23": lambda: PB.poisson2d(37, 23),
    "lognormal3d_24": lambda: PB.lognormal3d(24, 2.0),
    "aniso3d_20": lambda: PB.aniso3d(20, 1e-3),
    "elasticity_6": lambda: PB.elasticity3d(6),
    "lognormal2d_90": lambda: PB.lognormal2d(90, 2.0),
    # rows with more than 256 candidate C points: the workgroup-per-row path
    "wide_stencil_40_r5": lambda: wide_stencil_2d(40, 5),
}


@pytest.fixture(scope="module")
def camg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_07417_amd import camg as C
    C.load()
    return C


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _csr(A):
    if hasattr(A, "row_ptr"):
        return A.n, A.row_ptr, A.col_idx, A.val
    return A[0], A[2], A[3], A[4]


def _pair(camg, A, variant, **kw):
    n, rp, ci, v = _csr(A)
    g = camg.Solver.from_device(n, _dev(rp), _dev(ci), _dev(v), interp=getattr(camg, "INTERP_" + variant.upper()),
                                **kw)
    o = O.Hierarchy(A, interp=getattr(O, "INTERP_" + variant.upper()), **kw)
    return g, o


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", list(CASES))
def test_interp_hierarchy_bit_exact(camg, name, variant):
    print(f"[gpu] interp hierarchy {name} {variant}", flush=True)
    A = CASES[name]()
    g, o = _pair(camg, A, variant, max_coarse=40)
    assert g.nlev == o.nlev, (g.nlev, o.nlev)
    for l in range(o.nlev):
        ga, oa = g.A(l), o.A(l)
        assert np.array_equal(ga[2], oa[2]) and np.array_equal(ga[3], oa[3]), f"A_{l} pattern"
        assert np.array_equal(ga[4], oa[4]), f"A_{l} values"
        if l == o.nlev - 1:
            break
        assert np.array_equal(g.strong(l), o.strong(l)), f"strong_{l}"
        assert np.array_equal(g.cf(l), o.cf(l)), f"cf_{l}"
        for what in ("P", "R"):
            gp, op = getattr(g, what)(l), getattr(o, what)(l)
            assert gp[:2] == op[:2]
            assert np.array_equal(gp[2], op[2]) and np.array_equal(gp[3], op[3]), f"{what}_{l} pattern"
            assert np.array_equal(gp[4], op[4]), f"{what}_{l} values"
    g.close()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["lognormal3d_24", "aniso3d_20", "elasticity_6"])
def test_interp_vcycle_and_solve_parity(camg, name, variant):
    print(f"[gpu] interp solve {name} {variant}", flush=True)
    A = CASES[name]()
    g, o = _pair(camg, A, variant, max_coarse=40)
    y = np.random.default_rng(7).standard_normal(A.n)
    dz = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    g.vcycle_dev(_dev(y), dz)
    torch.cuda.synchronize()
    zo = o.vcycle(y)
    assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-12 * np.linalg.norm(zo)
    b = PB.rhs(A.n)
    ro = o.solve(b, 1e-8, max_iter=3000)
    assert ro.status == O.OK
    db, dx = _dev(b), torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    rg = g.solve_dev(db, dx, rtol=1e-8, hist_cap=3001)
    assert rg.status == camg.OK and abs(rg.iters - ro.iters) <= 1, (rg.iters, ro.iters)
    assert np.linalg.norm(dx.cpu().numpy() - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    assert rg.true_relres < 1e-8 * 1.01
    g.close()
    # equal iteration count (parity mode)
    g2, _ = _pair(camg, A, variant, max_coarse=40, max_iter=ro.iters)
    dx2 = torch.zeros_like(dx)
    r2 = g2.solve_dev(db, dx2, rtol=0.0)
    assert r2.status == camg.E_MAXIT and r2.iters == ro.iters
    assert np.linalg.norm(dx2.cpu().numpy() - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    g2.close()


def test_interp_multi_rhs_mixed_and_batch(camg):
    """The block engine, the mixed-precision V-cycle and the many-systems
    kernel take any P: extended+i hierarchies run through all three."""
    A = PB.lognormal3d(16, 2.0)
    k = 3
    B = PB.rhs_block(A.n, k)
    o = O.Hierarchy(A, interp=O.INTERP_EXTI)
    g = camg.Solver(A, interp=camg.INTERP_EXTI)
    dB = _dev(B)
    dX = torch.zeros_like(dB)
    r = g.solve_multi_dev(dB, dX)
    X = dX.cpu().numpy()
    assert r.status == camg.OK
    for j in range(k):
        ro = o.solve(B[:, j], 1e-8)
        assert abs(int(r.iters[j]) - ro.iters) <= 1
        assert np.linalg.norm(X[:, j] - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    g.close()
    gm = camg.Solver(A, interp=camg.INTERP_EXTI, precision=camg.MIXED_FP32)
    b = B[:, 0]
    rm = gm.solve(b)
    ro = o.solve(b, 1e-8)
    assert rm.status == camg.OK and rm.true_relres < 1e-8
    assert np.linalg.norm(rm.x - ro.x) / np.linalg.norm(ro.x) < 1e-6
    gm.close()
    hs = [camg.Solver(PB.poisson2d(20 + 3 * s), interp=camg.INTERP_HYBRID, max_coarse=40) for s in range(3)]
    bs = [_dev(PB.rhs(h.n)) for h in hs]
    xs = [torch.zeros_like(x) for x in bs]
    its, _, sts = camg.solve_batch_dev(hs, bs, xs)
    for s, h in enumerate(hs):
        A2 = PB.poisson2d(20 + 3 * s)
        ro = O.Hierarchy(A2, interp=O.INTERP_HYBRID, max_coarse=40).solve(PB.rhs(A2.n), 1e-8)
        assert sts[s] == camg.OK and abs(int(its[s]) - ro.iters) <= 1
        assert np.linalg.norm(xs[s].cpu().numpy() - ro.x) / np.linalg.norm(ro.x) <= 1e-9
        h.close()


def test_interp_full_size_lognormal_128(camg):
    """Level 0 of the 128^3 lognormal problem (n = 2,097,152): the GPU's
    extended+i P equals the oracle's, formed from the GPU's strength flags
    and C/F split (themselves checked bit for bit at the smaller sizes), and
    the solve converges in fewer iterations than with direct interpolation."""
    print("[gpu] interp full size lognormal3d_128", flush=True)
    A = PB.lognormal3d(128, 2.0)
    b = PB.rhs(A.n)
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), interp=camg.INTERP_EXTI)
    P = g.P(0)
    Po = O.interp(A, g.strong(0), g.cf(0), O.INTERP_EXTI)
    assert P[:2] == Po[:2]
    assert np.array_equal(P[2], Po[2]) and np.array_equal(P[3], Po[3]) and np.array_equal(P[4], Po[4])
    db, dx = _dev(b), torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    r = g.solve_dev(db, dx, rtol=1e-8)
    assert r.status == camg.OK and r.true_relres < 1e-8 * 1.01
    g.close()
    gd = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val))
    rd = gd.solve_dev(db, torch.zeros_like(dx), rtol=1e-8)
    assert r.iters < rd.iters, (r.iters, rd.iters)
    gd.close()


@pytest.mark.parametrize("variant", ["direct", "exti"])
@pytest.mark.parametrize("name", ["lognormal3d_24", "elasticity_6", "poisson2d_ragged_37x23"])
def test_chunked_galerkin_bit_exact(camg, name, variant):
    """A tiny rap_chunk forces the Galerkin product into many windows of
    coarse rows; every level must still equal the oracle's bit for bit."""
    print(f"[gpu] chunked galerkin {name} {variant}", flush=True)
    A = CASES[name]()
    code = variant.upper()
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), max_coarse=40,
                                interp=getattr(camg, "INTERP_" + code), rap_chunk=2000)
    o = O.Hierarchy(A, max_coarse=40, interp=getattr(O, "INTERP_" + code))
    assert g.nlev == o.nlev
    for l in range(o.nlev):
        ga, oa = g.A(l), o.A(l)
        assert np.array_equal(ga[2], oa[2]) and np.array_equal(ga[3], oa[3]), f"A_{l} pattern"
        assert np.array_equal(ga[4], oa[4]), f"A_{l} values"
    g.close()


@pytest.mark.parametrize("variant", ["direct", "exti"])
@pytest.mark.parametrize("g", [40, 100])
def test_transpose_long_rows(camg, g, variant):
    """A hub point that every grid point interpolates from: R has one row
    of g^2 + 1 entries (1601: sorted by a workgroup in LDS; 10001: from a global
    copy).  The hierarchy must match the oracle bit for bit and the solve
    must agree."""
    print(f"[gpu] long transpose rows hub {g} {variant}", flush=True)
    A = hub_graph(g)
    n, rp, ci, v = _csr(A)
    code = getattr(camg, "INTERP_" + variant.upper())
    gs = camg.Solver.from_device(n, _dev(rp), _dev(ci), _dev(v), max_coarse=40, interp=code)
    o = O.Hierarchy(A, max_coarse=40, interp=getattr(O, "INTERP_" + variant.upper()))
    assert gs.nlev == o.nlev == 2
    for what in ("P", "R"):
        gp, op = getattr(gs, what)(0), getattr(o, what)(0)
        assert np.array_equal(gp[2], op[2]) and np.array_equal(gp[3], op[3]) and np.array_equal(gp[4], op[4])
    assert np.diff(gs.R(0)[2]).max() == g * g + 1   # the grid points and the hub itself
    b = np.random.default_rng(g).uniform(-1.0, 1.0, n)
    r, ro = gs.solve(b), o.solve(b, 1e-8)
    assert r.status == camg.OK and abs(r.iters - ro.iters) <= 1
    assert np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    gs.close()
