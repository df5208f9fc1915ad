"""GPU library against the CPU oracle, through the C-ABI.

Set-up: the GPU kernels perform the oracle's floating-point operations in
the oracle's order, so every level (A_l, P_l, R_l, C/F split, strong flags,
D^{-1}, omega) must match bit for bit.  Solve: the V-cycle and the CG dot
products use different summation orders, so solutions are compared to
1e-9 relative (iteration counts within one).
"""
import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB
from tests.helpers import assert_fsai_close, dense, from_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _camg():
    from paper_2102_07417_amd import camg
    camg.load()
    return camg


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


CASES = {
    "poisson2d_64": lambda: PB.poisson2d(64),
    "poisson2d_ragged_37x23": lambda: PB.poisson2d(37, 23),
    "lognormal3d_24": lambda: PB.lognormal3d(24, 2.0),
    "aniso3d_20": lambda: PB.aniso3d(20, 1e-3),
    "elasticity_6": lambda: PB.elasticity3d(6),
    "lognormal2d_90": lambda: PB.lognormal2d(90, 2.0),
    # rows of 2 to several hundred entries in one matrix: lane groups of the
    # set-up kernels see ragged rows
    "powerlaw_graph_3000": lambda: PB.powerlaw_graph(3000),
}


@pytest.fixture(scope="module")
def camg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return _camg()


def _pair(camg, A, **kw):
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), **kw)
    okw = {k: v for k, v in kw.items() if k in ("theta", "seed", "nu_pre", "nu_post", "omega", "max_levels",
                                                "max_coarse", "max_iter")}
    o = O.Hierarchy(A, **okw)
    return g, o


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_bit_exact(camg, name):
    print(f"[gpu] hierarchy {name}", flush=True)
    A = CASES[name]()
    g, o = _pair(camg, A, max_coarse=40)
    assert g.nlev == o.nlev, (g.nlev, o.nlev)
    for l in range(o.nlev):
        ga, oa = g.A(l), o.A(l)
        assert np.array_equal(ga[2], oa[2]) and np.array_equal(ga[3], oa[3]), f"A_{l} pattern"
        assert np.array_equal(ga[4], oa[4]), f"A_{l} values"
        if l == o.nlev - 1:
            break
        assert np.array_equal(g.strong(l), o.strong(l)), f"strong_{l}"
        assert np.array_equal(g.cf(l), o.cf(l)), f"cf_{l}"
        assert g.omega(l) == o.omega(l)
        assert np.array_equal(g.dinv(l), o.dinv(l))
        for what in ("P", "R"):
            gp, op = getattr(g, what)(l), getattr(o, what)(l)
            assert gp[:2] == op[:2]
            assert np.array_equal(gp[2], op[2]) and np.array_equal(gp[3], op[3]), f"{what}_{l} pattern"
            assert np.array_equal(gp[4], op[4]), f"{what}_{l} values"
    # last level: dense inverse against numpy
    Ad = dense(g.A(g.nlev - 1))
    np.testing.assert_allclose(g.coarse_inverse(), np.linalg.inv(Ad), rtol=0,
                               atol=1e-11 * np.abs(np.linalg.inv(Ad)).max())
    g.close()


@pytest.mark.parametrize("name", ["poisson2d_64", "lognormal3d_24", "elasticity_6"])
def test_vcycle_matches_oracle(camg, name):
    print(f"[gpu] vcycle {name}", flush=True)
    A = CASES[name]()
    g, o = _pair(camg, A, max_coarse=40)
    rng = np.random.default_rng(11)
    for _ in range(3):
        y = rng.standard_normal(A.n)
        dz = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        g.vcycle_dev(_dev(y), dz)
        torch.cuda.synchronize()
        zo = o.vcycle(y)
        err = np.linalg.norm(dz.cpu().numpy() - zo) / np.linalg.norm(zo)
        assert err <= 1e-12, err
    g.close()


@pytest.mark.parametrize("name", list(CASES))
def test_solve_parity(camg, name):
    print(f"[gpu] solve {name}", flush=True)
    A = CASES[name]()
    b = PB.rhs(A.n)
    g, o = _pair(camg, A, max_iter=3000)
    ro = o.solve(b, 1e-8, max_iter=3000)
    assert ro.status == O.OK
    db, dx = _dev(b), torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    rg = g.solve_dev(db, dx, rtol=1e-8, hist_cap=3001)
    x = dx.cpu().numpy()
    assert rg.status == camg.OK
    assert abs(rg.iters - ro.iters) <= 1, (rg.iters, ro.iters)
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    assert rg.true_relres < 1e-8 * 1.01
    np.testing.assert_allclose(rg.hist[:5], ro.hist[:5], rtol=1e-10)
    # equal iteration count (parity mode): exactly the oracle's count
    g2, _ = _pair(camg, A, max_iter=ro.iters)
    dx2 = torch.zeros_like(dx)
    r2 = g2.solve_dev(db, dx2, rtol=0.0)
    assert r2.status == camg.E_MAXIT and r2.iters == ro.iters
    assert np.linalg.norm(dx2.cpu().numpy() - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    g.close()
    g2.close()


def test_solve_host_api_and_determinism(camg):
    A = PB.lognormal3d(20, 2.0)
    b = PB.rhs(A.n)
    s = camg.Solver(A)
    r1 = s.solve(b)
    r2 = s.solve(b)
    assert r1.status == camg.OK and r1.iters == r2.iters
    assert np.array_equal(r1.x, r2.x) and np.array_equal(r1.hist, r2.hist)
    s.close()


def test_galerkin_exact_integer(camg):
    rng = np.random.default_rng(3)
    A = PB.poisson2d(9)
    for nc in (1, 7, 30):
        P = rng.integers(-2, 3, size=(A.n, nc)).astype(float)
        P[rng.random(P.shape) > 0.3] = 0.0
        from tests.helpers import from_dense
        Pc = from_dense(P, keep_zero_diag=False)
        C = camg.camg_galerkin((A.n, A.n, A.row_ptr, A.col_idx, A.val), Pc)
        assert np.array_equal(dense(C), P.T @ dense(A) @ P)
        Co = O.galerkin((A.n, A.n, A.row_ptr, A.col_idx, A.val), Pc)
        assert np.array_equal(C[2], Co[2]) and np.array_equal(C[3], Co[3])


def test_galerkin_rows_beyond_the_lds_tables(camg):
    """A row of A P with more distinct columns than the largest LDS hash table
    (16384 slots) and more entries than the largest LDS fill bin takes the
    global-table symbolic and fill passes; the product still equals the
    oracle's entry by entry (integer data, so exactly)."""
    print("[gpu] galerkin with a 20001-column row", flush=True)
    n = 20001
    # arrow matrix: point 0 coupled to every other point
    rp = np.zeros(n + 1, np.int32)
    rp[1] = n
    rp[2:] = n + 2 * np.arange(1, n)
    ci = np.empty(rp[-1], np.int32)
    v = np.empty(rp[-1])
    ci[:n] = np.arange(n)
    v[:n] = -1.0
    v[0] = 2.0 * n
    ci[n::2] = 0
    ci[n + 1::2] = np.arange(1, n)
    v[n::2] = -1.0
    v[n + 1::2] = 4.0
    A = (n, n, rp, ci, v)
    # P: every point to itself, and points 1.. also to coarse point (i % 7)
    prp = np.zeros(n + 1, np.int32)
    pci, pv = [], []
    for i in range(n):
        cols = sorted({i % 7, 7 + i}) if i else [7]
        pci += cols
        pv += [1.0 if c >= 7 else 2.0 for c in cols]
        prp[i + 1] = len(pci)
    P = (n, n + 7, prp, np.array(pci, np.int32), np.array(pv))
    C = camg.camg_galerkin(A, P)
    Co = O.galerkin(A, P)
    assert np.array_equal(C[2], Co[2]) and np.array_equal(C[3], Co[3])
    assert np.array_equal(C[4], Co[4])
    assert np.diff(C[2]).max() > 16384


def test_single_level_and_tiny(camg):
    for A in [PB.poisson2d(1), PB.poisson2d(3), PB.poisson2d(16)]:
        b = PB.rhs(A.n)
        s = camg.Solver(A)
        r = s.solve(b)
        assert s.nlev == 1 and r.status == camg.OK and r.iters == 1
        np.testing.assert_allclose(r.x, np.linalg.solve(dense((A.n, A.n, A.row_ptr, A.col_idx, A.val)), b),
                                   rtol=1e-12, atol=1e-14)
        s.close()


def test_zero_rhs_and_maxit(camg):
    A = PB.poisson2d(40)
    s = camg.Solver(A, max_iter=3)
    r = s.solve(np.zeros(A.n))
    assert r.status == camg.OK and r.iters == 0 and np.all(r.x == 0)
    r = s.solve(PB.rhs(A.n))
    assert r.status == camg.E_MAXIT and r.iters == 3 and len(r.hist) == 4
    s.close()


def test_invalid_inputs(camg):
    from tests.test_oracle import _bad
    for kind in ["rp_dec", "col_range", "col_order", "nan", "nodiag", "asym", "negdiag"]:
        A, code = _bad(kind)
        n, _, rp, ci, v = A
        st, h = camg.camg_setup(n, rp, ci, v)
        assert st == code, (kind, st)
        assert not h.value
    st, h = camg.camg_setup(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert st == camg.E_ARG
    bad = camg.params(nu_pre=0)
    A = PB.poisson2d(5)
    st, h = camg.camg_setup(A.n, A.row_ptr, A.col_idx, A.val, bad)
    assert st == camg.E_ARG


def test_breakdown_on_indefinite(camg):
    L = dense(PB.poisson2d(12))
    n = L.shape[0] + 2
    M = np.zeros((n, n))
    M[:-2, :-2] = L
    M[-2:, -2:] = [[1.0, 2.0], [2.0, 1.0]]
    from tests.helpers import from_dense
    n_, _, rp, ci, v = from_dense(M)
    s = camg.Solver(PB.CSR(n, rp, ci, v), max_coarse=20)
    b = np.zeros(n)
    b[-2:] = [1.0, -1.0]
    r = s.solve(b)
    assert r.status in (camg.E_BREAKDOWN,)
    s.close()
    st, h = camg.camg_setup(n, rp, ci, v, camg.params(max_coarse=1000))
    assert st == camg.E_NOT_SPD


def test_full_size_lognormal_128(camg):
    """The benchmark's workload at full size: hierarchy bit-exact on every
    level and the FP64 solve within 1e-9 of the oracle's."""
    print("[gpu] full-size lognormal3d_128", flush=True)
    A = PB.workload("lognormal3d_128")
    b = PB.rhs(A.n)
    g, o = _pair(camg, A)
    assert g.nlev == o.nlev
    for l in range(o.nlev):
        ga, oa = g.A(l), o.A(l)
        assert np.array_equal(ga[3], oa[3]) and np.array_equal(ga[4], oa[4]), l
    dx = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    rg = g.solve_dev(_dev(b), dx, rtol=1e-8)
    ro = o.solve(b, 1e-8)
    assert abs(rg.iters - ro.iters) <= 1
    assert np.linalg.norm(dx.cpu().numpy() - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    assert rg.true_relres < 1e-8 * 1.01
    g.close()


def test_graph_replays_match_direct_launches(camg):
    """Each PCG iteration runs as a captured graph; replays across several
    solves, with unrelated eager GPU work in between, must give bitwise the
    same iterates as launching the kernels one by one."""
    A = PB.lognormal3d(20, 2.0)
    b1, b2 = PB.rhs(A.n, 1), PB.rhs(A.n, 2)
    s = camg.Solver(A)
    assert camg.camg_set_option(s.h, camg.OPT_GRAPH, 0) == camg.OK
    d1, d2 = s.solve(b1), s.solve(b2)
    assert camg.camg_set_option(s.h, camg.OPT_GRAPH, 1) == camg.OK
    g1 = s.solve(b1)
    t = torch.randn(1 << 20, device="cuda:0")
    float(t.sum())
    torch.cuda.synchronize()
    g2 = s.solve(b2)
    g1b = s.solve(b1)
    for d, g in [(d1, g1), (d2, g2), (d1, g1b)]:
        assert d.iters == g.iters and np.array_equal(d.x, g.x) and np.array_equal(d.hist, g.hist)
    s.close()


def test_two_iteration_graphs_stop_at_max_iter(camg):
    """Untimed iterations go two per graph launch: with rtol = 0 every
    iteration count, odd or even, stops exactly at max_iter with the iterates
    of direct launches, with and without the kernel timing that splits
    every few iterations into single launches."""
    A = PB.lognormal3d(16, 2.0)
    b = PB.rhs(A.n, 3)
    for m in [1, 2, 3, 4, 7, 8]:
        for prof in [0, 4]:
            s = camg.Solver(A, max_iter=m)
            assert camg.camg_set_option(s.h, camg.OPT_GRAPH, 0) == camg.OK
            d = s.solve(b, rtol=0.0)
            assert camg.camg_set_option(s.h, camg.OPT_GRAPH, 1) == camg.OK
            if prof:
                camg.camg_profile(s.h, prof)
            g = s.solve(b, rtol=0.0)
            if prof:
                camg.camg_profile(s.h, 0)
            assert d.status == g.status == camg.E_MAXIT and d.iters == g.iters == m, (m, prof, d.iters, g.iters)
            assert np.array_equal(d.x, g.x) and np.array_equal(d.hist, g.hist), (m, prof)
            s.close()


@pytest.mark.parametrize("name", ["lognormal3d_24", "elasticity_6", "aniso3d_20"])
def test_mixed_precision_reaches_fp64_tolerance(camg, name):
    """FP32 V-cycle inside FP64 PCG: the true residual still drops below
    rtol; the error against the FP64 oracle solution is reported."""
    print(f"[gpu] mixed {name}", flush=True)
    A = CASES[name]()
    b = PB.rhs(A.n)
    o = O.Hierarchy(A, max_iter=3000)
    ro = o.solve(b, 1e-8, max_iter=3000)
    s = camg.Solver(A, precision=camg.MIXED_FP32, max_iter=3000)
    r = s.solve(b, rtol=1e-8)
    err = np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x)
    print(f"[gpu] mixed {name}: iters {r.iters} (fp64 oracle {ro.iters}) true_relres {r.true_relres:.2e} "
          f"err_vs_oracle {err:.2e}", flush=True)
    assert r.status == camg.OK and r.true_relres < 1e-8
    assert r.iters <= ro.iters + 5
    assert err < 1e-6
    s.close()


def test_kernel_timing_hook(camg):
    A = PB.lognormal3d(24, 2.0)
    b = PB.rhs(A.n)
    s = camg.Solver(A)
    camg.camg_profile(s.h, 1)
    r = s.solve(b)
    ms, launches = camg.camg_profile(s.h, 0)
    assert launches == r.iters and ms > 0
    # every 4th iteration (k = 3, 7, ...), same solution bits as untimed solves
    camg.camg_profile(s.h, 4)
    r4 = s.solve(b)
    ms4, launches4 = camg.camg_profile(s.h, 0)
    assert launches4 == r4.iters // 4 and ms4 > 0
    r0 = s.solve(b)
    assert np.array_equal(r4.x, r0.x) and np.array_equal(r.x, r0.x)
    s.close()
    # a one-level hierarchy has no post-smoothing kernel to time, and the FSAI
    # post-smoothing (two kernels) is timed between stream events
    A1 = PB.lognormal3d(12, 2.0)
    for A2, kw in ((A1, {"max_coarse": 5000}), (A, {"smoother": camg.SMOOTH_FSAI})):
        b2 = PB.rhs(A2.n)
        s = camg.Solver(A2, **kw)
        assert s.nlev == (1 if "max_coarse" in kw else s.nlev)
        camg.camg_profile(s.h, 1)
        r = s.solve(b2)
        ms, launches = camg.camg_profile(s.h, 0)
        assert r.status == camg.OK and launches == r.iters and ms >= 0.0, kw
        if "smoother" in kw:
            assert ms > 0.0
        s.close()


# ----------------------------------------------------------------- multi-RHS
@pytest.mark.parametrize("name,k", [("lognormal3d_24", 5), ("poisson2d_64", 32), ("elasticity_6", 3)])
def test_multi_rhs_matches_oracle(camg, name, k):
    print(f"[gpu] multi {name} k={k}", flush=True)
    A = CASES[name]()
    B = PB.rhs_block(A.n, k)
    o = O.Hierarchy(A, max_iter=3000)
    s = camg.Solver(A, max_iter=3000)
    dB = torch.from_numpy(B).to("cuda:0")
    dX = torch.zeros_like(dB)
    r = s.solve_multi_dev(dB, dX, rtol=1e-8)
    X = dX.cpu().numpy()
    assert r.status == camg.OK
    for c in range(k):
        ro = o.solve(B[:, c], 1e-8, max_iter=3000)
        assert abs(int(r.iters[c]) - ro.iters) <= 1, (c, r.iters[c], ro.iters)
        assert np.linalg.norm(X[:, c] - ro.x) / np.linalg.norm(ro.x) <= 1e-9
        assert r.true_relres[c] < 1e-8 * 1.01
    # agrees with the single-vector path to rounding
    rs = s.solve(B[:, 0])
    assert np.linalg.norm(X[:, 0] - rs.x) / np.linalg.norm(rs.x) <= 1e-9
    s.close()


def test_multi_rhs_edge_cases(camg):
    """More columns than slots (chunks of 64), a zero column, one level."""
    for A, k in [(PB.poisson2d(16), 70), (PB.poisson2d(3), 5)]:
        print(f"[gpu] multi edge n={A.n} k={k}", flush=True)
        B = PB.rhs_block(A.n, k)
        B[:, 2] = 0.0
        s = camg.Solver(A)
        o = O.Hierarchy(A)
        dB = torch.from_numpy(B).to("cuda:0")
        dX = torch.full_like(dB, 7.0)
        r = s.solve_multi_dev(dB, dX, rtol=1e-8)
        X = dX.cpu().numpy()
        assert r.status == camg.OK
        assert r.iters[2] == 0 and np.all(X[:, 2] == 0.0)
        for c in (0, 1, k - 1):
            ro = o.solve(B[:, c], 1e-8)
            assert abs(int(r.iters[c]) - ro.iters) <= 1
            assert np.linalg.norm(X[:, c] - ro.x) / np.linalg.norm(ro.x) <= 1e-9
        s.close()


def test_multi_rhs_mixed_precision(camg):
    A = PB.lognormal3d(24, 2.0)
    B = PB.rhs_block(A.n, 8)
    s = camg.Solver(A, precision=camg.MIXED_FP32)
    dB = torch.from_numpy(B).to("cuda:0")
    dX = torch.zeros_like(dB)
    r = s.solve_multi_dev(dB, dX, rtol=1e-8)
    assert r.status == camg.OK and np.all(r.true_relres < 1e-8)
    o = O.Hierarchy(A)
    X = dX.cpu().numpy()
    for c in (0, 7):
        ro = o.solve(B[:, c], 1e-8)
        assert np.linalg.norm(X[:, c] - ro.x) / np.linalg.norm(ro.x) < 1e-6
    s.close()


def test_engine_column_alone_equals_in_mix(camg):
    """Continuous batching: a column's result is bitwise the same alone and
    among other columns started before and after it, in another slot."""
    A = PB.lognormal3d(20, 2.0)
    s = camg.Solver(A)
    b = torch.from_numpy(PB.rhs(A.n, 99)).to("cuda:0")
    others = torch.from_numpy(PB.rhs_block(A.n, 7, 5)).to("cuda:0")
    e = camg.Engine(s, 8, hist_cap=200)
    e.start(3, b)
    while e.step(4):
        pass
    xa = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    it_a = e.state()[0][3]
    e.finish(3, xa)
    # now: four columns first, b joins later in slot 6, more join after
    e.start(0, others[:, :4])
    e.step(3)
    e.start(6, b)
    e.step(2)
    e.start(4, others[:, 4:6])
    while e.step(5):
        pass
    it, dn, st = e.state()
    assert dn[6] == 1 and st[6] == 0 and it[6] == it_a
    xb = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    e.finish(6, xb)
    assert torch.equal(xa, xb)
    e.close()
    s.close()


def test_multi_rhs_autotuned_schedules_are_bitwise_equal(camg):
    """The autotuner only picks among schedules that add the same products in
    the same order: tuned and untuned engines give identical bits."""
    for prec in (camg.FP64, camg.MIXED_FP32):
        A = PB.lognormal3d(20, 2.0)
        B = torch.from_numpy(PB.rhs_block(A.n, 8)).to("cuda:0")
        outs = []
        for tune in (0, 1):
            s = camg.Solver(A, precision=prec)
            s.set_option(camg.OPT_AUTOTUNE, tune)
            X = torch.zeros_like(B)
            r = s.solve_multi_dev(B, X, rtol=1e-8)
            assert r.status == camg.OK
            outs.append(X)
            s.close()
        assert torch.equal(outs[0], outs[1])


def test_multi_rhs_stripe_sweep(camg):
    """Block sweeps in stripes: on a 32^3 Poisson grid a row's farthest
    neighbour is a plane (1024 rows) away, and 64 FP64 columns make a block
    row 512 bytes, so the planes' gathered rows outgrow the stripe budget
    (1.5 MiB over five stripe-planes: 614 rows) and the level-0 sweeps run
    stripe by stripe.  The columns match the oracle, and a column alone on a
    64-slot engine equals the same column inside the 64-column block bit for
    bit."""
    print("[gpu] multi stripe sweep", flush=True)
    A = PB.poisson3d(32)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert np.abs(A.col_idx - rows).max() == 1024
    k = 64
    B = PB.rhs_block(A.n, k)
    s = camg.Solver(A, max_iter=3000)
    dB = torch.from_numpy(B).to("cuda:0")
    dX = torch.zeros_like(dB)
    r = s.solve_multi_dev(dB, dX, rtol=1e-8)
    assert r.status == camg.OK and np.all(r.true_relres < 1e-8 * 1.01)
    X = dX.cpu().numpy()
    o = O.Hierarchy(A, max_iter=3000)
    for c in (0, 31, 63):
        ro = o.solve(B[:, c], 1e-8, max_iter=3000)
        assert abs(int(r.iters[c]) - ro.iters) <= 1, (c, r.iters[c], ro.iters)
        assert np.linalg.norm(X[:, c] - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    e = camg.Engine(s, 64, hist_cap=200)
    e.start(5, dB[:, 17].contiguous())
    while e.step(8):
        pass
    xa = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    assert e.state()[0][5] == r.iters[17]
    e.finish(5, xa)
    assert torch.equal(xa, dX[:, 17].contiguous())
    e.close()
    s.close()


# ----------------------------------------------------------------- FSAI smoother
FSAI_CASES = ["poisson2d_64", "lognormal3d_24", "aniso3d_20", "elasticity_6"]


@pytest.mark.parametrize("name", FSAI_CASES)
def test_fsai_hierarchy_vcycle_and_solve(camg, name):
    print(f"[gpu] fsai {name}", flush=True)
    A = CASES[name]()
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), max_coarse=40,
                                smoother=camg.SMOOTH_FSAI)
    o = O.Hierarchy(A, max_coarse=40, smoother=O.SMOOTH_FSAI)
    assert g.nlev == o.nlev
    for l in range(o.nlev - 1):
        assert_fsai_close(g.G(l), o.G(l), f"_{l}")
        assert abs(g.omega(l) - o.omega(l)) <= 1e-12 * o.omega(l), f"omega_{l}"
    rng = np.random.default_rng(3)
    for _ in range(2):
        y = rng.standard_normal(A.n)
        dz = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        g.vcycle_dev(_dev(y), dz)
        torch.cuda.synchronize()
        zo = o.vcycle(y)
        assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
    b = PB.rhs(A.n)
    r = g.solve(b)
    ro = o.solve(b, 1e-8)
    assert r.status == camg.OK and abs(r.iters - ro.iters) <= 1
    assert np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    g.close()


def test_fsai_two_steps_and_mixed(camg):
    A = PB.lognormal3d(20, 2.0)
    b = PB.rhs(A.n)
    g = camg.Solver(A, smoother=camg.SMOOTH_FSAI, nu_pre=2, nu_post=2)
    o = O.Hierarchy(A, smoother=O.SMOOTH_FSAI, nu_pre=2, nu_post=2)
    y = np.random.default_rng(4).standard_normal(A.n)
    dz = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    g.vcycle_dev(_dev(y), dz)
    torch.cuda.synchronize()
    zo = o.vcycle(y)
    assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
    r, ro = g.solve(b), o.solve(b, 1e-8)
    assert abs(r.iters - ro.iters) <= 1 and np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    g.close()
    gm = camg.Solver(A, smoother=camg.SMOOTH_FSAI, precision=camg.MIXED_FP32)
    rm = gm.solve(b)
    ro1 = O.Hierarchy(A, smoother=O.SMOOTH_FSAI).solve(b, 1e-8)
    assert rm.status == camg.OK and rm.true_relres < 1e-8 and rm.iters <= ro1.iters + 5
    assert np.linalg.norm(rm.x - ro1.x) / np.linalg.norm(ro1.x) < 1e-6
    # the block engine and the many-systems kernel run Jacobi only
    B = torch.from_numpy(PB.rhs_block(A.n, 2)).to("cuda:0")
    with pytest.raises(camg.CamgError):
        gm.solve_multi_dev(B, torch.zeros_like(B))
    db = _dev(b)
    with pytest.raises(camg.CamgError):
        camg.solve_batch_dev([gm], [db], [torch.zeros_like(db)])
    gm.close()


# ----------------------------------------------------------------- compact columns
def _far_coupled_chain(n=100_000, far=9_000, reach=9):
    """1D Laplacian plus weak couplings of i with i + far, ..., i + reach*far
    for every 1000th i: a tile holding such a row needs more than the eight
    windows of 8192 columns that compact columns allow."""
    import scipy.sparse as sp
    main = 2.2 * np.ones(n)
    A = sp.diags([-np.ones(n - 1), main, -np.ones(n - 1)], [-1, 0, 1], format="lil")
    for i in range(0, n - reach * far, 1000):
        for k in range(1, reach + 1):
            j = i + k * far
            A[i, j] = A[j, i] = -0.1
            A[i, i] += 0.1
            A[j, j] += 0.1
    A = A.tocsr()
    A.sort_indices()
    return PB.CSR(n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


def _poisson3d_box(nx, ny, nz):
    """7-point Poisson on an nx x ny x nz box (Dirichlet), x fastest."""
    import scipy.sparse as sp

    def lap(m):
        return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])

    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    A = (sp.kron(Iz, sp.kron(Iy, lap(nx))) + sp.kron(Iz, sp.kron(lap(ny), Ix)) + sp.kron(lap(nz), sp.kron(Iy, Ix)))
    A = sp.csr_matrix(A)
    A.sort_indices()
    return PB.CSR(A.shape[0], A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


@pytest.mark.parametrize("name,kw", [("lognormal3d_24", {}), ("lognormal3d_24", {"precision": 1}),
                                     ("lognormal3d_24", {"smoother": 1}), ("elasticity_6", {})])
def test_compact_columns_bitwise(camg, name, kw):
    """Row kernels reading 16-bit column differences give bitwise the
    iterates of the int32 columns (same products, same sums)."""
    print(f"[gpu] compact columns {name} {kw}", flush=True)
    A = CASES[name]()
    b = PB.rhs(A.n)
    s = camg.Solver(A, **kw)
    assert s.info.compact_cols & 1, "A_0 should carry compact columns"
    r1 = s.solve(b)
    y = np.random.default_rng(5).standard_normal(A.n)
    z1 = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    s.vcycle_dev(_dev(y), z1)
    s.set_option(camg.OPT_COMPACT_COLS, 0)
    r0 = s.solve(b)
    z0 = torch.zeros_like(z1)
    s.vcycle_dev(_dev(y), z0)
    torch.cuda.synchronize()
    assert r1.iters == r0.iters and np.array_equal(r1.x, r0.x)
    assert torch.equal(z1, z0)
    s.set_option(camg.OPT_COMPACT_COLS, 1)
    r2 = s.solve(b)
    assert np.array_equal(r2.x, r1.x)
    s.close()


def test_compact_columns_with_several_windows(camg):
    """A 260 x 260 x 3 grid: its planes of 67,600 unknowns put each tile's
    columns into three bands, beyond one 65536-column span; the windows of
    the compact columns cover them, bitwise like the int32 columns and within
    the oracle's tolerance."""
    print("[gpu] compact columns: several windows", flush=True)
    A = _poisson3d_box(260, 260, 3)
    b = PB.rhs(A.n)
    s = camg.Solver(A)
    assert s.info.compact_cols & 1
    r1 = s.solve(b)
    s.set_option(camg.OPT_COMPACT_COLS, 0)
    r0 = s.solve(b)
    assert r1.iters == r0.iters and np.array_equal(r1.x, r0.x)
    ro = O.Hierarchy(A).solve(b, 1e-8)
    assert abs(r1.iters - ro.iters) <= 1
    assert np.linalg.norm(r1.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    s.close()


def test_wide_tiles_keep_int32_columns(camg):
    print("[gpu] compact columns: wide tiles", flush=True)
    A = _far_coupled_chain()
    b = PB.rhs(A.n)
    s = camg.Solver(A, max_iter=3000)
    assert not (s.info.compact_cols & 1)
    r = s.solve(b)
    o = O.Hierarchy(A, max_iter=3000)
    ro = o.solve(b, 1e-8, max_iter=3000)
    assert r.status == camg.OK and abs(r.iters - ro.iters) <= 1
    assert np.linalg.norm(r.x - ro.x) / np.linalg.norm(ro.x) <= 1e-9
    s.close()


@pytest.mark.parametrize("n", [1, 15, 16, 17, 100, 255, 256, 257, 400])
def test_last_level_factor_sizes(camg, n):
    """The last level's factorisation (blocked on the matrix cores up to 256
    unknowns, unblocked above) across panel edges: its inverse against
    numpy, and a one-level solve against a dense solve."""
    rng = np.random.default_rng(n)
    d = 2.0 + rng.random(n)
    Ad = np.diag(d) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    if n > 20:  # a few long-range couplings so the factor is not banded
        for i in range(0, n - 17, 7):
            Ad[i, i + 17] = Ad[i + 17, i] = -0.3
            Ad[i, i] += 0.3
            Ad[i + 17, i + 17] += 0.3
    def csr(M):
        n_, _, rp, ci, v = from_dense(M)
        return PB.CSR(n_, rp, ci, v)

    s = camg.Solver(csr(Ad), max_coarse=1000)
    assert s.nlev == 1
    inv = np.linalg.inv(Ad)
    np.testing.assert_allclose(s.coarse_inverse(), inv, rtol=0, atol=1e-12 * np.abs(inv).max())
    b = PB.rhs(n)
    r = s.solve(b)
    assert r.status == camg.OK
    np.testing.assert_allclose(r.x, np.linalg.solve(Ad, b), rtol=0, atol=1e-11 * np.abs(np.linalg.solve(Ad, b)).max())
    s.close()
    # an indefinite last level is refused by either factorisation
    Ai = Ad.copy()
    Ai[n // 2, n // 2] = -1.0
    with pytest.raises(camg.CamgError) as e:
        camg.Solver(csr(Ai), max_coarse=1000)
    assert e.value.status == camg.E_NOT_SPD


def _band_with_hubs(n=20_000, half=40, hubs=(1_234, 9_876, 17_000), reach=3_000, seed=11):
    """A symmetric band of 2*half + 1 entries per row (mean row length over
    64, so the FP32 row kernels take the pipelined tile loop) plus a few hub
    rows coupled to `reach` points each: those rows exceed one 2048-entry
    tile, leaving empty tiles and tiles beyond two streaming steps.  Weakly
    diagonally dominant with negative couplings, hence SPD."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for d in range(1, half + 1):
        i = np.arange(n - d)
        rows.append(i)
        cols.append(i + d)
    for h in hubs:
        j = rng.choice(np.setdiff1d(np.arange(n), np.arange(h - half, h + half + 1)), reach, replace=False)
        rows.append(np.minimum(h, j))
        cols.append(np.maximum(h, j))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    w = -rng.uniform(0.5, 1.5, r.size)
    U = sp.coo_matrix((w, (r, c)), shape=(n, n)).tocsr()
    U.sum_duplicates()
    A = U + U.T
    A = A + sp.diags(1.05 * np.asarray(-A.sum(axis=1)).ravel())
    A = A.tocsr()
    A.sort_indices()
    return PB.CSR(n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


def test_pipelined_fp32_tiles(camg):
    """Mixed precision on long rows: the FP32 V-cycle within FP32 rounding of
    the oracle's, compact and int32 column words bitwise alike, and the
    solve to a true residual below 1e-8."""
    print("[gpu] pipelined FP32 tiles: band with hubs", flush=True)
    A = _band_with_hubs()
    assert A.row_ptr[-1] / A.n >= 64 and np.diff(A.row_ptr).max() > 2048
    b = PB.rhs(A.n)
    o = O.Hierarchy(A, max_iter=3000)
    s = camg.Solver(A, precision=camg.MIXED_FP32, max_iter=3000)
    assert s.nlev == o.nlev and s.info.compact_cols & 1
    y = np.random.default_rng(6).standard_normal(A.n)
    zo = o.vcycle(y)
    z1 = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    s.vcycle_dev(_dev(y), z1)
    torch.cuda.synchronize()
    err = np.linalg.norm(z1.cpu().numpy() - zo) / np.linalg.norm(zo)
    print(f"[gpu] FP32 V-cycle against the oracle: {err:.2e}", flush=True)
    assert err <= 2e-5
    r1 = s.solve(b)
    assert r1.status == camg.OK and r1.true_relres < 1e-8
    s.set_option(camg.OPT_COMPACT_COLS, 0)
    z0 = torch.zeros_like(z1)
    s.vcycle_dev(_dev(y), z0)
    r0 = s.solve(b)
    torch.cuda.synchronize()
    assert torch.equal(z1, z0)
    assert r0.iters == r1.iters and np.array_equal(r0.x, r1.x)
    s.close()
