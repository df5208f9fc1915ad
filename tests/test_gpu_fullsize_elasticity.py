"""The mechanics workload at full size (Q1 elasticity on 64^3 elements,
n = 811,200, nnz = 63,695,790, bottom face clamped) on the GPU against the
CPU oracle, in the set-up the benchmark times: every level of the direct and
of the BAMG + SRQM hierarchy bit for bit, one V-cycle, and a fixed number of
PCG iterations in FP64 and in mixed precision (the oracle's full solve, about
600 iterations, is too slow for a test; the GPU solves to 1e-8 are checked by
their true residuals)."""
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


@pytest.fixture(scope="module")
def c3():
    A = PB.elasticity3d(64)
    return A, PB.rhs(A.n), PB.elasticity_rigid_modes(64)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _same_levels(g, o):
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


@pytest.mark.timeout(600)
def test_direct_hierarchy_vcycle_and_pcg(camg, c3):
    A, b, _ = c3
    print("[gpu] full-size elasticity 64^3: direct hierarchy", flush=True)
    rp, ci, va = _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val)
    g = camg.Solver.from_device(A.n, rp, ci, va, max_iter=5)
    o = O.Hierarchy(A, max_iter=5)
    _same_levels(g, o)
    # one V-cycle
    y = np.random.default_rng(3).standard_normal(A.n)
    dz = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    g.vcycle_dev(_dev(y), dz)
    torch.cuda.synchronize()
    zo = o.vcycle(y)
    assert np.linalg.norm(dz.cpu().numpy() - zo) / np.linalg.norm(zo) <= 1e-12
    # five PCG iterations (rtol 0 runs exactly max_iter)
    ro = o.solve(b, 0.0, max_iter=5)
    db, dx = _dev(b), torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    r = g.solve_dev(db, dx, rtol=0.0)
    assert r.status == camg.E_MAXIT and r.iters == 5
    err = np.linalg.norm(dx.cpu().numpy() - ro.x) / np.linalg.norm(ro.x)
    print(f"[gpu] FP64, 5 iterations: relative difference {err:.2e}", flush=True)
    assert err <= 1e-12  # measured 1.8e-15
    g.close()
    # mixed precision (FP32 V-cycle): its difference from the FP64 oracle after
    # five iterations is the FP32 preconditioner's
    gm = camg.Solver.from_device(A.n, rp, ci, va, max_iter=5, precision=camg.MIXED_FP32)
    dxm = torch.zeros_like(dx)
    rm = gm.solve_dev(db, dxm, rtol=0.0)
    assert rm.iters == 5
    errm = np.linalg.norm(dxm.cpu().numpy() - ro.x) / np.linalg.norm(ro.x)
    print(f"[gpu] mixed, 5 iterations: relative difference {errm:.2e}", flush=True)
    assert errm <= 1e-6  # measured 3.8e-8
    gm.close()
    # the full solves reach the true residual
    for prec in (camg.FP64, camg.MIXED_FP32):
        gs = camg.Solver.from_device(A.n, rp, ci, va, max_iter=5000, precision=prec)
        dx.zero_()
        rs = gs.solve_dev(db, dx, rtol=1e-8)
        assert rs.status == camg.OK and rs.true_relres < 1e-8 * 1.01, (prec, rs.status, rs.true_relres)
        gs.close()


@pytest.mark.timeout(600)
def test_bamg_srqm_hierarchy_bit_exact(camg, c3):
    A, _, V = c3
    print("[gpu] full-size elasticity 64^3: BAMG + 3 SRQM steps", flush=True)
    kw = dict(interp=camg.INTERP_BAMG, srqm_iters=3)
    g = camg.Solver.from_device(A.n, _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val), V=_dev(V), **kw)
    o = O.Hierarchy(A, V=V, **kw)
    _same_levels(g, o)
    g.close()
