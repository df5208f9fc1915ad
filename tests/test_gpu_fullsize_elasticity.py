"""The mechanics workload at full size (Q1 elasticity on 64^3 elements,
n = 811,200, nnz = 63,695,790, bottom face clamped) on the GPU against the
CPU oracle, in the set-up the benchmark times: every level of the direct and
of the BAMG + SRQM hierarchy bit for bit, one V-cycle, five PCG iterations
in FP64 and in mixed precision, and the natural-stop solves against the
oracle's full solve (about 600 iterations, too slow to run in a test: it is
read from tests/golden/oracle_solve_elasticity_64.txt, written by
tests/golden/make_oracle_solves.py from the oracle alone)."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_oracle_solves as GOLD  # noqa: E402

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


@pytest.mark.timeout(600)
def test_natural_stop_against_oracle_solve(camg, c3):
    """FP64: iterations within one of the oracle's at the natural stop
    (rtol 1e-8), and at the oracle's iteration count (parity mode, rtol 0)
    x within 1e-9 relative on the oracle's 4096 sampled unknowns, the
    residual history beside the oracle's.  Mixed precision: true residual
    below 1e-8 and its error against the oracle's FP64 solution stated."""
    A, b, _ = c3
    g = GOLD.read("elasticity_64")
    assert g["n"] == A.n and g["nnz"] == A.nnz and g["status"] == 0
    ko, idx, xo, ho = g["iters"], g["idx"], g["x"], g["hist"]
    print(f"[gpu] full-size elasticity 64^3: natural stop vs oracle ({ko} iterations)", flush=True)
    rp, ci, va = _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val)
    db = _dev(b)
    dx = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")

    def rel_on_samples(x):
        return np.linalg.norm(x[idx] - xo) / np.linalg.norm(xo)

    s = camg.Solver.from_device(A.n, rp, ci, va, max_iter=5000)
    r = s.solve_dev(db, dx, rtol=1e-8, hist_cap=ko + 10)
    x = dx.cpu().numpy()
    hg = np.asarray(r.hist)
    m = min(len(hg), len(ho))
    hdiff = np.abs(hg[:m] - ho[:m]) / ho[:m]
    print(f"[gpu] FP64 natural stop: {r.iters} iterations (oracle {ko}), true_relres {r.true_relres:.3e} "
          f"(oracle {g['true_relres']:.3e}), sampled rel diff {rel_on_samples(x):.2e}, "
          f"history max rel diff {hdiff.max():.2e} (first 100: {hdiff[:100].max():.2e})", flush=True)
    assert r.status == camg.OK and abs(r.iters - ko) <= 1
    assert r.true_relres < 1e-8 * 1.01
    if r.iters == ko:
        assert rel_on_samples(x) <= 1e-9
    assert hdiff[:100].max() <= 1e-9 and hdiff.max() <= 1e-6
    # parity mode: exactly the oracle's iteration count
    s.close()
    s = camg.Solver.from_device(A.n, rp, ci, va, max_iter=ko)
    dx.zero_()
    r = s.solve_dev(db, dx, rtol=0.0)
    e = rel_on_samples(dx.cpu().numpy())
    print(f"[gpu] FP64 at {ko} iterations: sampled rel diff {e:.2e}", flush=True)
    assert r.iters == ko and e <= 1e-9
    s.close()
    # mixed precision: FP32 V-cycle inside FP64 PCG, its error stated against the oracle
    s = camg.Solver.from_device(A.n, rp, ci, va, max_iter=5000, precision=camg.MIXED_FP32)
    dx.zero_()
    r = s.solve_dev(db, dx, rtol=1e-8)
    em = rel_on_samples(dx.cpu().numpy())
    print(f"[gpu] mixed natural stop: {r.iters} iterations, true_relres {r.true_relres:.3e}, "
          f"sampled rel error vs FP64 oracle {em:.2e}", flush=True)
    assert r.status == camg.OK and r.true_relres < 1e-8 and em <= 1e-6
    s.close()
