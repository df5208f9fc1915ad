"""The block-of-right-hand-sides workload at full size (7-point anisotropic
diffusion on 160^3, eps = 1e-3, n = 4,096,000, 32 right-hand sides) on the
GPU against the CPU oracle, in the configurations the benchmark times: the
hierarchy bit for bit, the FP64 block solve and the autotuned mixed block
solve on every column to a true residual below 1e-8, and two columns
(the first and the last) against the oracle's own FP64 solves."""
import numpy as np
import pytest

import oracle as O
from paper_2102_07417_amd import problems as PB

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K = 32
CHECK = (0, K - 1)


@pytest.fixture(scope="module")
def camg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_07417_amd import camg as C
    C.load()
    return C


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.timeout(600)
def test_block_solves_at_full_size(camg):
    print("[gpu] full-size aniso3d_160, 32 right-hand sides", flush=True)
    A = PB.workload("aniso3d_160")
    B = PB.rhs_block(A.n, K)
    o = O.Hierarchy(A, max_iter=5000)
    rp, ci, va = _dev(A.row_ptr), _dev(A.col_idx), _dev(A.val)
    g = camg.Solver.from_device(A.n, rp, ci, va, max_iter=5000)
    assert g.nlev == o.nlev
    for l in range(o.nlev):
        ga, oa = g.A(l), o.A(l)
        assert np.array_equal(ga[3], oa[3]) and np.array_equal(ga[4], oa[4]), l
    ref = {j: o.solve(np.ascontiguousarray(B[:, j]), 1e-8, max_iter=5000) for j in CHECK}
    dB = _dev(B)
    # FP64 block solve
    dX = torch.zeros_like(dB)
    r = g.solve_multi_dev(dB, dX, rtol=1e-8)
    assert r.status == camg.OK and float(r.true_relres.max()) < 1e-8 * 1.01
    for j in CHECK:
        x = dX[:, j].cpu().numpy()
        assert abs(int(r.iters[j]) - ref[j].iters) <= 1, (j, int(r.iters[j]), ref[j].iters)
        assert np.linalg.norm(x - ref[j].x) / np.linalg.norm(ref[j].x) <= 1e-9
    g.close()
    # mixed block solve with autotuned row schedules
    gm = camg.Solver.from_device(A.n, rp, ci, va, max_iter=5000, precision=camg.MIXED_FP32)
    gm.set_option(camg.OPT_AUTOTUNE, 1)
    dX.zero_()
    rm = gm.solve_multi_dev(dB, dX, rtol=1e-8)
    assert rm.status == camg.OK and float(rm.true_relres.max()) < 1e-8 * 1.01
    for j in CHECK:
        x = dX[:, j].cpu().numpy()
        err = np.linalg.norm(x - ref[j].x) / np.linalg.norm(ref[j].x)
        print(f"[gpu] mixed block column {j}: {int(rm.iters[j])} iterations (oracle {ref[j].iters}), "
              f"relative difference {err:.2e}", flush=True)
        assert err <= 1e-10  # measured 1.8e-14
    gm.close()
