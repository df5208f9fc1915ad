"""The allocation-free many-systems solve (camg_solve_batch_noalloc_dev,
for callers that cannot allocate device memory) against the allocating one
(camg_solve_batch_dev) through the C-ABI: both run the same kernel on the
same descriptors, so iterations, statuses, true residuals and solutions
must agree bit for bit.  Two allocation-free calls run back to back, the
second with fewer and smaller systems, so the second reuses the static
array the first filled."""
import numpy as np
import pytest

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


def _systems(camg, grids, seed0, precision):
    solvers, bs = [], []
    for k, g in enumerate(grids):
        A = PB.lognormal2d(g, 2.0, seed0 + k)
        solvers.append(camg.Solver(A, precision=precision, max_iter=2000))
        bs.append(torch.from_numpy(PB.rhs(A.n, seed0 + 100 + k)).to("cuda:0"))
    return solvers, bs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_batch_matches_allocating_batch(camg, precision):
    prec = camg.FP64 if precision == "fp64" else camg.MIXED_FP32
    calls = [_systems(camg, [40, 33, 50, 27, 45, 36, 31], 11, prec),  # 7 systems, n up to 2500
             _systems(camg, [24, 30], 71, prec)]                       # then 2 smaller ones
    outs = []
    for solvers, bs in calls:
        print(f"[gpu] no-alloc batch {precision}: {len(solvers)} systems", flush=True)
        xs = [torch.full_like(b, float("nan")) for b in bs]
        outs.append((camg.solve_batch_dev(solvers, bs, xs, no_alloc=True), xs))
    torch.cuda.synchronize()
    for (solvers, bs), ((it_n, rel_n, st_n), xs_n) in zip(calls, outs):
        xs_a = [torch.full_like(b, float("nan")) for b in bs]
        it_a, rel_a, st_a = camg.solve_batch_dev(solvers, bs, xs_a)
        torch.cuda.synchronize()
        assert np.array_equal(it_n, it_a) and np.array_equal(st_n, st_a)
        assert np.array_equal(rel_n, rel_a)
        assert (st_n == camg.OK).all() and (rel_n < 1e-8).all() and (it_n > 0).all()
        for xa, xn in zip(xs_a, xs_n):
            assert torch.equal(xa, xn)
        for s in solvers:
            s.close()


def test_noalloc_batch_rejects_too_many_systems(camg):
    A = PB.poisson2d(8)
    s = camg.Solver(A)
    b = torch.from_numpy(PB.rhs(A.n)).to("cuda:0")
    m = camg.NOALLOC_MAX_SYSTEMS + 1
    with pytest.raises(camg.CamgError) as e:
        camg.solve_batch_dev([s] * m, [b] * m, [torch.zeros_like(b)] * m, no_alloc=True)
    assert e.value.status == camg.E_ARG
    s.close()
