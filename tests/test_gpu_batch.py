"""Many small systems in one launch (one workgroup per system), GPU: every
system against the CPU oracle and against the single-system path."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2102_07417_amd import problems as PB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def camg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_07417_amd import camg
    camg.load()
    return camg


def _systems():
    out = [PB.poisson2d(n) for n in (3, 10, 17, 40, 64)]
    out += [PB.poisson2d(37, 23), PB.lognormal3d(8, 2.0, 5), PB.lognormal3d(14, 2.0, 6), PB.aniso3d(12, 1e-3)]
    out += [PB.lognormal2d(60, 2.0, 7), PB.elasticity3d(6, 0.3)]
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_matches_oracle_and_single_path(camg, prec):
    print(f"[gpu] batch {prec}", flush=True)
    systems = _systems()
    p = camg.MIXED_FP32 if prec == "mixed" else camg.FP64
    solvers = [camg.Solver(A, precision=p) for A in systems]
    bs = [PB.rhs(A.n, 100 + k) for k, A in enumerate(systems)]
    db = [torch.from_numpy(b).to("cuda:0") for b in bs]
    dx = [torch.full_like(d, 5.0) for d in db]
    it, rel, st = camg.solve_batch_dev(solvers, db, dx, rtol=1e-8)
    assert np.all(st == camg.OK), st
    assert np.all(rel < 1e-8), rel
    for k, A in enumerate(systems):
        x = dx[k].cpu().numpy()
        ro = O.Hierarchy(A).solve(bs[k], 1e-8)
        if prec == "fp64":
            assert abs(int(it[k]) - ro.iters) <= 1, (k, it[k], ro.iters)
            assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) <= 1e-9, k
            rs = solvers[k].solve(bs[k])
            assert abs(int(it[k]) - rs.iters) <= 1
        else:
            assert int(it[k]) <= ro.iters + 5
            assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) <= 1e-6, k
    # deterministic: a second launch with the systems in another order gives the same bits
    perm = list(reversed(range(len(systems))))
    dx2 = [torch.zeros_like(d) for d in db]
    it2, rel2, st2 = camg.solve_batch_dev([solvers[k] for k in perm], [db[k] for k in perm],
                                          [dx2[k] for k in perm], rtol=1e-8)
    for k in range(len(systems)):
        assert torch.equal(dx[k], dx2[k])
    for s in solvers:
        s.close()


def test_batch_edge_cases(camg):
    A = PB.poisson2d(20)
    s1, s2 = camg.Solver(A), camg.Solver(A, max_iter=3)
    b = torch.from_numpy(PB.rhs(A.n)).to("cuda:0")
    z = torch.zeros_like(b)
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    it, rel, st = camg.solve_batch_dev([s1, s2], [z, b], [x1, x2], rtol=1e-8)
    assert st[0] == camg.OK and it[0] == 0 and torch.all(x1 == 0)
    assert st[1] == camg.E_MAXIT and it[1] == 3
    with pytest.raises(camg.CamgError):  # the same handle twice
        camg.solve_batch_dev([s1, s1], [b, b], [x1, x2])
    sm = camg.Solver(A, precision=camg.MIXED_FP32)
    with pytest.raises(camg.CamgError):  # mixed precisions in one batch
        camg.solve_batch_dev([s1, sm], [b, b], [x1, x2])
    s3 = camg.Solver(A, nu_pre=2)
    with pytest.raises(camg.CamgError):
        camg.solve_batch_dev([s3], [b], [x1])
    for s in (s1, s2, sm, s3):
        s.close()
