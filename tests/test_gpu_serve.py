"""Serving: resident hierarchies, continuous batching, admission by memory
(GPU).  Each request's solutions are checked against the CPU oracle, and a
request's result must be bitwise the same served alone and in a mix."""
import time

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


SYSTEMS = [("poisson2d_40", lambda: PB.poisson2d(40), "fp64"),
           ("lognormal3d_14", lambda: PB.lognormal3d(14, 2.0), "mixed"),
           ("elasticity_6", lambda: PB.elasticity3d(6, 0.3), "fp64")]


def _drain(srv, n, out=None, timeout=60.0):
    out = {} if out is None else out
    t0 = time.time()
    while len(out) < n:
        for c in srv.poll():
            out[c["tag"]] = c
        assert time.time() - t0 < timeout, "server did not finish"
    return out


def _requests(systems, count, seed=5):
    rng = np.random.default_rng(seed)
    reqs = []
    for t in range(count):
        s = int(rng.integers(len(systems)))
        k = int(rng.integers(1, 7))
        n = systems[s][1].n
        reqs.append((t, s, PB.rhs_block(n, k, 1000 + 17 * t)))
    return reqs


def _server(camg, systems, budget=1 << 31, slots=8):
    srv = camg.Server(budget)
    for name, A, prec in systems:
        s = camg.Solver(A, precision=camg.MIXED_FP32 if prec == "mixed" else camg.FP64)
        srv.add(s, slots)
    return srv


def test_server_results_match_oracle_and_alone(camg):
    systems = [(name, f(), prec) for name, f, prec in SYSTEMS]
    reqs = _requests(systems, 24)
    srv = _server(camg, systems)
    outs = {}
    done = {}
    for t, s, B in reqs:
        X = torch.zeros(B.shape, dtype=torch.float64).pin_memory()
        outs[t] = X
        srv.submit(s, torch.from_numpy(B).pin_memory(), X, rtol=1e-8, max_iter=500, tag=t)
        for c in srv.poll():  # arrivals interleave with running work
            done[c["tag"]] = c
    _drain(srv, len(reqs), done)
    st = srv.stats()
    assert st["queued"] == 0 and st["busy_slots"] == 0 and st["arena_used"] == 0
    srv.close()
    orcs = {i: O.Hierarchy(A) for i, (_, A, _) in enumerate(systems)}
    for t, s, B in reqs:
        c = done[t]
        assert c["status"] == camg.OK and c["true_relres"] < 1e-8
        X = outs[t].numpy()
        tol = 1e-6 if systems[s][2] == "mixed" else 1e-9
        for j in (0, B.shape[1] - 1):
            ro = orcs[s].solve(B[:, j], 1e-8)
            assert np.linalg.norm(X[:, j] - ro.x) / np.linalg.norm(ro.x) <= tol
    # the same requests alone, one per fresh server: bitwise equal
    for t, s, B in reqs[:6]:
        srv1 = _server(camg, systems)
        X1 = torch.zeros(B.shape, dtype=torch.float64).pin_memory()
        srv1.submit(s, torch.from_numpy(B).pin_memory(), X1, rtol=1e-8, max_iter=500, tag=0)
        _drain(srv1, 1)
        srv1.close()
        assert torch.equal(X1, outs[t]), f"request {t} differs alone vs in the mix"


def test_server_device_buffers_and_tight_budget(camg):
    """Device-resident buffers; a budget whose arena holds one request at a
    time forces admission waits; every request still completes."""
    systems = [(name, f(), prec) for name, f, prec in SYSTEMS[:2]]
    probe = camg.Server(1 << 40)
    sv = [camg.Solver(A) for _, A, _ in systems]
    fp = sum(camg.camg_engine_footprint(s.h, 8) for s in sv)
    probe.close()
    nmax = max(A.n for _, A, _ in systems)
    srv = camg.Server(fp + 16384 + 6 * nmax * 8 + 256)
    for s in sv:
        srv.add(s, 8)
    reqs = _requests(systems, 10, seed=9)
    outs = {}
    for t, s, B in reqs:
        dB = torch.from_numpy(B).to("cuda:0")
        outs[t] = torch.zeros_like(dB)
        srv.submit(s, dB, outs[t], rtol=1e-8, max_iter=500, tag=t)
    assert srv.stats()["queued"] == len(reqs)
    done = {c["tag"]: c for c in srv.poll()}
    st = srv.stats()
    assert st["queued"] > 0 and st["arena_used"] <= st["arena_size"]
    _drain(srv, len(reqs), done)
    for t, s, B in reqs:
        A = systems[s][1]
        X = outs[t].cpu().numpy()
        R = B - (A.to_scipy() @ X)
        assert np.all(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0) < 1e-8)
    srv.close()


def test_server_errors(camg):
    A = PB.poisson2d(20)
    s = camg.Solver(A)
    srv = camg.Server(1 << 30)
    sid = srv.add(s, 4)
    with pytest.raises(camg.CamgError):
        srv.add(s, 3)  # not a power of two
    B = np.zeros((A.n, 5))
    with pytest.raises(camg.CamgError):
        srv.submit(sid, B, np.zeros_like(B), tag=1)  # more columns than slots
    with pytest.raises(camg.CamgError):
        srv.submit(7, B[:, :2].copy(), np.zeros((A.n, 2)), tag=2)  # unknown system
    small = camg.Server(1000)
    with pytest.raises(camg.CamgError):
        small.add(s, 4)  # engine does not fit the budget
    small.close()
    # a zero right-hand side finishes at once with x = 0
    B0 = np.zeros((A.n, 2))
    X0 = np.full((A.n, 2), 3.0)
    srv.submit(sid, B0, X0, tag=3)
    d = _drain(srv, 1)
    assert d[3]["status"] == camg.OK and d[3]["iters"] == 0 and np.all(X0 == 0.0)
    srv.close()
