"""Write the oracle's natural-stop FP64 solves of full-size workloads to
text fixtures under tests/golden/.

Calls only the CPU oracle (oracle/) and the seeded problem generators
(paper_2102_07417_amd/problems.py); nothing here touches the GPU library.
The fixture of a workload holds the oracle's status, iteration count and
true relative residual, its residual history ||r_k|| (k = 0..iters), the
2-norm of x and x at 4096 evenly spaced unknowns (i_k = floor(k n / 4096)).
Floats are written with repr(), so they read back bit for bit.

The solve is PCG from x0 = 0 preconditioned by one V-cycle (Alg. "AMG
application in a V-cycle"), stopped at ||r|| < 1e-8 ||b|| on the recursive
residual (Section 4, set-up of the experiments), on the default hierarchy
(theta 0.25, PMIS seed 0, direct interpolation, one Jacobi step each way).

Usage:  python tests/golden/make_oracle_solves.py elasticity_64
(the 64^3-element elasticity solve takes tens of minutes on one core).
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2102_07417_amd import problems  # noqa: E402

SAMPLES = 4096
RTOL = 1e-8
MAX_ITER = 5000


def sample_index(n: int) -> np.ndarray:
    return (np.arange(SAMPLES, dtype=np.int64) * n) // SAMPLES


def fixture_path(name: str) -> str:
    return os.path.join(HERE, f"oracle_solve_{name}.txt")


def write(name: str) -> str:
    A = problems.workload(name)
    b = problems.rhs(A.n)
    t0 = time.perf_counter()
    h = oracle.Hierarchy(A, max_iter=MAX_ITER)
    t1 = time.perf_counter()
    r = h.solve(b, RTOL, max_iter=MAX_ITER)
    t2 = time.perf_counter()
    idx = sample_index(A.n)
    path = fixture_path(name)
    with open(path, "w") as f:
        f.write(f"# Oracle FP64 natural-stop PCG solve of workload {name} (n = {A.n}, nnz = {A.nnz}),\n")
        f.write("# b = problems.rhs(n) (seed 7417), rtol 1e-8, x0 = 0, default hierarchy.\n")
        f.write("# Written by tests/golden/make_oracle_solves.py (oracle and problem generators only).\n")
        f.write(f"# oracle set-up {t1 - t0:.1f} s, solve {t2 - t1:.1f} s on one core.\n")
        f.write(f"n {A.n}\nnnz {A.nnz}\nlevels {h.nlev}\nstatus {r.status}\niters {r.iters}\n")
        f.write(f"true_relres {r.true_relres!r}\nnorm_x {float(np.linalg.norm(r.x))!r}\n")
        f.write(f"samples {SAMPLES}\n")
        f.write("hist\n")
        for v in r.hist:
            f.write(f"{float(v)!r}\n")
        f.write("x\n")
        for i in idx:
            f.write(f"{int(i)} {float(r.x[i])!r}\n")
    return path


def read(name: str) -> dict:
    """Parse a fixture: scalars, hist (np.ndarray), idx and x samples."""
    out: dict = {}
    hist, idx, xs = [], [], []
    mode = None
    with open(fixture_path(name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            if t[0] in ("hist", "x") and len(t) == 1:
                mode = t[0]
                continue
            if mode == "hist":
                hist.append(float(t[0]))
            elif mode == "x":
                idx.append(int(t[0]))
                xs.append(float(t[1]))
            else:
                out[t[0]] = float(t[1]) if "." in t[1] or "e" in t[1] else int(t[1])
    out["hist"] = np.array(hist)
    out["idx"] = np.array(idx, dtype=np.int64)
    out["x"] = np.array(xs)
    return out


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["elasticity_64"]:
        print(write(nm), flush=True)
