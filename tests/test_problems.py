"""Generators: exact sizes, symmetry, definiteness and the value recipes."""
import numpy as np
import pytest

from paper_2102_07417_amd import problems as PB
from tests.helpers import dense, rows_sorted


def _check(A):
    assert A.row_ptr.dtype == np.int32 and A.col_idx.dtype == np.int32 and A.val.dtype == np.float64
    assert A.row_ptr[0] == 0 and np.all(np.diff(A.row_ptr) >= 0)
    assert rows_sorted((A.n, A.n, A.row_ptr, A.col_idx, A.val))
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0.0


@pytest.mark.parametrize("name,n,nnz", [("poisson2d_64", 4096, 20224)])
def test_small_workload_sizes(name, n, nnz):
    A = PB.workload(name)
    _check(A)
    assert (A.n, A.nnz) == (n, nnz)


def test_stencil_nnz_formulas():
    # 7-point on m^3 with Dirichlet elimination: 7 m^3 - 6 m^2 entries
    for m in [3, 5, 8]:
        A = PB.lognormal3d(m)
        assert (A.n, A.nnz) == (m ** 3, 7 * m ** 3 - 6 * m ** 2)
        A = PB.aniso3d(m)
        assert (A.n, A.nnz) == (m ** 3, 7 * m ** 3 - 6 * m ** 2)
    for m in [3, 10]:
        A = PB.poisson2d(m)
        assert (A.n, A.nnz) == (m * m, 5 * m * m - 4 * m)


def test_elasticity_sizes_and_rows():
    ne = 4
    A = PB.elasticity3d(ne)
    _check(A)
    assert A.n == 3 * (ne + 1) ** 2 * ne
    lens = np.diff(A.row_ptr)
    assert lens.max() == 81 and lens.min() == 3 * 8  # interior 27 nodes, top corner 8 nodes
    ev = np.linalg.eigvalsh(dense(A))
    assert ev.min() > 0


def test_elasticity_rigid_modes_free():
    # the unit-E element stiffness annihilates the 6 rigid body modes
    K = PB.q1_stiffness_unitE(0.3, 0.5)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == 6
    assert np.allclose(K, K.T)


def test_lognormal_recipe():
    m = 4
    A = PB.lognormal3d(m, 2.0, seed=5)
    _check(A)
    g = np.random.Generator(np.random.Philox(key=5))
    kx = np.exp(2.0 * g.standard_normal((m, m, m + 1)))
    D = dense(A)
    # coupling of cell (0,0,0) and (0,0,1) is the first interior x-face
    assert D[0, 1] == -kx[0, 0, 1]
    assert np.all(np.diag(D) > 0)
    z, y, x = np.unravel_index(np.arange(m ** 3), (m, m, m))
    bnd = (np.minimum.reduce([x, y, z]) == 0) | (np.maximum.reduce([x, y, z]) == m - 1)
    rs = D.sum(1)
    assert np.all(rs[bnd] > 0)                                  # boundary faces only add to a_ii
    assert np.all(np.abs(rs[~bnd]) <= 1e-13 * np.diag(D)[~bnd])  # interior cells: zero row sum
    assert np.linalg.eigvalsh(D).min() > 0


def test_aniso_values():
    A = PB.aniso3d(3, 1e-3)
    D = dense(A)
    assert D[0, 0] == 4.002 and D[0, 1] == -1 and D[0, 3] == -1 and D[0, 9] == -1e-3


def test_rhs_reproducible():
    a = PB.rhs(100, 7)
    b = PB.rhs(100, 7)
    assert np.array_equal(a, b) and a.min() >= -1 and a.max() <= 1
    B = PB.rhs_block(100, 3, 7)
    assert np.array_equal(B[:, 0], a) and np.array_equal(B[:, 2], PB.rhs(100, 9))


def test_poisson3d_torch_matches_numpy():
    for shape in [(5, 5, 5), (7, 4, 3), (1, 6, 2)]:
        A = PB.poisson3d(*shape)
        n, rp, ci, v = PB.poisson3d_torch(*shape)
        assert n == A.n
        assert np.array_equal(rp.numpy(), A.row_ptr) and np.array_equal(ci.numpy(), A.col_idx)
        assert np.array_equal(v.numpy(), A.val)


def test_elasticity_rigid_modes_in_kernel_away_from_clamp():
    # K annihilates the rigid body modes on every row whose node is not
    # coupled to the clamped z = 0 layer (z >= 2h)
    ne = 3
    A = PB.elasticity3d(ne)
    V = PB.elasticity_rigid_modes(ne)
    assert V.shape == (A.n, 6)
    KV = A.to_scipy() @ V
    nodes_per_layer = (ne + 1) ** 2
    far = np.arange(A.n) // 3 >= nodes_per_layer   # nodes with z >= 2h
    assert np.abs(KV[far]).max() < 1e-10 * np.abs(A.val).max()
    assert np.abs(KV[~far]).max() > 1e-6


def test_oracle_solve_fixture_is_a_natural_stop():
    """The stored oracle solve of the 64^3-element elasticity workload reads
    back consistently: its history has iters + 1 entries, starts at ||b||,
    and stops at the first residual below 1e-8 ||b|| (strict), as the
    stopping rule of the experiments prescribes."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_oracle_solves as G
    g = G.read("elasticity_64")
    h = g["hist"]
    assert g["status"] == 0 and len(h) == g["iters"] + 1 and g["n"] == 811200 and g["nnz"] == 63695790
    assert h[-1] < 1e-8 * h[0] and np.all(h[:-1] >= 1e-8 * h[0])
    assert abs(h[0] - np.linalg.norm(PB.rhs(g["n"]))) <= 1e-12 * h[0]
    assert len(g["idx"]) == g["samples"] == 4096 and np.array_equal(g["idx"], G.sample_index(g["n"]))
    assert g["true_relres"] < 1e-8 and np.all(np.isfinite(g["x"]))


def test_powerlaw_graph_ragged_spd():
    A = PB.powerlaw_graph(600, seed=3)
    _check(A)
    lens = np.diff(A.row_ptr)
    assert lens.min() <= 8 and lens.max() >= 100  # ragged: a few to hundreds per row
    D = dense(A)
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 0)
    np.testing.assert_allclose(np.diag(D) + off.sum(1), 1e-2, rtol=0, atol=1e-12)  # zero row sums + shift
    assert np.linalg.eigvalsh(D).min() > 0
    B = PB.powerlaw_graph(600, seed=3)
    assert np.array_equal(A.val, B.val) and np.array_equal(A.col_idx, B.col_idx)
