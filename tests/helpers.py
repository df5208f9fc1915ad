"""Small helpers shared by the tests (no AMG arithmetic here)."""
import numpy as np


def csr_tuple(A):
    if hasattr(A, "row_ptr"):
        return A.n, A.n, A.row_ptr, A.col_idx, A.val
    return A


def dense(A):
    nr, nc, rp, ci, v = csr_tuple(A)
    d = np.zeros((nr, nc))
    rows = np.repeat(np.arange(nr), np.diff(rp))
    d[rows, ci] = v
    return d


def pattern(A):
    nr, nc, rp, ci, v = csr_tuple(A)
    d = np.zeros((nr, nc), dtype=bool)
    rows = np.repeat(np.arange(nr), np.diff(rp))
    d[rows, ci] = True
    return d


def from_dense(M, keep_zero_diag=True):
    """CSR tuple of a dense matrix (structural entries = nonzeros, plus the diagonal)."""
    M = np.asarray(M, dtype=np.float64)
    nr, nc = M.shape
    rp = [0]
    ci, v = [], []
    for i in range(nr):
        for j in range(nc):
            if M[i, j] != 0 or (keep_zero_diag and i == j and nr == nc):
                ci.append(j)
                v.append(M[i, j])
        rp.append(len(ci))
    return (nr, nc, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, np.float64))


def rows_sorted(A):
    nr, nc, rp, ci, v = csr_tuple(A)
    for i in range(nr):
        seg = ci[rp[i]:rp[i + 1]]
        if np.any(np.diff(seg) <= 0):
            return False
    return True


def wide_stencil_2d(g, r):
    """Graph Laplacian (+ identity) of a g x g grid where every point is
    coupled with weight -1 to all points within Chebyshev distance r: rows
    with up to (2r + 1)^2 entries, every coupling strong.  Used to give
    interpolation long candidate lists."""
    idx = np.arange(g * g).reshape(g, g)
    M = np.zeros((g * g, g * g))
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dx == 0 and dy == 0:
                continue
            ys, xs = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
            yy, xx = ys + dy, xs + dx
            ok = (yy >= 0) & (yy < g) & (xx >= 0) & (xx < g)
            M[idx[ys[ok], xs[ok]], idx[yy[ok], xx[ok]]] = -1.0
    M[np.arange(g * g), np.arange(g * g)] = -M.sum(1) + 1.0
    return from_dense(M)


def hub_graph(g):
    """A g x g 5-point grid plus one hub point coupled with weight -1 to
    every grid point (diagonals: coupling count + 0.1, so the matrix is
    strictly diagonally dominant).  Every grid point depends strongly on
    the hub, so PMIS makes the hub the only C point and the restriction has
    one row of g^2 entries.  Assembled sparse, in CSR order."""
    n = g * g + 1
    hub = g * g
    rows = [[] for _ in range(n)]
    for y in range(g):
        for x in range(g):
            i = y * g + x
            for yy, xx in ((y - 1, x), (y, x - 1), (y, x + 1), (y + 1, x)):
                if 0 <= yy < g and 0 <= xx < g:
                    rows[i].append((yy * g + xx, -1.0))
            rows[i].append((hub, -1.0))
            rows[hub].append((i, -1.0))
    rp = [0]
    ci, v = [], []
    for i in range(n):
        ent = rows[i] + [(i, len(rows[i]) + 0.1)]
        ent.sort()
        ci += [c for c, _ in ent]
        v += [a for _, a in ent]
        rp.append(len(ci))
    return (n, n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, np.float64))


# Tolerance of the FSAI factor G between the device and the oracle.  Both
# solve the local systems A(P_i, P_i) g = e_last through the same Cholesky
# factor but substitute in different orders (the oracle row by row, the
# device column by column), so entries differ by rounding only: at most
# about m u kappa for m local unknowns and a local condition number kappa
# (m <= 192 by construction, kappa <= 2e3 on the problems tested, i.e.
# <= 5e-11; 2.5e-16 measured on elasticity level 0).
FSAI_RTOL = 1e-10


def assert_fsai_close(gG, oG, tag=""):
    """Same pattern; each row of values within FSAI_RTOL of the row's largest
    entry (G tuples as exported: nr, nc, row_ptr, col_idx, val)."""
    assert np.array_equal(gG[2], oG[2]) and np.array_equal(gG[3], oG[3]), f"G{tag} pattern"
    rp, gv, ov = oG[2], np.asarray(gG[4]), np.asarray(oG[4])
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    scale = np.zeros(len(rp) - 1)
    np.maximum.at(scale, rows, np.abs(ov))
    err = np.abs(gv - ov) / np.maximum(scale[rows], np.finfo(float).tiny)
    assert err.size == 0 or err.max() <= FSAI_RTOL, f"G{tag} values: max row-relative diff {err.max():.3e}"
