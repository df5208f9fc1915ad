"""Seeded synthetic SPD test problems in CSR form.

This module builds the matrices and right-hand sides that both the GPU path
and the CPU oracle consume.  It holds no part of the AMG method itself: only
finite-difference / finite-volume / finite-element assembly and random draws.

Every matrix is returned as ``CSR(n, row_ptr, col_idx, val)`` with int32
indices, float64 values, 0-based, columns strictly ascending in each row,
full (both-triangle) storage and Dirichlet boundary unknowns eliminated.

The shapes follow the classes of problems the paper evaluates on (Section 4,
Table of test matrices): 5- and 7-point Poisson stencils, heterogeneous
diffusion, anisotropic diffusion and 3D linear elasticity with ~81 nonzeros
per row.  The paper's own matrices are not available, so these synthetic
problems stand in for them.

Random streams: ``numpy.random.Generator(numpy.random.Philox(key=seed))``,
drawn in the order documented on each generator.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_A = 2021
SEED_B = 7417


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col_idx] = self.val
        return d

    def nbytes(self, val_bytes: int = 8) -> int:
        return 4 * (self.n + 1) + (4 + val_bytes) * self.nnz


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=seed))


def _stencil_csr(shape, offsets, diag, offvals) -> CSR:
    """Assemble a structured-grid stencil matrix.

    ``shape`` is the grid (slowest axis first, x fastest), ``offsets`` a list
    of neighbour offsets (same axis order) sorted so that the flattened column
    index increases, ``diag`` the diagonal (array of grid shape) and
    ``offvals[k]`` the coupling to neighbour ``offsets[k]`` (grid-shaped
    array, ignored where the neighbour lies outside the grid: Dirichlet
    elimination).
    """
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64).reshape(shape)
    cols, vals, masks = [], [], []
    diag_pos = None
    all_off = list(offsets)
    # insert the diagonal at its sorted position
    flat_off = [int(np.ravel_multi_index(tuple(np.array(o) + 1), (3,) * len(shape))) for o in all_off]
    order = sorted(range(len(all_off)), key=lambda k: flat_off[k])
    assert order == list(range(len(all_off))), "offsets must be in ascending column order"
    centre = int(np.ravel_multi_index((1,) * len(shape), (3,) * len(shape)))
    diag_pos = sum(1 for f in flat_off if f < centre)
    entries = []
    for k, off in enumerate(all_off):
        if k == diag_pos:
            entries.append(("d", None))
        entries.append(("o", k))
    if diag_pos == len(all_off):
        entries.append(("d", None))
    for kind, k in entries:
        if kind == "d":
            cols.append(idx.reshape(-1))
            vals.append(np.asarray(diag, dtype=np.float64).reshape(-1))
            masks.append(np.ones(n, dtype=bool))
            continue
        off = all_off[k]
        m = np.ones(shape, dtype=bool)
        src = [slice(None)] * len(shape)
        for ax, o in enumerate(off):
            if o > 0:
                sl = [slice(None)] * len(shape)
                sl[ax] = slice(shape[ax] - o, None)
                m[tuple(sl)] = False
            elif o < 0:
                sl = [slice(None)] * len(shape)
                sl[ax] = slice(0, -o)
                m[tuple(sl)] = False
        shift = int(np.sum(np.array(off) * np.array([int(np.prod(shape[a + 1:])) for a in range(len(shape))])))
        cols.append((idx + shift).reshape(-1))
        vals.append(np.asarray(offvals[k], dtype=np.float64).reshape(-1))
        masks.append(m.reshape(-1))
    C = np.stack(cols, axis=1)
    V = np.stack(vals, axis=1)
    M = np.stack(masks, axis=1)
    counts = M.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = C[M].astype(np.int32)
    val = V[M].astype(np.float64)
    return CSR(n, row_ptr.astype(np.int32), col_idx, val)


_OFF2 = [(-1, 0), (0, -1), (0, 1), (1, 0)]
_OFF3 = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0), (1, 0, 0)]


def poisson2d(nx: int, ny: int | None = None) -> CSR:
    """5-point Laplacian on an nx-by-ny interior grid: diagonal 4, neighbours -1."""
    ny = nx if ny is None else ny
    shape = (ny, nx)
    one = np.ones(shape)
    return _stencil_csr(shape, _OFF2, 4.0 * one, [-one] * 4)


def poisson3d(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """7-point Laplacian on an nx-by-ny-by-nz interior grid: diagonal 6, neighbours -1."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    shape = (nz, ny, nx)
    one = np.ones(shape)
    return _stencil_csr(shape, _OFF3, 6.0 * one, [-one] * 6)


def poisson3d_torch(nx: int, ny: int | None = None, nz: int | None = None, device="cpu"):
    """The matrix of ``poisson3d`` assembled with torch on ``device`` (for
    grids whose host assembly would be slow, e.g. 404^3 with 4.6e8
    nonzeros).  Returns (n, row_ptr int32, col_idx int32, val float64)
    tensors equal to ``poisson3d``'s arrays."""
    import torch

    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    i = torch.arange(n, dtype=torch.int64, device=device)
    x = i % nx
    y = (i // nx) % ny
    z = i // (nx * ny)
    one = torch.ones_like(i, dtype=torch.bool)
    # neighbours in ascending column order: z-1, y-1, x-1, self, x+1, y+1, z+1
    offs = [-nx * ny, -nx, -1, 0, 1, nx, nx * ny]
    masks = [z > 0, y > 0, x > 0, one, x < nx - 1, y < ny - 1, z < nz - 1]
    cnt = torch.zeros(n, dtype=torch.int32, device=device)
    for m in masks:
        cnt += m.to(torch.int32)
    del x, y, z
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(cnt, 0, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col_idx = torch.empty(nnz, dtype=torch.int32, device=device)
    val = torch.empty(nnz, dtype=torch.float64, device=device)
    pos = row_ptr[:-1].clone()
    for o, m in zip(offs, masks):
        rows = torch.nonzero(m).squeeze(1) if o != 0 else i
        p = pos[rows]
        col_idx[p] = (rows + o).to(torch.int32)
        val[p] = 6.0 if o == 0 else -1.0
        pos[rows] += 1
        del rows, p
    return n, row_ptr.to(torch.int32), col_idx, val


def aniso3d(n: int, eps: float = 1e-3) -> CSR:
    """7-point anisotropic diffusion on n^3: x/y couplings -1, z couplings -eps,
    diagonal 4 + 2 eps (Dirichlet eliminated)."""
    shape = (n, n, n)
    one = np.ones(shape)
    offv = [-eps * one, -one, -one, -one, -one, -eps * one]  # order of _OFF3: -z,-y,-x,+x,+y,+z
    return _stencil_csr(shape, _OFF3, (4.0 + 2.0 * eps) * one, offv)


def lognormal3d(n: int, sigma: float = 2.0, seed: int = SEED_A) -> CSR:
    """Cell-centred finite-volume diffusion on an n^3 grid of unit cells.

    Every face f (interior and boundary) carries kappa_f = exp(sigma * N(0,1)).
    Draw order: all x-faces, then y-faces, then z-faces, each in lexicographic
    order with x fastest (x-faces have shape (n, n, n+1) as [z, y, x_face]).
    a_ij = -kappa_f for the face between cells i and j; a_ii is the sum of the
    six face coefficients of cell i (a boundary face acts as a Dirichlet ghost
    and only adds to the diagonal).
    """
    g = _rng(seed)
    kx = np.exp(sigma * g.standard_normal((n, n, n + 1)))
    ky = np.exp(sigma * g.standard_normal((n, n + 1, n)))
    kz = np.exp(sigma * g.standard_normal((n + 1, n, n)))
    diag = (kx[:, :, :-1] + kx[:, :, 1:]) + (ky[:, :-1, :] + ky[:, 1:, :]) + (kz[:-1] + kz[1:])
    offv = [
        -kz[:-1],          # -z neighbour: face below
        -ky[:, :-1, :],    # -y
        -kx[:, :, :-1],    # -x
        -kx[:, :, 1:],     # +x
        -ky[:, 1:, :],     # +y
        -kz[1:],           # +z
    ]
    return _stencil_csr((n, n, n), _OFF3, diag, offv)


def lognormal2d(n: int, sigma: float = 2.0, seed: int = SEED_A) -> CSR:
    """2D analogue of :func:`lognormal3d` on an n^2 grid (x-faces then y-faces)."""
    g = _rng(seed)
    kx = np.exp(sigma * g.standard_normal((n, n + 1)))
    ky = np.exp(sigma * g.standard_normal((n + 1, n)))
    diag = (kx[:, :-1] + kx[:, 1:]) + (ky[:-1] + ky[1:])
    offv = [-ky[:-1], -kx[:, :-1], -kx[:, 1:], -ky[1:]]
    return _stencil_csr((n, n), _OFF2, diag, offv)


# ---------------------------------------------------------------------------
# Ragged rows: a graph Laplacian with power-law degrees
# ---------------------------------------------------------------------------

def powerlaw_graph(n: int, seed: int = SEED_A, max_degree: int = 200, shift: float = 1e-2) -> CSR:
    """Weighted graph Laplacian plus ``shift`` on the diagonal, on n nodes
    whose out-degrees follow a power law, so rows range from a couple of
    entries to a few hundred in one matrix (an M-matrix, diagonally dominant,
    SPD).  Draws, in order: u ~ U[0, 1) per node, target degree
    d_i = min(max_degree, floor(2 / (u_i + 1e-9)^0.9)); the sum(d) targets of
    the edges, integers in [0, n), node by node; after dropping self loops
    and merging each undirected pair {i, j} into one edge (listed by
    ascending (min, max)), one weight U[0.1, 1) per edge."""
    g = _rng(seed)
    u = g.random(n)
    d = np.minimum(max_degree, np.floor(2.0 / (u + 1e-9) ** 0.9)).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), d)
    dst = g.integers(0, n, size=int(d.sum()), dtype=np.int64)
    keep = src != dst
    lo, hi = np.minimum(src[keep], dst[keep]), np.maximum(src[keep], dst[keep])
    key = np.unique(lo * n + hi)
    lo, hi = key // n, key % n
    w = 0.1 + 0.9 * g.random(key.size)
    deg = np.bincount(lo, weights=w, minlength=n) + np.bincount(hi, weights=w, minlength=n)
    rows = np.concatenate([lo, hi, np.arange(n)])
    cols = np.concatenate([hi, lo, np.arange(n)])
    vals = np.concatenate([-w, -w, deg + shift])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return CSR(n, rp.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


# ---------------------------------------------------------------------------
# 3D linear elasticity, trilinear (Q1) hexahedra
# ---------------------------------------------------------------------------

def q1_stiffness_unitE(nu: float, h: float) -> np.ndarray:
    """24x24 stiffness of a cube element of side h with E = 1, Poisson ratio nu,
    2x2x2 Gauss quadrature.  Local nodes are ordered lexicographically
    (x fastest, then y, then z); dofs are interleaved (u_x, u_y, u_z) per node."""
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    corners = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=float)
    sgn = 2 * corners - 1  # reference coordinates in {-1, 1}
    gp = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    K = np.zeros((24, 24))
    for gz in gp:
        for gy in gp:
            for gx in gp:
                xi = np.array([gx, gy, gz])
                # dN/dxi for each node: (1/8) * s_d * prod_{e != d} (1 + s_e xi_e)
                dN = np.zeros((8, 3))
                for d in range(3):
                    f = np.ones(8)
                    for e in range(3):
                        if e != d:
                            f *= 1 + sgn[:, e] * xi[e]
                    dN[:, d] = 0.125 * sgn[:, d] * f
                dNdx = dN * (2.0 / h)  # Jacobian of the map is (h/2) I
                B = np.zeros((6, 24))
                for a in range(8):
                    bx, by, bz = dNdx[a]
                    c = 3 * a
                    B[0, c] = bx
                    B[1, c + 1] = by
                    B[2, c + 2] = bz
                    B[3, c] = by; B[3, c + 1] = bx
                    B[4, c + 1] = bz; B[4, c + 2] = by
                    B[5, c] = bz; B[5, c + 2] = bx
                K += B.T @ D @ B * (h / 2.0) ** 3
    return 0.5 * (K + K.T)


def elasticity3d(ne: int, nu: float = 0.3, seed: int = SEED_A) -> CSR:
    """Q1 linear elasticity on the unit cube meshed by ne^3 cube elements.

    E_e = exp(N(0,1)) per element, drawn in element-lexicographic order
    (x fastest).  K = sum_e E_e K_ref(nu, h) with h = 1/ne.  Dofs are
    interleaved per node; nodes are numbered lexicographically (x fastest);
    the nodes on z = 0 are clamped and removed.  Every pair of nodes that
    shares an element keeps its full 3x3 block in the pattern (81 entries in
    an interior row).  The result is made exactly symmetric by averaging each
    block with the transpose of its mirror block.
    """
    h = 1.0 / ne
    E = np.exp(_rng(seed).standard_normal((ne, ne, ne)))  # [ez, ey, ex]
    Kr = q1_stiffness_unitE(nu, h)
    nn = ne + 1
    # blocks[z, y, x, o, 3, 3]: coupling of node (z,y,x) with node + offset o
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    oid = {o: k for k, o in enumerate(offs)}
    blocks = np.zeros((nn, nn, nn, 27, 3, 3))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
            o = oid[(bz - az, by - ay, bx - ax)]
            kab = Kr[3 * a:3 * a + 3, 3 * b:3 * b + 3]
            blocks[az:az + ne, ay:ay + ne, ax:ax + ne, o] += E[..., None, None] * kab
    # exact symmetrisation: B(i, o) <- (B(i, o) + B(i+o, -o)^T) / 2
    sym = np.empty_like(blocks)
    for k, (dz, dy, dx) in enumerate(offs):
        mk = oid[(-dz, -dy, -dx)]
        src = np.zeros((nn, nn, nn, 3, 3))
        zs = slice(max(dz, 0), nn + min(dz, 0)); zd = slice(max(-dz, 0), nn + min(-dz, 0))
        ys = slice(max(dy, 0), nn + min(dy, 0)); yd = slice(max(-dy, 0), nn + min(-dy, 0))
        xs = slice(max(dx, 0), nn + min(dx, 0)); xd = slice(max(-dx, 0), nn + min(-dx, 0))
        src[zd, yd, xd] = np.swapaxes(blocks[zs, ys, xs, mk], -1, -2)
        sym[..., k, :, :] = 0.5 * (blocks[..., k, :, :] + src)
    del blocks
    # drop the clamped z = 0 node layer
    sym = sym[1:]
    nz_nodes = nn - 1
    shape = (nz_nodes, nn, nn)
    nnodes = int(np.prod(shape))
    node = np.arange(nnodes, dtype=np.int64).reshape(shape)
    valid = np.zeros(shape + (27,), dtype=bool)
    nbr = np.zeros(shape + (27,), dtype=np.int64)
    for k, (dz, dy, dx) in enumerate(offs):
        zz = np.arange(nz_nodes)[:, None, None] + dz
        yy = np.arange(nn)[None, :, None] + dy
        xx = np.arange(nn)[None, None, :] + dx
        ok = (zz >= 0) & (zz < nz_nodes) & (yy >= 0) & (yy < nn) & (xx >= 0) & (xx < nn)
        valid[..., k] = ok
        nbr[..., k] = node + dz * nn * nn + dy * nn + dx
    valid = valid.reshape(nnodes, 27)
    nbr = nbr.reshape(nnodes, 27)
    sym = sym.reshape(nnodes, 27, 3, 3)
    # row (node, comp c): columns (nbr k, comp d) for valid k, ascending (k order is ascending)
    cnt_node = valid.sum(axis=1) * 3
    n = nnodes * 3
    row_cnt = np.repeat(cnt_node, 3)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(row_cnt, out=row_ptr[1:])
    # columns: for each node row, [3*nbr_k + d for k valid for d in 0..2]
    colk = (3 * nbr[:, :, None] + np.arange(3)[None, None, :])  # [node, 27, 3]
    vmask = np.repeat(valid[:, :, None], 3, axis=2)              # [node, 27, 3]
    col_idx = np.empty(int(row_ptr[-1]), dtype=np.int32)
    val = np.empty(int(row_ptr[-1]), dtype=np.float64)
    for c in range(3):
        rows = np.arange(nnodes) * 3 + c
        cols_c = colk[vmask].reshape(-1)  # identical column list for the 3 rows of a node
        vals_c = sym[:, :, c, :][vmask].reshape(-1)
        # scatter: row r = 3*node + c begins at row_ptr[r]
        starts = row_ptr[rows]
        lens = cnt_node
        pos = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens) + np.arange(lens.sum())
        col_idx[pos] = cols_c
        val[pos] = vals_c
    return CSR(n, row_ptr.astype(np.int32), col_idx, val)


def elasticity_rigid_modes(ne: int) -> np.ndarray:
    """The six rigid body modes of ``elasticity3d(ne)`` at its free dofs
    (n x 6, row-major): translations along x, y, z, then rotations about z
    (-y, x, 0), x (0, -z, y) and y (z, 0, -x), from the nodal coordinates
    (node (ix, iy, iz) at (ix, iy, iz) / ne, iz = 1..ne; dofs interleaved)."""
    nn = ne + 1
    iz, iy, ix = np.meshgrid(np.arange(1, nn), np.arange(nn), np.arange(nn), indexing="ij")
    x, y, z = (ix.ravel() / ne, iy.ravel() / ne, iz.ravel() / ne)
    m = x.size
    V = np.zeros((m, 3, 6))
    V[:, 0, 0] = 1.0
    V[:, 1, 1] = 1.0
    V[:, 2, 2] = 1.0
    V[:, 0, 3], V[:, 1, 3] = -y, x
    V[:, 1, 4], V[:, 2, 4] = -z, y
    V[:, 0, 5], V[:, 2, 5] = z, -x
    return V.reshape(3 * m, 6)


def rhs(n: int, seed: int = SEED_B) -> np.ndarray:
    """b ~ U[-1, 1] per entry, Philox(key=seed)."""
    return _rng(seed).uniform(-1.0, 1.0, n)


def rhs_block(n: int, k: int, seed: int = SEED_B) -> np.ndarray:
    """n-by-k row-major block; column j is ``rhs(n, seed + j)``."""
    B = np.empty((n, k))
    for j in range(k):
        B[:, j] = rhs(n, seed + j)
    return B


# Named workloads (sizes from the generator definitions above)
def workload(name: str) -> CSR:
    if name == "poisson2d_64":
        return poisson2d(64)
    if name == "lognormal3d_128":
        return lognormal3d(128, 2.0, SEED_A)
    if name == "elasticity_64":
        return elasticity3d(64, 0.3, SEED_A)
    if name == "aniso3d_160":
        return aniso3d(160, 1e-3)
    raise KeyError(name)


# The resident systems of the serving workload.
SERVING_SYSTEMS = [
    ("poisson2d_100", lambda: poisson2d(100)),
    ("poisson2d_316", lambda: poisson2d(316)),
    ("poisson3d_48", lambda: poisson3d(48)),
    ("lognormal3d_64", lambda: lognormal3d(64, 2.0, SEED_A)),
    ("poisson3d_100", lambda: poisson3d(100)),
    ("lognormal2d_1000", lambda: lognormal2d(1000, 2.0, SEED_A)),
    ("lognormal3d_128", lambda: lognormal3d(128, 2.0, SEED_A)),
    ("poisson3d_158", lambda: poisson3d(158)),
]
