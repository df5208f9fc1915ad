"""Python view of the CPU FP64 oracle (oracle/orc.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the GPU
library and never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# CAMG_ORACLE_LIB lets the mutation tests load a deliberately broken build
_LIBPATH = os.environ.get("CAMG_ORACLE_LIB") or os.path.join(HERE, "liborc.so")
_lib = None

OK, MAXIT, E_ARG, E_CSR, E_NOT_SPD, E_BREAKDOWN, E_COARSE, E_NOMEM = 0, 1, -1, -2, -3, -4, -5, -6
F, U, CPT = -1, 0, 1
X_A, X_P, X_R, X_CF, X_STRONG, X_DINV, X_OMEGA, X_CHOL, X_STCNT, X_ROUNDS, X_G = range(11)
SMOOTH_JACOBI, SMOOTH_FSAI, SMOOTH_FSAI_JACOBI, SMOOTH_AFSAI = 0, 1, 2, 3
AFSAI_MAXM, AFSAI_MAXCAND = 32, 2048
INTERP_DIRECT, INTERP_CLASSICAL, INTERP_EXTI, INTERP_HYBRID, INTERP_BAMG = 0, 1, 2, 3, 4


class Params(C.Structure):
    _fields_ = [("theta", C.c_double), ("seed", C.c_uint64), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("omega", C.c_double), ("max_levels", C.c_int32),
                ("max_coarse", C.c_int32), ("max_iter", C.c_int32), ("smoother", C.c_int32),
                ("interp", C.c_int32), ("bamg_lmin", C.c_int32), ("bamg_lmax", C.c_int32),
                ("bamg_eps", C.c_double), ("bamg_mu", C.c_double), ("psmooth", C.c_int32),
                ("pfilter", C.c_double), ("srqm_iters", C.c_int32), ("afsai_steps", C.c_int32),
                ("afsai_step", C.c_int32), ("afsai_eps", C.c_double)]


class CsrOut(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("rp", C.POINTER(C.c_int32)),
                ("ci", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIBPATH)
        vp = C.c_void_p
        i32, u64, dbl = C.c_int32, C.c_uint64, C.c_double
        L.orc_params_default.argtypes = [C.POINTER(Params)]
        L.orc_validate.argtypes = [i32, vp, vp, vp]
        L.orc_strength.argtypes = [i32, vp, vp, vp, dbl, vp, vp]
        L.orc_splitmix64.argtypes = [u64, u64]; L.orc_splitmix64.restype = u64
        L.orc_pmis_rand.argtypes = [u64, i32, i32]; L.orc_pmis_rand.restype = u64
        L.orc_pmis.argtypes = [i32, vp, vp, vp, vp, u64, i32, vp, vp]
        L.orc_interp_direct.argtypes = [i32, vp, vp, vp, vp, vp, C.POINTER(CsrOut)]
        L.orc_interp.argtypes = [i32, vp, vp, vp, vp, vp, i32, C.POINTER(CsrOut)]
        L.orc_orthonormalize.argtypes = [i32, i32, vp]
        L.orc_bamg.argtypes = [i32, vp, vp, vp, vp, i32, vp, i32, i32, dbl, dbl, C.POINTER(CsrOut)]
        L.orc_psmooth.argtypes = [C.POINTER(CsrOut), vp, dbl, C.POINTER(CsrOut), C.POINTER(CsrOut)]
        L.orc_pfilter.argtypes = [C.POINTER(CsrOut), dbl, i32, vp, C.POINTER(CsrOut)]
        L.orc_setup_tv.argtypes = [i32, vp, vp, vp, i32, vp, C.POINTER(Params), C.POINTER(vp)]
        L.orc_symeig.argtypes = [i32, vp, vp, vp]
        L.orc_srqm.argtypes = [C.POINTER(CsrOut), vp, C.POINTER(CsrOut), C.POINTER(CsrOut), i32, vp, i32, vp]
        L.orc_transpose.argtypes = [C.POINTER(CsrOut), C.POINTER(CsrOut)]
        L.orc_spgemm.argtypes = [C.POINTER(CsrOut), C.POINTER(CsrOut), C.POINTER(CsrOut)]
        L.orc_cholesky.argtypes = [i32, vp]
        L.orc_chol_solve.argtypes = [i32, vp, vp, vp]
        L.orc_gershgorin_omega.argtypes = [i32, vp, vp, vp]; L.orc_gershgorin_omega.restype = dbl
        L.orc_fsai.argtypes = [C.POINTER(CsrOut), C.POINTER(CsrOut)]
        L.orc_afsai.argtypes = [C.POINTER(CsrOut), i32, i32, dbl, C.POINTER(CsrOut), vp]
        L.orc_afsai_rows.argtypes = [C.POINTER(CsrOut), i32, i32, dbl, i32, vp, vp, vp, vp, vp]
        L.orc_fsai_omega.argtypes = [C.POINTER(CsrOut), C.POINTER(CsrOut), C.c_uint64, i32, vp]
        L.orc_csr_free.argtypes = [C.POINTER(CsrOut)]
        L.orc_setup.argtypes = [i32, vp, vp, vp, C.POINTER(Params), C.POINTER(vp)]
        L.orc_num_levels.argtypes = [vp]
        L.orc_level_sizes.argtypes = [vp, i32, vp, vp, vp, vp]
        L.orc_export.argtypes = [vp, i32, i32, vp, vp, vp]
        L.orc_vcycle.argtypes = [vp, vp, vp]
        L.orc_solve.argtypes = [vp, vp, dbl, i32, i32, vp, vp, vp, i32, vp]
        L.orc_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _csr_arrays(A):
    """Accept problems.CSR, a (nrows, ncols, rp, ci, val) tuple, or a scipy CSR matrix."""
    if hasattr(A, "row_ptr"):
        return A.n, A.n, A.row_ptr, A.col_idx, A.val
    if hasattr(A, "indptr"):
        return A.shape[0], A.shape[1], A.indptr, A.indices, A.data
    nr, nc, rp, ci, v = A
    return nr, nc, rp, ci, v


def _to_out(n, nc, rp, ci, v):
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.float64)
    o = CsrOut(n, nc, rp.ctypes.data_as(C.POINTER(C.c_int32)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
               v.ctypes.data_as(C.POINTER(C.c_double)))
    return o, (rp, ci, v)


def _from_out(o):
    nnz = o.rp[o.nrows] if o.nrows > 0 else 0
    rp = np.ctypeslib.as_array(o.rp, shape=(o.nrows + 1,)).copy()
    ci = np.ctypeslib.as_array(o.ci, shape=(max(nnz, 1),))[:nnz].copy() if nnz else np.zeros(0, np.int32)
    v = np.ctypeslib.as_array(o.val, shape=(max(nnz, 1),))[:nnz].copy() if nnz else np.zeros(0)
    res = (int(o.nrows), int(o.ncols), rp, ci, v)
    lib().orc_csr_free(C.byref(o))
    return res


def params(**kw) -> Params:
    p = Params()
    lib().orc_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def validate(A) -> int:
    n, _, rp, ci, v = _csr_arrays(A)
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    v = np.ascontiguousarray(v, np.float64)
    return lib().orc_validate(n, _p(rp), _p(ci), _p(v))


def strength(A, theta=0.25):
    n, _, rp, ci, v = _csr_arrays(A)
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    v = np.ascontiguousarray(v, np.float64)
    s = np.zeros(len(ci), np.uint8)
    cnt = np.zeros(n, np.int32)
    lib().orc_strength(n, _p(rp), _p(ci), _p(v), theta, _p(s), _p(cnt))
    return s, cnt


def splitmix64(seed: int, counter: int) -> int:
    return int(lib().orc_splitmix64(seed, counter))


def pmis_rand(seed: int, level: int, i: int) -> int:
    return int(lib().orc_pmis_rand(seed, level, i))


def pmis(A, strong, st_count, seed=0, level=0):
    n, _, rp, ci, _ = _csr_arrays(A)
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    strong = np.ascontiguousarray(strong, np.uint8); st_count = np.ascontiguousarray(st_count, np.int32)
    cf = np.zeros(n, np.int8)
    rounds = np.zeros(1, np.int32)
    st = lib().orc_pmis(n, _p(rp), _p(ci), _p(strong), _p(st_count), seed, level, _p(cf), _p(rounds))
    assert st == OK
    return cf, int(rounds[0])


def interp_direct(A, strong, cf):
    n, _, rp, ci, v = _csr_arrays(A)
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    v = np.ascontiguousarray(v, np.float64)
    strong = np.ascontiguousarray(strong, np.uint8); cf = np.ascontiguousarray(cf, np.int8)
    o = CsrOut()
    st = lib().orc_interp_direct(n, _p(rp), _p(ci), _p(v), _p(strong), _p(cf), C.byref(o))
    assert st == OK
    return _from_out(o)


def interp(A, strong, cf, variant):
    """P for a given strength pattern and C/F split (INTERP_* variant)."""
    n, _, rp, ci, v = _csr_arrays(A)
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    v = np.ascontiguousarray(v, np.float64)
    strong = np.ascontiguousarray(strong, np.uint8); cf = np.ascontiguousarray(cf, np.int8)
    o = CsrOut()
    st = lib().orc_interp(n, _p(rp), _p(ci), _p(v), _p(strong), _p(cf), variant, C.byref(o))
    assert st == OK
    return _from_out(o)


def orthonormalize(V):
    """Orthonormal basis of the test space V (n x nt), as the BAMG set-up forms it."""
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    n, nt = V.shape
    st = lib().orc_orthonormalize(n, nt, _p(V))
    if st != OK:
        raise OracleError(st)
    return V


def bamg(A, strong, cf, V, lmin=1, lmax=2, eps=1e-3, mu=10.0):
    """BAMG prolongation for test space V (n x nt, used as given) and a C/F split."""
    n, _, rp, ci, v = _csr_arrays(A)
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    strong = np.ascontiguousarray(strong, np.uint8); cf = np.ascontiguousarray(cf, np.int8)
    V = np.ascontiguousarray(V, np.float64)
    o = CsrOut()
    st = lib().orc_bamg(n, _p(rp), _p(ci), _p(strong), _p(cf), V.shape[1], _p(V), lmin, lmax, eps, mu, C.byref(o))
    if st != OK:
        raise OracleError(st)
    return _from_out(o)


def psmooth(A, dinv, omega, P):
    """P - omega D^{-1} A P (union pattern)."""
    oa, ka = _to_out(*_csr_arrays(A))
    op, kp = _to_out(*_csr_arrays(P))
    d = np.ascontiguousarray(dinv, np.float64)
    r = CsrOut()
    assert lib().orc_psmooth(C.byref(oa), _p(d), float(omega), C.byref(op), C.byref(r)) == OK
    return _from_out(r)


def pfilter(P, rho, W):
    """Filtered P (rho of each row's absolute sum kept) compensated on W (nc x nt)."""
    op, kp = _to_out(*_csr_arrays(P))
    W = np.ascontiguousarray(W, np.float64)
    if W.ndim == 1:
        W = W[:, None]
    r = CsrOut()
    assert lib().orc_pfilter(C.byref(op), float(rho), W.shape[1], _p(W), C.byref(r)) == OK
    return _from_out(r)


def symeig(Cm):
    """Eigenvalues and eigenvectors (columns) of a symmetric matrix, m <= 16."""
    Cm = np.array(Cm, dtype=np.float64, order="C", copy=True)
    m = Cm.shape[0]
    lam = np.zeros(m)
    Q = np.zeros((m, m))
    st = lib().orc_symeig(m, _p(Cm), _p(lam), _p(Q))
    if st != OK:
        raise OracleError(st)
    return lam, Q


def srqm(A, V, iters, dinv=None, G=None):
    """SRQM refinement of an orthonormal test space V (n x nt) with the
    preconditioner D^{-1} (dinv) or G^T G (G, a lower CSR).  Returns the new
    V and the number of steps taken."""
    oa, ka = _to_out(*_csr_arrays(A))
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    n, nt = V.shape
    done = np.zeros(1, np.int32)
    if G is not None:
        og, kg = _to_out(*_csr_arrays(G))
        ot = CsrOut()
        assert lib().orc_transpose(C.byref(og), C.byref(ot)) == OK
        st = lib().orc_srqm(C.byref(oa), None, C.byref(og), C.byref(ot), nt, _p(V), iters, _p(done))
        lib().orc_csr_free(C.byref(ot))
    else:
        d = np.ascontiguousarray(dinv, np.float64)
        st = lib().orc_srqm(C.byref(oa), _p(d), None, None, nt, _p(V), iters, _p(done))
    if st != OK:
        raise OracleError(st)
    return V, int(done[0])


def transpose(X):
    o, keep = _to_out(*_csr_arrays(X))
    r = CsrOut()
    assert lib().orc_transpose(C.byref(o), C.byref(r)) == OK
    return _from_out(r)


def spgemm(X, Y):
    ox, kx = _to_out(*_csr_arrays(X))
    oy, ky = _to_out(*_csr_arrays(Y))
    r = CsrOut()
    assert lib().orc_spgemm(C.byref(ox), C.byref(oy), C.byref(r)) == OK
    return _from_out(r)


def galerkin(A, P):
    """A_c = P^T (A P) as the oracle forms it."""
    R = transpose(P)
    AP = spgemm(A, P)
    return spgemm(R, AP)


def cholesky(a: np.ndarray):
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    st = lib().orc_cholesky(a.shape[0], _p(a))
    return st, a


def chol_solve(L: np.ndarray, y: np.ndarray) -> np.ndarray:
    L = np.ascontiguousarray(L, np.float64); y = np.ascontiguousarray(y, np.float64)
    z = np.zeros_like(y)
    lib().orc_chol_solve(L.shape[0], _p(L), _p(y), _p(z))
    return z


def gershgorin_omega(A) -> float:
    n, _, rp, ci, v = _csr_arrays(A)
    rp = np.ascontiguousarray(rp, np.int32); ci = np.ascontiguousarray(ci, np.int32)
    v = np.ascontiguousarray(v, np.float64)
    return float(lib().orc_gershgorin_omega(n, _p(rp), _p(ci), _p(v)))


def fsai(A):
    """Static FSAI factor G on the lower-triangular pattern of A (status, G)."""
    o, keep = _to_out(*_csr_arrays(A))
    r = CsrOut()
    st = lib().orc_fsai(C.byref(o), C.byref(r))
    if st != OK:
        lib().orc_csr_free(C.byref(r))
        return st, None
    return st, _from_out(r)


def afsai(A, steps=10, step=2, eps=0.01):
    """Adaptive FSAI factor (status, G, largest candidate set)."""
    o, keep = _to_out(*_csr_arrays(A))
    r = CsrOut()
    mc = np.zeros(1, np.int32)
    st = lib().orc_afsai(C.byref(o), steps, step, eps, C.byref(r), _p(mc))
    if st != OK:
        lib().orc_csr_free(C.byref(r))
        return st, None, int(mc[0])
    return st, _from_out(r), int(mc[0])


def afsai_rows(A, rows, steps=10, step=2, eps=0.01):
    """Rows `rows` of the adaptive FSAI factor: list of (columns, values)."""
    o, keep = _to_out(*_csr_arrays(A))
    sel = np.ascontiguousarray(rows, np.int32)
    mcap = steps * step + 1
    cols = np.zeros(max(len(sel), 1) * mcap, np.int32)
    vals = np.zeros(max(len(sel), 1) * mcap)
    cnt = np.zeros(max(len(sel), 1), np.int32)
    mc = np.zeros(1, np.int32)
    st = lib().orc_afsai_rows(C.byref(o), steps, step, eps, len(sel), _p(sel), _p(cols), _p(vals), _p(cnt), _p(mc))
    if st != OK:
        raise OracleError(st)
    return [(cols[t * mcap:t * mcap + cnt[t]].copy(), vals[t * mcap:t * mcap + cnt[t]].copy())
            for t in range(len(sel))]


def fsai_omega(A, G, seed=2021, level=0) -> float:
    oa, ka = _to_out(*_csr_arrays(A))
    og, kg = _to_out(*_csr_arrays(G))
    w = np.zeros(1)
    assert lib().orc_fsai_omega(C.byref(oa), C.byref(og), seed, level, _p(w)) == OK
    return float(w[0])


class Hierarchy:
    """Oracle AMG hierarchy (setup) plus V-cycle and PCG."""

    def __init__(self, A, V=None, **kw):
        n, _, rp, ci, v = _csr_arrays(A)
        self._keep = (np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32),
                      np.ascontiguousarray(v, np.float64))
        self.n = n
        self.params = params(**kw)
        h = C.c_void_p()
        if V is None:
            st = lib().orc_setup(n, _p(self._keep[0]), _p(self._keep[1]), _p(self._keep[2]),
                                 C.byref(self.params), C.byref(h))
        else:
            Vc = np.ascontiguousarray(V, np.float64)
            st = lib().orc_setup_tv(n, _p(self._keep[0]), _p(self._keep[1]), _p(self._keep[2]), Vc.shape[1],
                                    _p(Vc), C.byref(self.params), C.byref(h))
        self.status = st
        self.h = h if st == OK else None
        if st != OK:
            raise OracleError(st)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    @property
    def nlev(self) -> int:
        return lib().orc_num_levels(self.h)

    def sizes(self, l):
        a = [np.zeros(1, np.int32) for _ in range(4)]
        assert lib().orc_level_sizes(self.h, l, *[_p(x) for x in a]) == OK
        return tuple(int(x[0]) for x in a)  # n, nnzA, nnzP, nc

    def A(self, l):
        n, nnz, _, _ = self.sizes(l)
        rp = np.zeros(n + 1, np.int32); ci = np.zeros(nnz, np.int32); v = np.zeros(nnz)
        assert lib().orc_export(self.h, l, X_A, _p(rp), _p(ci), _p(v)) == OK
        return (n, n, rp, ci, v)

    def _pr(self, l, what):
        n, _, nnzp, nc = self.sizes(l)
        rows = n if what == X_P else nc
        cols = nc if what == X_P else n
        rp = np.zeros(rows + 1, np.int32); ci = np.zeros(nnzp, np.int32); v = np.zeros(nnzp)
        assert lib().orc_export(self.h, l, what, _p(rp), _p(ci), _p(v)) == OK
        return (rows, cols, rp, ci, v)

    def P(self, l):
        return self._pr(l, X_P)

    def R(self, l):
        return self._pr(l, X_R)

    def cf(self, l):
        n = self.sizes(l)[0]
        a = np.zeros(n, np.int8)
        assert lib().orc_export(self.h, l, X_CF, _p(a), None, None) == OK
        return a

    def strong(self, l):
        nnz = self.sizes(l)[1]
        a = np.zeros(nnz, np.uint8)
        assert lib().orc_export(self.h, l, X_STRONG, _p(a), None, None) == OK
        return a

    def dinv(self, l):
        a = np.zeros(self.sizes(l)[0])
        assert lib().orc_export(self.h, l, X_DINV, _p(a), None, None) == OK
        return a

    def has_G(self, l):
        """Whether level l smooths with FSAI (its factor can be exported)."""
        try:
            self.G(l)
            return True
        except AssertionError:
            return False

    def G(self, l):
        """FSAI factor of level l (FSAI smoother only)."""
        n = self.sizes(l)[0]
        rp = np.zeros(n + 1, np.int32)
        assert lib().orc_export(self.h, l, X_G, _p(rp), None, None) == OK
        nnzg = int(rp[n])
        ci = np.zeros(max(nnzg, 1), np.int32); v = np.zeros(max(nnzg, 1))
        assert lib().orc_export(self.h, l, X_G, _p(rp), _p(ci), _p(v)) == OK
        ci, v = ci[:nnzg], v[:nnzg]
        return (n, n, rp, ci, v)

    def omega(self, l):
        a = np.zeros(1)
        assert lib().orc_export(self.h, l, X_OMEGA, _p(a), None, None) == OK
        return float(a[0])

    def chol(self):
        l = self.nlev - 1
        n = self.sizes(l)[0]
        a = np.zeros((n, n))
        assert lib().orc_export(self.h, l, X_CHOL, _p(a), None, None) == OK
        return a

    def vcycle(self, y):
        y = np.ascontiguousarray(y, np.float64)
        z = np.zeros_like(y)
        lib().orc_vcycle(self.h, _p(y), _p(z))
        return z

    def solve(self, b, rtol=1e-8, max_iter=None, precond=True):
        b = np.ascontiguousarray(b, np.float64)
        mi = self.params.max_iter if max_iter is None else max_iter
        x = np.zeros_like(b)
        it = np.zeros(1, np.int32)
        hist = np.zeros(mi + 1)
        rel = np.zeros(1)
        st = lib().orc_solve(self.h, _p(b), rtol, mi, 1 if precond else 0, _p(x), _p(it), _p(hist),
                             mi + 1, _p(rel))
        k = int(it[0])
        return SolveResult(st, x, k, hist[:k + 1].copy(), float(rel[0]))

    def complexities(self):
        ns = [self.sizes(l)[0] for l in range(self.nlev)]
        nz = [self.sizes(l)[1] for l in range(self.nlev)]
        return sum(ns) / ns[0], sum(nz) / nz[0]


class SolveResult:
    def __init__(self, status, x, iters, hist, true_relres):
        self.status, self.x, self.iters, self.hist, self.true_relres = status, x, iters, hist, true_relres

    def __repr__(self):
        return f"SolveResult(status={self.status}, iters={self.iters}, true_relres={self.true_relres:.3e})"


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status
