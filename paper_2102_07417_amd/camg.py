"""ctypes binding of libcamg (include/camg.h).

Argument marshalling only: every step of set-up and solve runs in the HIP
kernels of the library.  Device arrays are passed as torch CUDA tensors
(``.data_ptr()``), streams as ``torch.cuda.Stream`` objects; host arrays as
numpy arrays.  If the shared library is missing this module raises at
import of the library (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libcamg.so")

OK, E_MAXIT, E_ACCURACY, E_ARG, E_CSR, E_NOT_SPD, E_BREAKDOWN, E_COARSE, E_NOMEM, E_DEVICE, E_BUSY = (
    0, 1, 2, -1, -2, -3, -4, -5, -6, -7, -8)
# outcomes of a solve whose outputs are valid (the last iterate)
SOLVE_OUTCOMES = (OK, E_MAXIT, E_ACCURACY, E_BREAKDOWN)
FP64, MIXED_FP32 = 0, 1
X_A, X_P, X_R, X_CF, X_STRONG, X_DINV, X_OMEGA, X_COARSE_INV, X_STCNT, X_G = range(10)
MAX_LEVELS = 32

EXPORTED = [
    "camg_abi_version", "camg_status_str", "camg_last_error", "camg_params_default", "camg_setup",
    "camg_setup_dev", "camg_setup_tv", "camg_setup_tv_dev", "camg_solve", "camg_solve_dev", "camg_solve_multi_dev", "camg_vcycle_dev", "camg_info",
    "camg_level_sizes", "camg_export_level", "camg_galerkin", "camg_free_host", "camg_destroy", "camg_profile",
    "camg_set_option", "camg_engine_footprint", "camg_engine_create", "camg_engine_start", "camg_engine_step",
    "camg_engine_state", "camg_engine_finish", "camg_engine_destroy", "camg_server_create", "camg_server_add",
    "camg_server_submit", "camg_server_poll", "camg_server_stats", "camg_server_destroy", "camg_solve_batch_dev",
    "camg_solve_batch_noalloc_dev",
]
OPT_GRAPH = 1
SMOOTH_JACOBI, SMOOTH_FSAI, SMOOTH_FSAI_JACOBI, SMOOTH_AFSAI = 0, 1, 2, 3
AFSAI_MAXM, AFSAI_MAXCAND = 32, 2048
INTERP_DIRECT, INTERP_CLASSICAL, INTERP_EXTI, INTERP_HYBRID, INTERP_BAMG = 0, 1, 2, 3, 4
OPT_AUTOTUNE = 2
OPT_COMPACT_COLS = 3


class camg_params(C.Structure):
    _fields_ = [("theta", C.c_double), ("seed", C.c_uint64), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("omega", C.c_double), ("max_levels", C.c_int32), ("max_coarse", C.c_int32),
                ("precision", C.c_int32), ("max_iter", C.c_int32), ("smoother", C.c_int32),
                ("interp", C.c_int32), ("rap_chunk", C.c_int64), ("bamg_lmin", C.c_int32),
                ("bamg_lmax", C.c_int32), ("bamg_eps", C.c_double), ("bamg_mu", C.c_double),
                ("psmooth", C.c_int32), ("pfilter", C.c_double), ("srqm_iters", C.c_int32),
                ("afsai_steps", C.c_int32), ("afsai_step", C.c_int32), ("afsai_eps", C.c_double)]


class camg_info_t(C.Structure):
    _fields_ = [("levels", C.c_int32), ("n", C.c_int32 * MAX_LEVELS), ("nnz", C.c_int64 * MAX_LEVELS),
                ("nnz_p", C.c_int64 * MAX_LEVELS), ("pmis_rounds", C.c_int32 * MAX_LEVELS),
                ("omega", C.c_double * MAX_LEVELS), ("grid_complexity", C.c_double),
                ("operator_complexity", C.c_double), ("device_bytes", C.c_int64), ("setup_ms", C.c_double),
                ("precision", C.c_int32), ("setup_phase_ms", C.c_double * 8),
                ("compact_cols", C.c_int32)]
SETUP_PHASES = ["input", "smoother", "strength_pmis", "interpolation", "transpose", "galerkin", "last_level",
                "solve_prep"]


_lib = None


def load(path: str | None = None):
    """Load libcamg.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIBPATH
    if not os.path.exists(p):
        raise OSError(f"libcamg.so not found at {p}; build it with paper_2102_07417_amd/build.py")
    L = C.CDLL(p)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.camg_abi_version.restype = i32
    L.camg_status_str.argtypes = [C.c_int]; L.camg_status_str.restype = C.c_char_p
    L.camg_last_error.restype = C.c_char_p
    L.camg_params_default.argtypes = [C.POINTER(camg_params)]
    L.camg_setup.argtypes = [i32, vp, vp, vp, C.POINTER(camg_params), C.POINTER(vp)]
    L.camg_setup_dev.argtypes = [i32, vp, vp, vp, C.POINTER(camg_params), vp, C.POINTER(vp)]
    L.camg_setup_tv.argtypes = [i32, vp, vp, vp, i32, vp, C.POINTER(camg_params), C.POINTER(vp)]
    L.camg_setup_tv_dev.argtypes = [i32, vp, vp, vp, i32, vp, C.POINTER(camg_params), vp, C.POINTER(vp)]
    L.camg_solve.argtypes = [vp, vp, dbl, vp, vp, vp, i32, vp]
    L.camg_solve_dev.argtypes = [vp, vp, dbl, vp, vp, vp, i32, vp, vp]
    L.camg_solve_multi_dev.argtypes = [vp, i32, vp, dbl, vp, vp, vp, i32, vp, vp]
    L.camg_vcycle_dev.argtypes = [vp, vp, vp, vp]
    L.camg_info.argtypes = [vp, C.POINTER(camg_info_t)]
    L.camg_level_sizes.argtypes = [vp, i32, vp, vp, vp, vp]
    L.camg_export_level.argtypes = [vp, i32, i32, vp, vp, vp]
    L.camg_galerkin.argtypes = [i32, vp, vp, vp, i32, vp, vp, vp, C.POINTER(C.POINTER(C.c_int32)),
                                C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.POINTER(C.c_double)), C.POINTER(i64)]
    L.camg_free_host.argtypes = [vp]
    L.camg_destroy.argtypes = [vp]
    L.camg_profile.argtypes = [vp, i32, vp, vp]
    L.camg_set_option.argtypes = [vp, i32, i64]
    L.camg_engine_footprint.argtypes = [vp, i32, vp]
    L.camg_engine_create.argtypes = [vp, i32, i32, vp, C.POINTER(vp)]
    L.camg_engine_start.argtypes = [vp, i32, i32, vp, i32, dbl, i32]
    L.camg_engine_step.argtypes = [vp, i32, vp]
    L.camg_engine_state.argtypes = [vp, vp, vp, vp]
    L.camg_engine_finish.argtypes = [vp, i32, i32, vp, i32, vp]
    L.camg_engine_destroy.argtypes = [vp]
    L.camg_solve_batch_dev.argtypes = [i32, vp, vp, vp, dbl, vp, vp, vp, vp]
    L.camg_solve_batch_dev.restype = C.c_int
    L.camg_solve_batch_noalloc_dev.argtypes = [i32, vp, vp, vp, dbl, vp, vp, vp, vp]
    L.camg_solve_batch_noalloc_dev.restype = C.c_int
    L.camg_server_create.argtypes = [i64, C.POINTER(vp)]
    L.camg_server_add.argtypes = [vp, vp, i32, i32, vp]
    L.camg_server_submit.argtypes = [vp, i32, i32, vp, i32, vp, i32, dbl, i32, i64]
    L.camg_server_poll.argtypes = [vp, vp, i32, vp]
    L.camg_server_stats.argtypes = [vp, vp, vp, vp, vp]
    L.camg_server_destroy.argtypes = [vp]
    for name in ("camg_server_create", "camg_server_add", "camg_server_submit", "camg_server_poll",
                 "camg_server_stats", "camg_server_destroy"):
        getattr(L, name).restype = C.c_int
    for name in ("camg_engine_footprint", "camg_engine_create", "camg_engine_start", "camg_engine_step",
                 "camg_engine_state", "camg_engine_finish", "camg_engine_destroy"):
        getattr(L, name).restype = C.c_int
    for name in ("camg_profile", "camg_set_option", "camg_setup", "camg_setup_dev", "camg_solve", "camg_solve_dev", "camg_solve_multi_dev",
                 "camg_vcycle_dev", "camg_info", "camg_level_sizes", "camg_export_level", "camg_galerkin",
                 "camg_destroy"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


class CamgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"camg status {status}: {msg}")
        self.status = status


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check(st: int, allow=(OK,)):
    if st not in allow:
        raise CamgError(st, load().camg_last_error().decode())
    return st


def _dev(t, name, dtype, shape=None, numel=None, device=True):
    """Device pointer of a torch tensor after checking that it lives on a
    GPU, has the expected dtype, is contiguous and has the expected shape or
    size.  The C entry points read and write these buffers from kernels, so
    a host tensor, a strided view or a short buffer must never reach them."""
    if not hasattr(t, "data_ptr") or not hasattr(t, "is_cuda"):
        raise TypeError(f"{name}: a torch tensor on the GPU is expected, got {type(t).__name__}")
    import torch
    want = {"f64": torch.float64, "i32": torch.int32}[dtype]
    if t.dtype != want:
        raise TypeError(f"{name}: dtype {t.dtype}, {want} expected")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, {tuple(shape)} expected")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, {numel} expected")
    if device and not t.is_cuda:
        raise ValueError(f"{name}: tensor is on {t.device}, a GPU tensor is expected")
    return C.c_void_p(t.data_ptr())


def _n_of(h):
    """Unknowns of the hierarchy's finest level."""
    n = np.zeros(1, np.int32)
    _check(load().camg_level_sizes(h, 0, _p(n), None, None, None))
    return int(n[0])


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def params(**kw) -> camg_params:
    p = camg_params()
    load().camg_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


# ------------------------------------------------------------------ C-ABI names
def camg_setup(n, row_ptr, col_idx, val, prm=None):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    h = C.c_void_p()
    st = load().camg_setup(int(n), _p(rp), _p(ci), _p(v), C.byref(prm) if prm is not None else None, C.byref(h))
    return st, h


def _dev_csr(n, d_row_ptr, d_col_idx, d_val):
    for dev in (False, True):  # every size check first, then the devices
        prp = _dev(d_row_ptr, "row_ptr", "i32", numel=int(n) + 1, device=dev)
        pci = _dev(d_col_idx, "col_idx", "i32", device=dev)
        pv = _dev(d_val, "val", "f64", numel=d_col_idx.numel(), device=dev)
    nnz = int(d_row_ptr[-1].item()) if int(n) >= 0 else 0
    if not 0 <= nnz <= d_col_idx.numel():
        raise ValueError(f"row_ptr[n] = {nnz} does not fit col_idx / val of {d_col_idx.numel()} entries")
    return prp, pci, pv


def camg_setup_dev(n, d_row_ptr, d_col_idx, d_val, prm=None, stream=None):
    h = C.c_void_p()
    prp, pci, pv = _dev_csr(n, d_row_ptr, d_col_idx, d_val)
    st = load().camg_setup_dev(int(n), prp, pci, pv, C.byref(prm) if prm is not None else None,
                               _stream_ptr(stream), C.byref(h))
    return st, h


def camg_setup_tv(n, row_ptr, col_idx, val, V, prm=None):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    V = np.ascontiguousarray(V, np.float64)
    h = C.c_void_p()
    st = load().camg_setup_tv(int(n), _p(rp), _p(ci), _p(v), int(V.shape[1]), _p(V),
                              C.byref(prm) if prm is not None else None, C.byref(h))
    return st, h


def camg_setup_tv_dev(n, d_row_ptr, d_col_idx, d_val, d_V, prm=None, stream=None):
    h = C.c_void_p()
    prp, pci, pv = _dev_csr(n, d_row_ptr, d_col_idx, d_val)
    if d_V.dim() != 2:
        raise ValueError("V: an n-by-nt block is expected")
    pV = _dev(d_V, "V", "f64", shape=(int(n), d_V.shape[1]))
    st = load().camg_setup_tv_dev(int(n), prp, pci, pv, int(d_V.shape[1]), pV,
                                  C.byref(prm) if prm is not None else None, _stream_ptr(stream), C.byref(h))
    return st, h


def camg_solve(h, b, rtol, x, hist_cap=0):
    b = np.ascontiguousarray(b, np.float64)
    it = np.zeros(1, np.int32)
    hist = np.zeros(max(hist_cap, 1))
    rel = np.zeros(1)
    st = load().camg_solve(h, _p(b), float(rtol), _p(x), _p(it), _p(hist) if hist_cap else None, int(hist_cap),
                           _p(rel))
    return st, int(it[0]), hist[:min(hist_cap, int(it[0]) + 1)], float(rel[0])


def camg_solve_dev(h, d_b, rtol, d_x, hist_cap=0, stream=None):
    _dev(d_b, "b", "f64")
    _dev(d_x, "x", "f64")
    n = _n_of(h)
    pb = _dev(d_b, "b", "f64", numel=n)
    px = _dev(d_x, "x", "f64", numel=n)
    it = np.zeros(1, np.int32)
    hist = np.zeros(max(hist_cap, 1))
    rel = np.zeros(1)
    st = load().camg_solve_dev(h, pb, float(rtol), px, _p(it),
                               _p(hist) if hist_cap else None, int(hist_cap), _p(rel), _stream_ptr(stream))
    return st, int(it[0]), hist[:min(hist_cap, int(it[0]) + 1)], float(rel[0])


def camg_solve_multi_dev(h, k, d_B, rtol, d_X, hist_cap=0, stream=None):
    it = np.zeros(k, np.int32)
    hist = np.zeros((k, max(hist_cap, 1)))
    rel = np.zeros(k)
    _dev(d_B, "B", "f64")
    _dev(d_X, "X", "f64")
    n = _n_of(h)
    pB = _dev(d_B, "B", "f64", shape=(n, int(k)))
    pX = _dev(d_X, "X", "f64", shape=(n, int(k)))
    st = load().camg_solve_multi_dev(h, int(k), pB, float(rtol), pX,
                                     _p(it), _p(hist) if hist_cap else None, int(hist_cap), _p(rel),
                                     _stream_ptr(stream))
    return st, it, hist, rel


def camg_vcycle_dev(h, d_y, d_z, stream=None):
    _dev(d_y, "y", "f64")
    _dev(d_z, "z", "f64")
    n = _n_of(h)
    py = _dev(d_y, "y", "f64", numel=n)
    pz = _dev(d_z, "z", "f64", numel=n)
    return load().camg_vcycle_dev(h, py, pz, _stream_ptr(stream))


def camg_info(h):
    info = camg_info_t()
    _check(load().camg_info(h, C.byref(info)))
    return info


def camg_level_sizes(h, l):
    a = [np.zeros(1, np.int32), np.zeros(1, np.int64), np.zeros(1, np.int64), np.zeros(1, np.int32)]
    _check(load().camg_level_sizes(h, int(l), *[_p(x) for x in a]))
    return tuple(int(x[0]) for x in a)


def camg_export_level(h, l, what, a, b=None, c=None):
    return load().camg_export_level(h, int(l), int(what), _p(a), None if b is None else _p(b),
                                    None if c is None else _p(c))


def camg_galerkin(A, P):
    """A, P: (nrows, ncols, rp, ci, val) tuples.  Returns the CSR tuple of P^T A P."""
    n, _, arp, aci, av = A
    _, nc, prp, pci, pv = P
    arrs = [np.ascontiguousarray(x, t) for x, t in [(arp, np.int32), (aci, np.int32), (av, np.float64),
                                                     (prp, np.int32), (pci, np.int32), (pv, np.float64)]]
    crp, cci, cv = C.POINTER(C.c_int32)(), C.POINTER(C.c_int32)(), C.POINTER(C.c_double)()
    nnz = C.c_int64()
    L = load()
    _check(L.camg_galerkin(int(n), _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), int(nc), _p(arrs[3]), _p(arrs[4]),
                           _p(arrs[5]), C.byref(crp), C.byref(cci), C.byref(cv), C.byref(nnz)))
    m = int(nnz.value)
    rp = np.ctypeslib.as_array(crp, shape=(nc + 1,)).copy()
    ci = np.ctypeslib.as_array(cci, shape=(max(m, 1),))[:m].copy()
    v = np.ctypeslib.as_array(cv, shape=(max(m, 1),))[:m].copy()
    for p in (crp, cci, cv):
        L.camg_free_host(C.cast(p, C.c_void_p))
    return (nc, nc, rp, ci, v)


def camg_profile(h, enable):
    """Returns (total_ms, launches) of the timed level-0 post-smoothing kernel
    since the last call, then enables/disables timing."""
    t = np.zeros(1)
    n = np.zeros(1, np.int64)
    _check(load().camg_profile(h, int(enable), _p(t), _p(n)))
    return float(t[0]), int(n[0])


def camg_set_option(h, option, value):
    return load().camg_set_option(h, int(option), int(value))


def camg_engine_footprint(h, slots):
    out = np.zeros(1, np.int64)
    _check(load().camg_engine_footprint(h, int(slots), _p(out)))
    return int(out[0])


class Engine:
    """Slot engine of a Solver: columns start, run and finish independently
    (continuous batching).  Device blocks are torch CUDA tensors."""

    def __init__(self, solver, slots, hist_cap=1, stream=None):
        self.solver = solver
        self.slots = slots
        e = C.c_void_p()
        _check(load().camg_engine_create(solver.h, int(slots), int(hist_cap), _stream_ptr(stream), C.byref(e)))
        self.e = e

    def start(self, slot0, d_B, rtol=1e-8, max_iter=1000):
        """d_B: n-by-m row-major (or length-n) float64 CUDA tensor."""
        m, ldb, pB = _dev_rows(d_B, "B", self.solver.n)
        _check(load().camg_engine_start(self.e, int(slot0), int(m), pB, int(ldb), float(rtol), int(max_iter)))

    def step(self, max_steps=1):
        r = np.zeros(1, np.int32)
        _check(load().camg_engine_step(self.e, int(max_steps), _p(r)))
        return int(r[0])

    def state(self):
        it = np.zeros(self.slots, np.int32)
        dn = np.zeros(self.slots, np.int32)
        st = np.zeros(self.slots, np.int32)
        _check(load().camg_engine_state(self.e, _p(it), _p(dn), _p(st)))
        return it, dn, st

    def finish(self, slot0, d_X):
        m, ldx, pX = _dev_rows(d_X, "X", self.solver.n)
        rel = np.zeros(m)
        _check(load().camg_engine_finish(self.e, int(slot0), int(m), pX, int(ldx), _p(rel)))
        return rel

    def close(self):
        if self.e:
            load().camg_engine_destroy(self.e)
            self.e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_rows(t, name, n):
    """(columns, row stride, pointer) of an n-by-m row-major float64 GPU
    block whose rows are contiguous (a column slice of a wider block is
    fine), or of a length-n vector."""
    if not hasattr(t, "is_cuda") or not t.is_cuda:
        raise ValueError(f"{name}: a float64 GPU tensor is expected")
    if t.dtype != torch_float64():
        raise TypeError(f"{name}: dtype {t.dtype}, torch.float64 expected")
    if t.dim() == 1:
        return 1, 1, _dev(t, name, "f64", numel=n)
    if t.dim() != 2 or t.shape[0] != n or t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name}: an {n}-by-m block with contiguous rows is expected, got shape "
                         f"{tuple(t.shape)} strides {tuple(t.stride())}")
    return int(t.shape[1]), int(t.stride(0)), C.c_void_p(t.data_ptr())


def torch_float64():
    import torch
    return torch.float64


NOALLOC_MAX_SYSTEMS = 1024


def solve_batch_dev(solvers, d_bs, d_xs, rtol=1e-8, stream=None, no_alloc=False):
    """Many small systems in one launch (one workgroup per system).  Returns
    (iters, true_relres, status) arrays; raises on a call error.  no_alloc:
    call camg_solve_batch_noalloc_dev (per-call buffers in the library's
    static device array, at most NOALLOC_MAX_SYSTEMS systems)."""
    m = len(solvers)
    if len(d_bs) != m or len(d_xs) != m:
        raise ValueError("one b and one x per system expected")
    hs = (C.c_void_p * m)(*[s.h for s in solvers])
    bs = (C.c_void_p * m)(*[_dev(t, f"b[{k}]", "f64", numel=solvers[k].n).value for k, t in enumerate(d_bs)])
    xs = (C.c_void_p * m)(*[_dev(t, f"x[{k}]", "f64", numel=solvers[k].n).value for k, t in enumerate(d_xs)])
    it = np.zeros(m, np.int32)
    rel = np.zeros(m)
    st = np.zeros(m, np.int32)
    fn = load().camg_solve_batch_noalloc_dev if no_alloc else load().camg_solve_batch_dev
    _check(fn(m, C.cast(hs, C.c_void_p), C.cast(bs, C.c_void_p), C.cast(xs, C.c_void_p),
              float(rtol), _p(it), _p(rel), _p(st), _stream_ptr(stream)))
    return it, rel, st


class camg_completion(C.Structure):
    _fields_ = [("tag", C.c_int64), ("status", C.c_int32), ("iters", C.c_int32), ("true_relres", C.c_double),
                ("queue_ms", C.c_double), ("latency_ms", C.c_double)]


def _buf_ptr(a, n, k):
    """Pointer and row stride (elements) of a row-major n-by-k (or length-n
    when k = 1) block: a torch tensor (CUDA or host) or a numpy array."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or a.strides[-1] != 8:
            raise ValueError("float64 block with contiguous rows expected")
        shape, ld = a.shape, (a.strides[0] // 8 if a.ndim == 2 else 1)
        ptr = a.ctypes.data
    else:
        if a.dtype != torch_float64() or a.stride(-1) != 1:
            raise ValueError("float64 block with contiguous rows expected")
        shape, ld = tuple(a.shape), (a.stride(0) if a.dim() == 2 else 1)
        ptr = a.data_ptr()
    if tuple(shape) not in ((n, k),) + (((n,),) if k == 1 else ()) or (len(shape) == 2 and ld < k):
        raise ValueError(f"block of shape {tuple(shape)}, ({n}, {k}) expected")
    return C.c_void_p(ptr), ld


class Server:
    """Resident hierarchies serving solve requests (continuous batching).
    Buffers passed to submit() are kept referenced until their request
    completes."""

    def __init__(self, budget_bytes):
        s = C.c_void_p()
        _check(load().camg_server_create(int(budget_bytes), C.byref(s)))
        self.s = s
        self.solvers = []
        self.live = {}
        self._out = (camg_completion * 512)()

    def add(self, solver, slots, iters_per_batch=0):
        sid = np.zeros(1, np.int32)
        _check(load().camg_server_add(self.s, solver.h, int(slots), int(iters_per_batch), _p(sid)))
        self.solvers.append(solver)
        return int(sid[0])

    def submit(self, system, B, X, rtol=1e-8, max_iter=1000, tag=0):
        k = 1 if B.ndim == 1 else B.shape[1]
        # an unknown system index is the library's to refuse (CAMG_E_ARG)
        n = self.solvers[int(system)].n if 0 <= int(system) < len(self.solvers) else B.shape[0]
        pb, ldb = _buf_ptr(B, n, k)
        px, ldx = _buf_ptr(X, n, k)
        _check(load().camg_server_submit(self.s, int(system), int(k), pb, int(ldb), px, int(ldx), float(rtol),
                                         int(max_iter), int(tag)))
        self.live[int(tag)] = (B, X)

    def poll(self):
        n = np.zeros(1, np.int32)
        _check(load().camg_server_poll(self.s, C.cast(self._out, C.c_void_p), len(self._out), _p(n)))
        res = []
        for i in range(int(n[0])):
            c = self._out[i]
            self.live.pop(int(c.tag), None)
            res.append({"tag": int(c.tag), "status": int(c.status), "iters": int(c.iters),
                        "true_relres": float(c.true_relres), "queue_ms": float(c.queue_ms),
                        "latency_ms": float(c.latency_ms)})
        return res

    def stats(self):
        u = np.zeros(2, np.int64)
        q = np.zeros(2, np.int32)
        _check(load().camg_server_stats(self.s, _p(u[0:1]), _p(u[1:2]), _p(q[0:1]), _p(q[1:2])))
        return {"arena_used": int(u[0]), "arena_size": int(u[1]), "queued": int(q[0]), "busy_slots": int(q[1])}

    def close(self):
        if self.s:
            load().camg_server_destroy(self.s)
            self.s = None
        self.live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def camg_destroy(h):
    return load().camg_destroy(h)


# ------------------------------------------------------------------ convenience
class Solver:
    """An AMG hierarchy resident on the current GPU.

    ``Solver(A)`` with A a problems.CSR (host arrays, copied to the device),
    or ``Solver.from_device(n, rp, ci, val)`` with torch CUDA tensors."""

    def __init__(self, A=None, stream=None, _handle=None, V=None, **kw):
        self.h = None
        if _handle is not None:
            self.h = _handle
        else:
            prm = params(**kw)
            if V is None:
                st, h = camg_setup(A.n, A.row_ptr, A.col_idx, A.val, prm)
            else:
                st, h = camg_setup_tv(A.n, A.row_ptr, A.col_idx, A.val, V, prm)
            _check(st)
            self.h = h
        self.info = camg_info(self.h)
        self.n = self.info.n[0]

    @classmethod
    def from_device(cls, n, d_rp, d_ci, d_val, stream=None, V=None, **kw):
        """V: optional test space (torch CUDA tensor, n x nt float64) for BAMG."""
        prm = params(**kw)
        if V is None:
            st, h = camg_setup_dev(n, d_rp, d_ci, d_val, prm, stream)
        else:
            st, h = camg_setup_tv_dev(n, d_rp, d_ci, d_val, V, prm, stream)
        _check(st)
        return cls(_handle=h)

    def close(self):
        if self.h:
            camg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nlev(self):
        return self.info.levels

    def sizes(self, l):
        return camg_level_sizes(self.h, l)

    def _csr(self, l, what):
        n, nnza, nnzp, nc = self.sizes(l)
        if what == X_A:
            nr, ncol, nnz = n, n, nnza
        elif what == X_P:
            nr, ncol, nnz = n, nc, nnzp
        else:
            nr, ncol, nnz = nc, n, nnzp
        rp = np.zeros(nr + 1, np.int32)
        ci = np.zeros(max(nnz, 1), np.int32)
        v = np.zeros(max(nnz, 1))
        _check(camg_export_level(self.h, l, what, rp, ci, v))
        return (nr, ncol, rp, ci[:nnz], v[:nnz])

    def A(self, l):
        return self._csr(l, X_A)

    def P(self, l):
        return self._csr(l, X_P)

    def R(self, l):
        return self._csr(l, X_R)

    def G(self, l):
        """FSAI factor of level l (the level must smooth with FSAI or aFSAI)."""
        n = self.sizes(l)[0]
        rp = np.zeros(n + 1, np.int32)
        _check(camg_export_level(self.h, l, X_G, rp))
        nnz = int(rp[n])
        ci = np.zeros(max(nnz, 1), np.int32)
        v = np.zeros(max(nnz, 1))
        _check(camg_export_level(self.h, l, X_G, rp, ci, v))
        return (n, n, rp, ci[:nnz], v[:nnz])

    def _vec(self, l, what, dtype, size=None):
        n = self.sizes(l)[0]
        a = np.zeros(size if size is not None else n, dtype)
        _check(camg_export_level(self.h, l, what, a))
        return a

    def cf(self, l):
        return self._vec(l, X_CF, np.int8)

    def strong(self, l):
        return self._vec(l, X_STRONG, np.uint8, self.sizes(l)[1])

    def stcnt(self, l):
        return self._vec(l, X_STCNT, np.int32)

    def dinv(self, l):
        return self._vec(l, X_DINV, np.float64)

    def omega(self, l):
        return float(self._vec(l, X_OMEGA, np.float64, 1)[0])

    def coarse_inverse(self):
        l = self.nlev - 1
        n = self.sizes(l)[0]
        a = np.zeros((n, n))
        _check(camg_export_level(self.h, l, X_COARSE_INV, a))
        return a

    def solve(self, b, rtol=1e-8, hist_cap=None):
        """Host vectors in and out."""
        x = np.zeros(self.n)
        cap = 100001 if hist_cap is None else hist_cap
        st, it, hist, rel = camg_solve(self.h, b, rtol, x, hist_cap=cap)
        _check(st, allow=SOLVE_OUTCOMES)
        return SolveResult(st, x, it, hist, rel)

    def solve_dev(self, d_b, d_x, rtol=1e-8, hist_cap=0, stream=None):
        st, it, hist, rel = camg_solve_dev(self.h, d_b, rtol, d_x, hist_cap=hist_cap, stream=stream)
        _check(st, allow=SOLVE_OUTCOMES)
        return SolveResult(st, None, it, hist, rel)

    def vcycle_dev(self, d_y, d_z, stream=None):
        _check(camg_vcycle_dev(self.h, d_y, d_z, stream))

    def set_option(self, option, value):
        _check(camg_set_option(self.h, option, value))

    def solve_multi_dev(self, d_B, d_X, rtol=1e-8, hist_cap=0, stream=None):
        """d_B, d_X: n-by-k row-major float64 CUDA tensors."""
        k = d_B.shape[1]
        st, it, hist, rel = camg_solve_multi_dev(self.h, k, d_B, rtol, d_X, hist_cap=hist_cap, stream=stream)
        _check(st, allow=SOLVE_OUTCOMES)
        return MultiResult(st, it, hist, rel)


class MultiResult:
    def __init__(self, status, iters, hist, true_relres):
        self.status, self.iters, self.hist, self.true_relres = status, iters, hist, true_relres


class SolveResult:
    def __init__(self, status, x, iters, hist, true_relres):
        self.status, self.x, self.iters, self.hist, self.true_relres = status, x, iters, hist, true_relres

    def __repr__(self):
        return f"SolveResult(status={self.status}, iters={self.iters}, true_relres={self.true_relres:.3e})"
