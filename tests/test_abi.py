"""The C-ABI library on the CPU: it loads, exports every function the
header declares, the Python binding lists the same set, and the binding's
structures have the header's layout (checked against a C program compiled
from the header).  No call here touches a GPU."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2102_07417_amd import camg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "camg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(camg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    try:
        return camg.load()
    except OSError as e:
        pytest.fail(f"libcamg.so missing or not loadable (run the build first): {e}")


def test_header_declares_functions():
    names = _declared()
    assert len(names) >= 30
    for must in ("camg_setup", "camg_solve", "camg_solve_dev", "camg_vcycle_dev", "camg_galerkin",
                 "camg_solve_multi_dev", "camg_server_poll", "camg_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows the same set
    assert sorted(camg.EXPORTED) == _declared()


def test_pure_host_calls(lib):
    assert lib.camg_abi_version() == 8
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7, -8):
        s = lib.camg_status_str(code)
        assert isinstance(s, bytes) and len(s) > 0
    p = camg.camg_params()
    lib.camg_params_default(C.byref(p))
    assert p.theta == 0.25 and p.nu_pre == 1 and p.nu_post == 1 and p.max_coarse == 256 and p.max_levels == 25
    assert p.precision == camg.FP64 and p.omega == 0.0 and p.smoother == camg.SMOOTH_JACOBI
    assert p.interp == camg.INTERP_DIRECT
    assert p.bamg_lmin == 1 and p.bamg_lmax == 2 and p.bamg_eps == 1e-3 and p.bamg_mu == 10.0


def test_argument_errors_without_device(lib):
    # null handles and pointers are rejected before any device work
    assert lib.camg_info(None, None) == camg.E_ARG
    assert lib.camg_destroy(None) == camg.OK
    assert lib.camg_engine_destroy(None) == camg.OK
    assert lib.camg_server_destroy(None) == camg.OK
    assert len(lib.camg_last_error()) >= 0


def test_noalloc_batch_limit_without_device(lib):
    # more systems than the static array holds: refused before any handle or
    # device is looked at
    m = camg.NOALLOC_MAX_SYSTEMS + 1
    hs = (C.c_void_p * m)()
    ptrs = (C.c_void_p * m)()
    st = lib.camg_solve_batch_noalloc_dev(m, C.cast(hs, C.c_void_p), C.cast(ptrs, C.c_void_p),
                                          C.cast(ptrs, C.c_void_p), 1e-8, None, None, None, None)
    assert st == camg.E_ARG and b"CAMG_NOALLOC_MAX_SYSTEMS" in lib.camg_last_error()
    # the header's limit is the binding's
    assert re.search(r"#define CAMG_NOALLOC_MAX_SYSTEMS (\d+)", open(HEADER).read()).group(1) == \
        str(camg.NOALLOC_MAX_SYSTEMS)


@pytest.mark.parametrize("field,value", [("interp", 4), ("interp", -1), ("smoother", 4), ("theta", 1.5),
                                         ("precision", 3), ("rap_chunk", -1), ("interp", 5),
                                         ("psmooth", 2), ("pfilter", 0.0), ("srqm_iters", -1),
                                         ("srqm_iters", 101), ("srqm_iters", 1)])
def test_bad_parameters_rejected_without_device(lib, field, value):
    # parameters are checked before the device is touched
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    v = np.array([2.0])
    p = camg.camg_params()
    lib.camg_params_default(C.byref(p))
    setattr(p, field, value)
    h = C.c_void_p()
    st = lib.camg_setup(1, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                        v.ctypes.data_as(C.c_void_p), C.byref(p), C.byref(h))
    assert st == camg.E_ARG and not h.value


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "camg.h"
int main(void) {
  printf("params %zu %zu %zu %zu %zu %zu %zu\n", sizeof(camg_params), offsetof(camg_params, omega),
         offsetof(camg_params, precision), offsetof(camg_params, max_iter), offsetof(camg_params, smoother),
         offsetof(camg_params, interp), offsetof(camg_params, rap_chunk));
  printf("bamg %zu %zu %zu %zu %zu %zu\n", offsetof(camg_params, bamg_lmin), offsetof(camg_params, bamg_eps),
         offsetof(camg_params, bamg_mu), offsetof(camg_params, psmooth), offsetof(camg_params, pfilter),
         offsetof(camg_params, srqm_iters));
  printf("afsai %zu %zu %zu\n", offsetof(camg_params, afsai_steps), offsetof(camg_params, afsai_step),
         offsetof(camg_params, afsai_eps));
  printf("info %zu %zu %zu %zu\n", sizeof(camg_info_t), offsetof(camg_info_t, nnz_p),
         offsetof(camg_info_t, setup_phase_ms), offsetof(camg_info_t, compact_cols));
  printf("completion %zu %zu %zu\n", sizeof(camg_completion), offsetof(camg_completion, true_relres),
         offsetof(camg_completion, latency_ms));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = dict((l.split()[0], [int(v) for v in l.split()[1:]])
               for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    P = camg.camg_params
    assert out["params"] == [C.sizeof(P), P.omega.offset, P.precision.offset, P.max_iter.offset, P.smoother.offset,
                             P.interp.offset, P.rap_chunk.offset]
    assert out["bamg"] == [P.bamg_lmin.offset, P.bamg_eps.offset, P.bamg_mu.offset, P.psmooth.offset,
                           P.pfilter.offset, P.srqm_iters.offset]
    assert out["afsai"] == [P.afsai_steps.offset, P.afsai_step.offset, P.afsai_eps.offset]
    I = camg.camg_info_t
    assert out["info"] == [C.sizeof(I), I.nnz_p.offset, I.setup_phase_ms.offset, I.compact_cols.offset]
    Q = camg.camg_completion
    assert out["completion"] == [C.sizeof(Q), Q.true_relres.offset, Q.latency_ms.offset]


def test_bamg_setup_rejected_without_device(lib):
    # BAMG without a test space, or with lmax above 2, is refused before any device work
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    v = np.array([2.0])
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    for kw in ({}, {"bamg_lmax": 3}):
        p = camg.camg_params()
        lib.camg_params_default(C.byref(p))
        p.interp = camg.INTERP_BAMG
        for k, val in kw.items():
            setattr(p, k, val)
        h = C.c_void_p()
        assert lib.camg_setup(1, vp(rp), vp(ci), vp(v), C.byref(p), C.byref(h)) == camg.E_ARG
        V = np.ones((1, 9))
        assert lib.camg_setup_tv(1, vp(rp), vp(ci), vp(v), 9, vp(V), C.byref(p), C.byref(h)) == camg.E_ARG


def test_afsai_parameters_rejected_without_device(lib):
    """Adaptive FSAI parameters outside their range are refused before any
    device work: afsai_steps * afsai_step + 1 above 32, a negative step
    count, no entries per step, a negative or NaN tolerance."""
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    v = np.array([2.0])
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    for kw in ({"afsai_steps": 16, "afsai_step": 2}, {"afsai_steps": -1}, {"afsai_step": 0},
               {"afsai_eps": -0.5}, {"afsai_eps": float("nan")}):
        p = camg.camg_params()
        lib.camg_params_default(C.byref(p))
        assert (p.afsai_steps, p.afsai_step, p.afsai_eps) == (10, 2, 0.01)
        p.smoother = camg.SMOOTH_AFSAI
        for k, val in kw.items():
            setattr(p, k, val)
        h = C.c_void_p()
        assert lib.camg_setup(1, vp(rp), vp(ci), vp(v), C.byref(p), C.byref(h)) == camg.E_ARG
        assert b"aFSAI" in lib.camg_last_error()
    hdr = open(HEADER).read()
    assert int(re.search(r"#define CAMG_AFSAI_MAXM (\d+)", hdr).group(1)) == camg.AFSAI_MAXM
    assert int(re.search(r"#define CAMG_AFSAI_MAXCAND (\d+)", hdr).group(1)) == camg.AFSAI_MAXCAND


def test_device_wrappers_refuse_bad_buffers(lib):
    """The *_dev wrappers check device, dtype, contiguity and size before a
    pointer reaches the library (a host address in a kernel would fault the
    GPU; a strided or short buffer would give wrong columns or out-of-bounds
    accesses).  Host tensors stand in for every case; nothing reaches a GPU."""
    torch = pytest.importorskip("torch")
    n = 6
    rp = torch.arange(0, 3 * (n + 1), 3, dtype=torch.int32)
    ci = torch.zeros(3 * n, dtype=torch.int32)
    va = torch.ones(3 * n, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        camg.camg_setup_dev(n, rp, ci, va)                       # host memory
    with pytest.raises(TypeError, match="dtype"):
        camg.camg_setup_dev(n, rp.long(), ci, va)                # int64 row pointer
    with pytest.raises(TypeError, match="dtype"):
        camg.camg_setup_dev(n, rp, ci, va.float())               # float32 values
    with pytest.raises(ValueError, match="contiguous"):
        camg.camg_setup_dev(n, rp, torch.zeros((3 * n, 2), dtype=torch.int32)[:, 0], va)
    with pytest.raises(ValueError, match="elements"):
        camg.camg_setup_dev(n, rp[:-1], ci, va)                  # row pointer of n entries
    with pytest.raises(ValueError, match="elements"):
        camg.camg_setup_dev(n, rp, ci, va[:-1])                  # values shorter than columns
    with pytest.raises(TypeError, match="torch tensor"):
        camg.camg_setup_dev(n, np.zeros(n + 1, np.int32), ci, va)
    b = torch.zeros(n, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        camg.camg_solve_dev(None, b, 1e-8, b.clone())
    with pytest.raises(TypeError, match="dtype"):
        camg.camg_solve_dev(None, b.float(), 1e-8, b.clone())
    with pytest.raises(ValueError, match="contiguous"):
        camg.camg_solve_dev(None, torch.zeros((n, 2), dtype=torch.float64)[:, 1], 1e-8, b.clone())
    with pytest.raises(ValueError, match="GPU tensor"):
        camg.camg_vcycle_dev(None, b, b.clone())
    B = torch.zeros((n, 3), dtype=torch.float64)
    with pytest.raises(ValueError, match="contiguous"):
        camg.camg_solve_multi_dev(None, 3, B.t().contiguous().t(), 1e-8, B.clone())   # column-major block
    with pytest.raises(ValueError, match="GPU tensor"):
        camg.camg_solve_multi_dev(None, 3, B, 1e-8, B.clone())
    with pytest.raises(ValueError, match="one b and one x"):
        camg.solve_batch_dev([], [b], [])
    # host blocks handed to the server: shape checked against the system size
    with pytest.raises(ValueError, match="expected"):
        camg._buf_ptr(np.zeros((n, 2)), n + 1, 2)
    with pytest.raises(ValueError, match="expected"):
        camg._buf_ptr(np.zeros((n, 2)), n, 3)
    assert camg._buf_ptr(np.zeros((n, 4))[:, :2], n, 2)[1] == 4   # column slice: row stride 4
