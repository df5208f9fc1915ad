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
