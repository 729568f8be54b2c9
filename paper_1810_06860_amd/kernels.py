"""Python wrappers of the kernel-level entry points (include/mcsvt_kernels.h).

Each call runs one kernel family of the SVT step on the GPU with host arrays
in and out; used to check and time the building blocks one by one.
"""

import ctypes as C

import numpy as np

from ._ffi import PRECISIONS, check, lib
from .svt import current_stream


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def gaussian(rows, cols, seed, step, attempt):
    out = np.zeros((rows, cols))
    check(lib().mc_k_gaussian(rows, cols, seed, step, attempt, current_stream(),
                              _p(out, C.c_double)))
    return out


def layout(m, n, rows, cols):
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    nnz = rows.size
    out = dict(row_ptr=np.zeros(m + 1, np.int32), col_idx=np.zeros(nnz, np.int32),
               order=np.zeros(nnz, np.int32), col_ptr=np.zeros(n + 1, np.int32),
               row_idx=np.zeros(nnz, np.int32), perm=np.zeros(nnz, np.int32))
    check(lib().mc_k_layout(m, n, nnz, _p(rows, C.c_int64), _p(cols, C.c_int32),
                            current_stream(),
                            *[_p(out[k], C.c_int32) for k in
                              ("row_ptr", "col_idx", "order", "col_ptr",
                               "row_idx", "perm")]))
    return out


def spmm(m, n, rows, cols, vals, X, transpose=False, precision="fp64"):
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    b = X.shape[1]
    out = np.zeros((n if transpose else m, b))
    check(lib().mc_k_spmm(m, n, vals.size, _p(rows, C.c_int64),
                          _p(cols, C.c_int32), _p(vals, C.c_double),
                          int(transpose), b, _p(X, C.c_double), _prec(precision),
                          current_stream(), _p(out, C.c_double)))
    return out


def band_schedule(ptr, idx, gathered, cap, bands=8):
    """Banded SpMM schedule of a host CSR-like structure (host code only).

    Returns (segs, fix, nslot): segs (nseg x 4: row, begin, end, slot) in
    launch order, fix (nfix x 4: row, first slot, count, 0).
    """
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    rows = ptr.size - 1
    nseg, nfix, nslot = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    st = lib().mc_k_band_schedule(rows, _p(ptr, C.c_int32), _p(idx, C.c_int32),
                                  gathered, cap, bands, None, C.byref(nseg), None,
                                  C.byref(nfix), C.byref(nslot))
    from ._ffi import MC_ERANGE
    if st != MC_ERANGE:
        check(st)
    segs = np.zeros((max(nseg.value, 1), 4), np.int32)
    fix = np.zeros((max(nfix.value, 1), 4), np.int32)
    check(lib().mc_k_band_schedule(rows, _p(ptr, C.c_int32), _p(idx, C.c_int32),
                                   gathered, cap, bands, _p(segs, C.c_int32),
                                   C.byref(nseg), _p(fix, C.c_int32), C.byref(nfix),
                                   C.byref(nslot)))
    return segs[:nseg.value], fix[:nfix.value], nslot.value


def gram(A, B=None, precision="fp64"):
    A = np.ascontiguousarray(A, dtype=np.float64)
    sym = B is None
    Bc = A if sym else np.ascontiguousarray(B, dtype=np.float64)
    N, p = A.shape
    q = Bc.shape[1]
    out = np.zeros((p, q))
    check(lib().mc_k_gram(N, p, q, _p(A, C.c_double), _p(Bc, C.c_double),
                          int(sym), _prec(precision), current_stream(),
                          _p(out, C.c_double)))
    return out


def gram_noalloc(A, B=None, out=None):
    """C = A^T B on device tensors (FP64, row-major, contiguous rows) through
    the allocation-free entry point; out (p x q) is a caller-owned device
    tensor, allocated here when not given.  Enqueued on the current stream."""
    import torch
    sym = B is None
    N, p = A.shape
    q = p if sym else B.shape[1]
    if out is None:
        out = torch.empty((p, q), dtype=torch.float64, device=A.device)
    for t in (A, out) + (() if sym else (B,)):
        if t.dtype != torch.float64 or not t.is_cuda or t.stride(1) != 1:
            raise ValueError("FP64 device tensors with contiguous rows expected")
    check(lib().mc_k_gram_noalloc(N, p, q, A.data_ptr(),
                                  A.stride(0), None if sym else B.data_ptr(),
                                  A.stride(0) if sym else B.stride(0), int(sym),
                                  current_stream(), out.data_ptr(), out.stride(0)))
    return out


def panel(X, W, alpha=1.0, colscale=None, beta=0.0, C0=None, precision="fp64"):
    X = np.ascontiguousarray(X, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    N, p = X.shape
    q = W.shape[1]
    s = None if colscale is None else np.ascontiguousarray(colscale, dtype=np.float64)
    c0 = None if C0 is None else np.ascontiguousarray(C0, dtype=np.float64)
    out = np.zeros((N, q))
    check(lib().mc_k_panel(N, p, q, _p(X, C.c_double), _p(W, C.c_double),
                           float(alpha), None if s is None else _p(s, C.c_double),
                           float(beta), None if c0 is None else _p(c0, C.c_double),
                           _prec(precision), current_stream(), _p(out, C.c_double)))
    return out


def cholqr2(H):
    H = np.ascontiguousarray(H, dtype=np.float64)
    Q = np.zeros_like(H)
    check(lib().mc_k_cholqr2(H.shape[0], H.shape[1], _p(H, C.c_double),
                             current_stream(), _p(Q, C.c_double)))
    return Q


def syev(G, k):
    G = np.ascontiguousarray(G, dtype=np.float64)
    L = G.shape[0]
    ev = np.zeros(k)
    W = np.zeros((L, k))
    sweeps = C.c_int32()
    check(lib().mc_k_syev(L, _p(G, C.c_double), k, current_stream(),
                          _p(ev, C.c_double), _p(W, C.c_double), C.byref(sweeps)))
    return ev, W, sweeps.value


def sddmm(m, n, rows, cols, mvals, y, U, sig, V, delta):
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    mvals = np.ascontiguousarray(mvals, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    r = int(np.size(sig))
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(m, r)
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(n, r)
    sig = np.ascontiguousarray(sig, dtype=np.float64)
    x = np.zeros(mvals.size)
    ynew = np.zeros(mvals.size)
    ss = np.zeros(1)
    check(lib().mc_k_sddmm(m, n, mvals.size, _p(rows, C.c_int64),
                           _p(cols, C.c_int32), _p(mvals, C.c_double),
                           _p(y, C.c_double), r, _p(U, C.c_double),
                           _p(sig, C.c_double), _p(V, C.c_double), delta,
                           current_stream(), _p(x, C.c_double),
                           _p(ynew, C.c_double), _p(ss, C.c_double)))
    return x, ynew, float(ss[0])
