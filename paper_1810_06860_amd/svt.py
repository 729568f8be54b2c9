"""Python face of the library: one object per completion solve.

Every step of the solve runs in the HIP library; this module only converts
arguments (NumPy arrays -> C pointers, dicts -> mc_svt_params) and hands the
current torch HIP stream to the library.
"""

import ctypes as C

import numpy as np

from ._ffi import (MC_EDONE, MC_ENOTCONV, MC_OK, PRECISIONS, PROF_FAMILIES,
                   MCError, Params, ProfEntry, Result, StepInfo, check, lib)

_PARAM_KEYS = [f for f, _ in Params._fields_]


def default_params():
    p = Params()
    lib().mc_svt_default_params(C.byref(p))
    return {k: getattr(p, k) for k in _PARAM_KEYS}


def to_params(d=None):
    p = Params()
    lib().mc_svt_default_params(C.byref(p))
    for k, v in (d or {}).items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k in _PARAM_KEYS:
            setattr(p, k, v)
    return p


def current_stream():
    """The torch HIP stream of the current device, or None (default stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class SVT:
    """Fast SVT solve (Alg. 6) with state resident on the GPU between steps."""

    def __init__(self, m, n, rows, cols, vals, params=None, stream=None,
                 is_csr=False):
        self.m, self.n = int(m), int(n)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        vals = _f64(vals)
        self.nnz = int(vals.size)
        self._prm = to_params(params)
        self._h = C.c_void_p()
        st = stream if stream is not None else current_stream()
        status = lib().mc_svt_init(self.m, self.n, self.nnz,
                                   _ptr(rows, C.c_int64), _ptr(cols, C.c_int32),
                                   _ptr(vals, C.c_double), int(bool(is_csr)),
                                   C.byref(self._prm), st, C.byref(self._h))
        check(status, None)

    @classmethod
    def from_device(cls, m, n, rows, cols, vals, params=None, stream=None,
                    is_csr=False):
        """The same solve set up from device tensors (mc_svt_init_dev): rows
        int64 (COO row ids, or the CSR row pointer with is_csr), cols int32,
        vals float64, all contiguous on the GPU."""
        import torch
        for t, dt in ((rows, torch.int64), (cols, torch.int32), (vals, torch.float64)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise ValueError("rows, cols, vals must be contiguous GPU tensors "
                                 "of int64, int32, float64")
        self = cls.__new__(cls)
        self.m, self.n = int(m), int(n)
        self.nnz = int(vals.numel())
        self._prm = to_params(params)
        self._h = C.c_void_p()
        st = stream if stream is not None else current_stream()
        status = lib().mc_svt_init_dev(self.m, self.n, self.nnz, rows.data_ptr(),
                                       cols.data_ptr(), vals.data_ptr(),
                                       int(bool(is_csr)), C.byref(self._prm), st,
                                       C.byref(self._h))
        check(status, None)
        return self

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if self._h:
            lib().mc_svt_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # -- stepping ---------------------------------------------------------
    def step(self):
        info = StepInfo()
        check(lib().mc_svt_step(self._h, C.byref(info)), self._h)
        return info.as_dict()

    def solve(self):
        res = Result()
        status = lib().mc_svt_solve(self._h, C.byref(res))
        if status not in (MC_OK, MC_ENOTCONV):
            check(status, self._h)
        out = res.as_dict()
        out["status"] = status
        return out

    def result(self):
        res = Result()
        check(lib().mc_svt_get_result(self._h, C.byref(res)), self._h)
        return res.as_dict()

    # -- measurement ------------------------------------------------------
    def profile(self, on=True):
        check(lib().mc_svt_profile(self._h, int(bool(on))), self._h)

    def get_profile(self):
        arr = (ProfEntry * len(PROF_FAMILIES))()
        check(lib().mc_svt_get_profile(self._h, arr, len(PROF_FAMILIES)), self._h)
        return {name: dict(launches=arr[j].launches, ms=arr[j].ms,
                           bytes=arr[j].bytes, flops=arr[j].flops)
                for j, name in enumerate(PROF_FAMILIES)}

    # -- outputs ----------------------------------------------------------
    def factors(self):
        """(U, sig, V) with X = U diag(sig) V^T."""
        r = C.c_int32()
        cap = max(1, self.result()["rank"])
        U = np.zeros((self.m, cap))
        V = np.zeros((self.n, cap))
        sig = np.zeros(cap)
        check(lib().mc_svt_get_factors(self._h, _ptr(U, C.c_double),
                                       _ptr(sig, C.c_double), _ptr(V, C.c_double),
                                       cap, cap, cap, C.byref(r)), self._h)
        k = r.value
        return U[:, :k], sig[:k], V[:, :k]

    def observed(self):
        out = np.zeros(self.nnz)
        check(lib().mc_svt_get_observed(self._h, _ptr(out, C.c_double)), self._h)
        return out

    def y(self):
        out = np.zeros(self.nnz)
        check(lib().mc_svt_get_y(self._h, _ptr(out, C.c_double)), self._h)
        return out

    def sigma(self):
        k = C.c_int32()
        cap = max(1, min(self.m, self.n))
        out = np.zeros(cap)
        check(lib().mc_svt_get_sigma(self._h, _ptr(out, C.c_double), cap,
                                     C.byref(k)), self._h)
        return out[:k.value].copy()


def step_many(solves):
    """One step of each solve (mc_svt_step_many); returns (infos, statuses)."""
    n = len(solves)
    hs = (C.c_void_p * n)(*[s.handle for s in solves])
    infos = (StepInfo * n)()
    status = (C.c_int * n)()
    lib().mc_svt_step_many(hs, n, infos, status)
    return [infos[j].as_dict() for j in range(n)], list(status)


def step_group(solves):
    """One step of each solve with their sparse products batched into shared
    launches (mc_svt_step_group); returns (infos, statuses)."""
    n = len(solves)
    hs = (C.c_void_p * n)(*[s.handle for s in solves])
    infos = (StepInfo * n)()
    status = (C.c_int * n)()
    lib().mc_svt_step_group(hs, n, infos, status)
    return [infos[j].as_dict() for j in range(n)], list(status)


def footprint(m, n, nnz, params=None):
    p = to_params(params)
    return int(lib().mc_svt_footprint(m, n, nnz, C.byref(p)))


RSVD_METHODS = {"pi": 4, "bki": 5}


def _coo(rows, cols, vals):
    return (np.ascontiguousarray(rows, dtype=np.int64),
            np.ascontiguousarray(cols, dtype=np.int32), _f64(vals))


def _one_shot(fn, m, n, rows, cols, vals, k, s, p, seed, step, attempt, precision,
              stream):
    rows, cols, vals = _coo(rows, cols, vals)
    U = np.zeros((m, k))
    S = np.zeros(k)
    V = np.zeros((n, k))
    st = stream if stream is not None else current_stream()
    prec = PRECISIONS[precision] if isinstance(precision, str) else precision
    check(fn(m, n, vals.size, _ptr(rows, C.c_int64), _ptr(cols, C.c_int32),
             _ptr(vals, C.c_double), k, s, p, seed, step, attempt, prec, st,
             _ptr(U, C.c_double), _ptr(S, C.c_double), _ptr(V, C.c_double)), None)
    return U, S, V


def rsvd_bki(m, n, rows, cols, vals, k, s, p, seed, step=1, attempt=0,
             precision="fp64", stream=None):
    """Top-k SVD of a sparse matrix by rSVD-BKI on the GPU: (U, S, V)."""
    return _one_shot(lib().mc_rsvd_bki, m, n, rows, cols, vals, k, s, p, seed, step,
                     attempt, precision, stream)


def rsvd_pi(m, n, rows, cols, vals, k, s, p, seed, step=1, attempt=0,
            precision="fp64", stream=None):
    """Top-k SVD of a sparse matrix by rSVD-PI on the GPU: (U, S, V)."""
    return _one_shot(lib().mc_rsvd_pi, m, n, rows, cols, vals, k, s, p, seed, step,
                     attempt, precision, stream)


class RSVD:
    """A sparse matrix kept on the device for repeated truncated SVDs
    (mc_rsvd_init / mc_rsvd_run)."""

    def __init__(self, m, n, rows, cols, vals, s=10, precision="fp64", seed=1,
                 stream=None):
        rows, cols, vals = _coo(rows, cols, vals)
        self.m, self.n, self.s = m, n, s
        self._stream = stream if stream is not None else current_stream()
        prec = PRECISIONS[precision] if isinstance(precision, str) else precision
        h = C.c_void_p()
        st = lib().mc_rsvd_init(m, n, vals.size, _ptr(rows, C.c_int64),
                                _ptr(cols, C.c_int32), _ptr(vals, C.c_double), s, prec,
                                seed, self._stream, C.byref(h))
        self.handle = None
        self._check(st)
        self.handle = h

    def _check(self, status):
        if status != MC_OK:
            msg = lib().mc_rsvd_last_error(self.handle)
            raise MCError(status, msg.decode() if msg else "")

    def run(self, method, k, p, step=1, attempt=0, factors=True):
        """(U, S, V) of one call; U and V are None when factors is False."""
        meth = RSVD_METHODS[method] if isinstance(method, str) else method
        S = np.zeros(k)
        U = np.zeros((self.m, k)) if factors else None
        V = np.zeros((self.n, k)) if factors else None
        nul = C.POINTER(C.c_double)()
        self._check(lib().mc_rsvd_run(
            self.handle, meth, k, p, step, attempt,
            _ptr(U, C.c_double) if factors else nul, _ptr(S, C.c_double),
            _ptr(V, C.c_double) if factors else nul))
        return U, S, V

    def profile(self, on=True):
        self._check(lib().mc_rsvd_profile(self.handle, int(bool(on))))

    def get_profile(self):
        arr = (ProfEntry * len(PROF_FAMILIES))()
        self._check(lib().mc_rsvd_get_profile(self.handle, arr, len(PROF_FAMILIES)))
        return {name: dict(launches=arr[j].launches, ms=arr[j].ms,
                           bytes=arr[j].bytes, flops=arr[j].flops)
                for j, name in enumerate(PROF_FAMILIES)}

    def close(self):
        if self.handle:
            lib().mc_rsvd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
