"""ctypes view of include/mcsvt.h (argument marshalling only).

The shared library is built in-tree by ``paper_1810_06860_amd.build`` (or
``__graft_entry__.build()``).  There is no fallback: if libmcsvt.so is
missing, ``lib()`` raises.
"""

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmcsvt.so")

MC_OK, MC_EINVAL, MC_EDUP, MC_ERANGE, MC_ENOMEM, MC_EDEVICE = 0, 1, 2, 3, 4, 5
MC_ENUMERIC, MC_EDONE, MC_ENOTCONV = 6, 7, 8
STATUS_NAMES = {0: "MC_OK", 1: "MC_EINVAL", 2: "MC_EDUP", 3: "MC_ERANGE",
                4: "MC_ENOMEM", 5: "MC_EDEVICE", 6: "MC_ENUMERIC",
                7: "MC_EDONE", 8: "MC_ENOTCONV"}
MC_FP64, MC_FP32_EIG64, MC_BF16_EIG64 = 0, 1, 2
PRECISIONS = {"fp64": MC_FP64, "fp32": MC_FP32_EIG64, "bf16": MC_BF16_EIG64}


class Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("delta", C.c_double), ("eps", C.c_double),
                ("ritz_tol", C.c_double), ("c", C.c_double),
                ("i_max", C.c_int32), ("l", C.c_int32), ("s", C.c_int32),
                ("p_init", C.c_int32), ("p_min", C.c_int32),
                ("p_max", C.c_int32), ("adaptive_p", C.c_int32),
                ("i_reuse", C.c_int32), ("q_reuse", C.c_int32),
                ("recycle", C.c_int32), ("k_max", C.c_int32),
                ("precision", C.c_int32), ("use_graphs", C.c_int32),
                ("seed", C.c_uint64)]


class StepInfo(C.Structure):
    _fields_ = [("i", C.c_int32), ("r", C.c_int32), ("k", C.c_int32),
                ("p", C.c_int32), ("fresh", C.c_int32),
                ("recycled", C.c_int32), ("rejected", C.c_int32),
                ("converged", C.c_int32), ("res", C.c_double),
                ("sigma_max", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rank", C.c_int32),
                ("converged", C.c_int32), ("fresh", C.c_int32),
                ("recycled", C.c_int32), ("rejected", C.c_int32),
                ("res", C.c_double), ("c", C.c_double), ("norm2", C.c_double),
                ("mnorm", C.c_double), ("shifts", C.c_int32), ("redone", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ProfEntry(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


PROF_FAMILIES = ["spmm_fwd", "spmm_bwd", "sddmm", "gram", "panel_gemm",
                 "cholesky", "eigensolve", "rng"]

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)

_P = C.POINTER
_SIGNATURES = {
    "mc_abi_version": (C.c_int32, []),
    "mc_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, C.c_void_p]),
    "mc_svt_default_params": (None, [_P(Params)]),
    "mc_svt_footprint": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int64, _P(Params)]),
    "mc_svt_init": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P(C.c_int64),
                              _P(C.c_int32), _P(C.c_double), C.c_int32,
                              _P(Params), C.c_void_p, _P(C.c_void_p)]),
    "mc_svt_init_dev": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_int32,
                                  _P(Params), C.c_void_p, _P(C.c_void_p)]),
    "mc_svt_step": (C.c_int, [C.c_void_p, _P(StepInfo)]),
    "mc_svt_step_many": (C.c_int, [_P(C.c_void_p), C.c_int32, _P(StepInfo),
                                   _P(C.c_int)]),
    "mc_svt_step_group": (C.c_int, [_P(C.c_void_p), C.c_int32, _P(StepInfo),
                                    _P(C.c_int)]),
    "mc_svt_solve": (C.c_int, [C.c_void_p, _P(Result)]),
    "mc_svt_get_result": (C.c_int, [C.c_void_p, _P(Result)]),
    "mc_svt_get_factors": (C.c_int, [C.c_void_p, _P(C.c_double), _P(C.c_double),
                                     _P(C.c_double), C.c_int64, C.c_int64,
                                     C.c_int32, _P(C.c_int32)]),
    "mc_svt_get_observed": (C.c_int, [C.c_void_p, _P(C.c_double)]),
    "mc_svt_get_y": (C.c_int, [C.c_void_p, _P(C.c_double)]),
    "mc_svt_get_sigma": (C.c_int, [C.c_void_p, _P(C.c_double), C.c_int32,
                                   _P(C.c_int32)]),
    "mc_svt_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "mc_svt_get_profile": (C.c_int, [C.c_void_p, _P(ProfEntry), C.c_int32]),
    "mc_svt_destroy": (C.c_int, [C.c_void_p]),
    "mc_svt_last_error": (C.c_char_p, [C.c_void_p]),
    "mc_rsvd_bki": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P(C.c_int64),
                              _P(C.c_int32), _P(C.c_double), C.c_int32,
                              C.c_int32, C.c_int32, C.c_uint64, C.c_uint32,
                              C.c_uint32, C.c_int32, C.c_void_p,
                              _P(C.c_double), _P(C.c_double), _P(C.c_double)]),
    "mc_rsvd_pi": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P(C.c_int64),
                             _P(C.c_int32), _P(C.c_double), C.c_int32,
                             C.c_int32, C.c_int32, C.c_uint64, C.c_uint32,
                             C.c_uint32, C.c_int32, C.c_void_p,
                             _P(C.c_double), _P(C.c_double), _P(C.c_double)]),
    "mc_rsvd_init": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P(C.c_int64),
                               _P(C.c_int32), _P(C.c_double), C.c_int32, C.c_int32,
                               C.c_uint64, C.c_void_p, _P(C.c_void_p)]),
    "mc_rsvd_run": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                              C.c_uint32, C.c_uint32, _P(C.c_double),
                              _P(C.c_double), _P(C.c_double)]),
    "mc_rsvd_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "mc_rsvd_get_profile": (C.c_int, [C.c_void_p, _P(ProfEntry), C.c_int32]),
    "mc_rsvd_destroy": (C.c_int, [C.c_void_p]),
    "mc_rsvd_last_error": (C.c_char_p, [C.c_void_p]),
    # include/mcsvt_kernels.h
    "mc_k_gaussian": (C.c_int, [C.c_int64, C.c_int64, C.c_uint64, C.c_uint32,
                                C.c_uint32, C.c_void_p, _P(C.c_double)]),
    "mc_k_layout": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P(C.c_int64),
                              _P(C.c_int32), C.c_void_p, _P(C.c_int32),
                              _P(C.c_int32), _P(C.c_int32), _P(C.c_int32),
                              _P(C.c_int32), _P(C.c_int32)]),
    "mc_k_band_schedule": (C.c_int, [C.c_int64, _P(C.c_int32), _P(C.c_int32),
                                     C.c_int64, C.c_int32, C.c_int32,
                                     _P(C.c_int32), _P(C.c_int64), _P(C.c_int32),
                                     _P(C.c_int64), _P(C.c_int64)]),
    "mc_k_spmm": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P(C.c_int64),
                            _P(C.c_int32), _P(C.c_double), C.c_int32, C.c_int32,
                            _P(C.c_double), C.c_int32, C.c_void_p,
                            _P(C.c_double)]),
    "mc_k_gram": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, _P(C.c_double),
                            _P(C.c_double), C.c_int32, C.c_int32, C.c_void_p,
                            _P(C.c_double)]),
    "mc_k_gram_noalloc": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_int64]),
    "mc_k_panel": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, _P(C.c_double),
                             _P(C.c_double), C.c_double, _P(C.c_double), C.c_double,
                             _P(C.c_double), C.c_int32, C.c_void_p, _P(C.c_double)]),
    "mc_k_cholqr2": (C.c_int, [C.c_int64, C.c_int32, _P(C.c_double), C.c_void_p,
                               _P(C.c_double)]),
    "mc_k_syev": (C.c_int, [C.c_int32, _P(C.c_double), C.c_int32, C.c_void_p,
                            _P(C.c_double), _P(C.c_double), _P(C.c_int32)]),
    "mc_k_sddmm": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P(C.c_int64),
                             _P(C.c_int32), _P(C.c_double), _P(C.c_double),
                             C.c_int32, _P(C.c_double), _P(C.c_double),
                             _P(C.c_double), C.c_double, C.c_void_p,
                             _P(C.c_double), _P(C.c_double), _P(C.c_double)]),
}

_lib = None
_hooks = None          # the registered allocator callbacks, kept alive


def _use_torch_allocator(handle):
    """Route the library's device allocations through torch's caching
    allocator (mc_set_allocator), so that PyTorch owns the device memory of
    every solve.  Skipped without a visible GPU or with MCSVT_ALLOCATOR=hip."""
    global _hooks
    if os.environ.get("MCSVT_ALLOCATOR", "torch") == "hip":
        return
    try:
        import torch
        if not torch.cuda.is_available():
            return
    except ImportError:
        return

    def alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:
            return None                      # the library reports MC_ENOMEM

    def release(ptr, nbytes, stream, ctx):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    hooks = (ALLOC_FN(alloc), FREE_FN(release))
    if handle.mc_set_allocator(hooks[0], hooks[1], None) == MC_OK:
        _hooks = hooks


class MCError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


def lib():
    """The loaded libmcsvt.so with typed entry points (raises if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_1810_06860_amd.build)")
        # torch carries its own HIP runtime under the same soname; load it
        # first so that libmcsvt binds to that one copy (two runtimes in one
        # process cannot share streams or memory, and the second one fails)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        handle = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _use_torch_allocator(handle)
        _lib = handle
    return _lib


def check(status, handle=None):
    if status != MC_OK:
        msg = lib().mc_svt_last_error(handle)
        raise MCError(status, msg.decode() if msg else "")
    return status
