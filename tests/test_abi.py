"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects bad input before touching the GPU."""

import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1810_06860_amd", "libmcsvt.so")


def declared_functions():
    names = set()
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(mc_\w+)\s*\(", text):
            start = text.rfind("\n", 0, m.start()) + 1
            line = text[start:m.start()]
            if "typedef" in line or "(*" in text[m.start() - 2:m.start() + 2]:
                continue
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built: run python -m paper_1810_06860_amd.build")
    from paper_1810_06860_amd import _ffi
    return _ffi.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1810_06860_amd import _ffi
    assert declared_functions() <= set(_ffi._SIGNATURES)


def test_default_params_and_version(lib):
    from paper_1810_06860_amd import default_params
    assert lib.mc_abi_version() == 2
    p = default_params()
    assert p["l"] == 5 and p["s"] == 10 and p["p_init"] == 3
    assert p["q_reuse"] == 10 and p["eps"] == 1e-4 and p["recycle"] == 0


def test_footprint_grows_with_size(lib):
    from paper_1810_06860_amd import footprint
    a = footprint(500, 500, 50_000)
    b = footprint(70_000, 10_700, 10_000_000, dict(k_max=100))
    assert 0 < a < b
    assert footprint(0, 5, 5) == 0


def test_footprint_prices_the_rank_cap(lib):
    # k_max = 0 leaves the rank search bounded by min(m, n) alone, and the
    # footprint prices exactly that bound
    from paper_1810_06860_amd import footprint
    full = footprint(600, 400, 40_000)
    assert full == footprint(600, 400, 40_000, dict(k_max=400))
    assert footprint(600, 400, 40_000, dict(k_max=50)) < full
    assert footprint(600, 400, 40_000, dict(k_max=50, p_max=4)) < \
        footprint(600, 400, 40_000, dict(k_max=50))


def _init(m, n, rows, cols, vals, params=None):
    from paper_1810_06860_amd import SVT
    return SVT(m, n, rows, cols, vals, params)


@pytest.mark.parametrize("case", ["nnz0", "m0", "nan", "too_many", "bad_p"])
def test_init_rejects_bad_input_on_host(lib, case):
    from paper_1810_06860_amd import MCError
    from paper_1810_06860_amd._ffi import MC_EDUP, MC_EINVAL
    rows = np.array([0, 1])
    cols = np.array([0, 1])
    vals = np.array([1.0, 2.0])
    want = MC_EINVAL
    kw = {}
    if case == "nnz0":
        rows, cols, vals = rows[:0], cols[:0], vals[:0]
        args = (3, 3)
    elif case == "m0":
        args = (0, 3)
    elif case == "nan":
        vals = np.array([1.0, np.nan])
        args = (3, 3)
    elif case == "too_many":
        rows = np.zeros(5, dtype=np.int64)
        cols = np.zeros(5, dtype=np.int32)
        vals = np.ones(5)
        args = (1, 2)
        want = MC_EDUP
    else:
        # parameters are validated before the first device call
        args = (3, 3)
        kw = dict(params=dict(p_min=4, p_init=3, p_max=8))
    with pytest.raises(MCError) as ei:
        _init(*args, rows, cols, vals, **kw)
    assert ei.value.status == want
    assert lib.mc_svt_last_error(None)


def test_rsvd_rejects_oversized_krylov_space(lib):
    from paper_1810_06860_amd import MCError, rsvd_bki
    rows = np.arange(10)
    cols = np.arange(10)
    with pytest.raises(MCError):
        rsvd_bki(10, 10, rows, cols, np.ones(10), k=5, s=5, p=1, seed=1)


def test_null_handle_calls(lib):
    from paper_1810_06860_amd._ffi import MC_EINVAL, StepInfo
    info = StepInfo()
    assert lib.mc_svt_step(None, C.byref(info)) == MC_EINVAL
    assert lib.mc_svt_destroy(None) == 0


def test_rsvd_entry_points_validate_before_the_device(lib):
    from paper_1810_06860_amd import MCError, RSVD, rsvd_pi
    from paper_1810_06860_amd._ffi import MC_EINVAL
    rows = np.arange(10)
    cols = np.arange(10)
    with pytest.raises(MCError) as ei:            # k + s > min(m, n)
        rsvd_pi(10, 10, rows, cols, np.ones(10), k=6, s=5, p=0, seed=1)
    assert ei.value.status == MC_EINVAL
    with pytest.raises(MCError) as ei:            # non-finite value
        RSVD(10, 10, rows, cols, np.r_[np.ones(9), np.nan])
    assert ei.value.status == MC_EINVAL
    with pytest.raises(MCError) as ei:            # unknown precision
        RSVD(10, 10, rows, cols, np.ones(10), precision=7)
    assert ei.value.status == MC_EINVAL
    S = np.zeros(2)
    assert lib.mc_rsvd_run(None, 4, 2, 0, 1, 0, None,
                           S.ctypes.data_as(C.POINTER(C.c_double)), None) == MC_EINVAL
    assert lib.mc_rsvd_destroy(None) == 0
    assert lib.mc_rsvd_last_error(None)


def test_headers_compile_as_c_and_link_against_the_library(tmp_path):
    """The public headers are plain C: a C99 program that includes both and
    calls an entry point compiles with -pedantic and links to libmcsvt.so."""
    import shutil
    import subprocess
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(
        '#include "mcsvt.h"\n#include "mcsvt_kernels.h"\n'
        "int main(void) {\n"
        "  mc_svt_params p;\n"
        "  mc_svt_default_params(&p);\n"
        "  mc_rsvd_t h = 0;\n"
        "  (void)h;\n"
        "  return (mc_abi_version() == MCSVT_ABI_VERSION && p.l == 5) ? 0 : 1;\n"
        "}\n")
    exe = tmp_path / "use"
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                    LIB, "-Wl,-rpath," + os.path.dirname(LIB)],
                   check=True, capture_output=True)
    run = subprocess.run([str(exe)], capture_output=True, timeout=60)
    assert run.returncode == 0, run.stderr


@pytest.mark.parametrize("case", ["n0", "sym_pq", "ld", "null_b", "oversize"])
def test_noalloc_gram_validates_before_the_device(lib, case):
    # every rejection happens before the first device call (the pointers are
    # placeholders that are never dereferenced)
    from paper_1810_06860_amd._ffi import MC_EINVAL, MC_ERANGE
    a = 4096
    args = dict(N=8, p=4, q=4, A=a, lda=4, B=a, ldb=4, sym=1, C=a, ldc=4)
    want = MC_EINVAL
    if case == "n0":
        args["N"] = 0
    elif case == "sym_pq":
        args["q"] = 3
    elif case == "ld":
        args["lda"] = 3
    elif case == "null_b":
        args.update(sym=0, B=None)
    else:
        args.update(p=2048, q=2048, lda=2048, ldb=2048, ldc=2048)
        want = MC_ERANGE
    st = lib.mc_k_gram_noalloc(args["N"], args["p"], args["q"], args["A"],
                               args["lda"], args["B"], args["ldb"], args["sym"],
                               None, args["C"], args["ldc"])
    assert st == want
    assert lib.mc_svt_last_error(None)
