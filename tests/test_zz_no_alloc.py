"""The allocation-free Gram entry point (mc_k_gram_noalloc) against the
allocating one (mc_k_gram) and the plain product A^T B, through the C ABI on
device tensors: two calls in a row, the second smaller, then a shape whose
partial sums fill the fixed scratch array (fewer row splits than the
allocating path takes)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _alloc_count(torch):
    st = torch.cuda.memory_stats()
    return st.get("allocation.all.allocated", 0), torch.cuda.memory_allocated()


def _check(torch, kernels, A, B, tol):
    dA = torch.from_numpy(A).cuda()
    dB = None if B is None else torch.from_numpy(B).cuda()
    q = A.shape[1] if B is None else B.shape[1]
    out = torch.full((A.shape[1], q), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    before = _alloc_count(torch)
    kernels.gram_noalloc(dA, dB, out=out)
    torch.cuda.synchronize()
    assert _alloc_count(torch) == before, "the allocation-free Gram allocated"
    got = out.cpu().numpy()
    ref = kernels.gram(A, B)                         # allocating entry point
    plain = A.T @ (A if B is None else B)
    scale = np.abs(plain).max()
    print(f"N={A.shape[0]} p={A.shape[1]} q={q}: vs mc_k_gram "
          f"{np.abs(got - ref).max() / scale:.1e}, vs A^T B "
          f"{np.abs(got - plain).max() / scale:.1e}")
    np.testing.assert_allclose(got, ref, rtol=0, atol=tol * scale)
    np.testing.assert_allclose(got, plain, rtol=0, atol=1e-12 * scale)


def test_noalloc_gram_two_calls_second_smaller():
    import torch
    from paper_1810_06860_amd import kernels
    g = np.random.default_rng(31)
    A1 = g.standard_normal((6000, 96))
    _check(torch, kernels, A1, None, 1e-13)                    # symmetric
    A2 = g.standard_normal((2500, 40))
    B2 = g.standard_normal((2500, 24))
    _check(torch, kernels, A2, B2, 1e-13)                      # smaller, cross


def test_noalloc_gram_fills_scratch():
    # p q = 2^18 doubles: the 2^21-double array holds 8 row splits, where the
    # allocating path takes about 100
    import torch
    from paper_1810_06860_amd import kernels
    g = np.random.default_rng(32)
    A = g.standard_normal((50000, 512))
    _check(torch, kernels, A, None, 1e-12)


def test_noalloc_gram_rejects_oversize_without_launch():
    import torch
    from paper_1810_06860_amd import _ffi
    lib = _ffi.lib()
    dA = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    st = lib.mc_k_gram_noalloc(4, 2048, 2048, dA.data_ptr(), 2048, None, 2048, 1,
                               None, dA.data_ptr(), 2048)
    assert st == _ffi.MC_ERANGE
    assert b"16 MiB" in lib.mc_svt_last_error(None)
