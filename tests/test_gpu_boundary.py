"""The boundary's device-side forms: set-up from device arrays (COO and CSR)
against set-up from host arrays, its error codes, and device memory taken
from torch's caching allocator."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _steps(s, n):
    out = []
    for _ in range(n):
        out.append(s.step())
    return out


@pytest.mark.parametrize("form", ["coo", "csr"])
def test_init_from_device_arrays_equals_host_init(form):
    import torch
    from paper_1810_06860_amd import SVT
    prob = synth.planted(320, 270, 5, 0.35, seed_data=81, seed_phi=181)
    prm = dict(eps=1e-6, i_max=40)
    host = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    # a shuffled COO order, to check that the caller's order is honoured
    perm = np.random.default_rng(3).permutation(prob.nnz)
    rows, cols, vals = prob.rows[perm], prob.cols[perm], prob.vals[perm]
    if form == "coo":
        r_t = torch.as_tensor(rows, dtype=torch.int64, device="cuda")
    else:
        order = np.lexsort((cols, rows))
        rows, cols, vals = rows[order], cols[order], vals[order]
        ptr = np.zeros(prob.m + 1, dtype=np.int64)
        np.add.at(ptr, rows + 1, 1)
        r_t = torch.as_tensor(np.cumsum(ptr), dtype=torch.int64, device="cuda")
    c_t = torch.as_tensor(cols, dtype=torch.int32, device="cuda")
    v_t = torch.as_tensor(vals, dtype=torch.float64, device="cuda")
    dev = SVT.from_device(prob.m, prob.n, r_t, c_t, v_t, prm, is_csr=(form == "csr"))
    assert dev.result()["c"] == host.result()["c"]
    assert _steps(dev, 12) == _steps(host, 12)
    Ua, sa, Va = dev.factors()
    Ub, sb, Vb = host.factors()
    assert np.array_equal(sa, sb) and np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)
    # P_Phi(X) comes back in the device caller's input order
    xd = dev.observed()
    xh = host.observed()
    if form == "coo":
        assert np.array_equal(xd, xh[perm])


@pytest.mark.parametrize("case,status", [("nan", 1), ("range", 3), ("dup", 2),
                                         ("bad_ptr", 1)])
def test_init_from_device_arrays_rejects_bad_input(case, status):
    import torch
    from paper_1810_06860_amd import MCError, SVT
    rows = np.array([0, 1, 2, 2], np.int64)
    cols = np.array([0, 1, 0, 2], np.int32)
    vals = np.array([1.0, 2.0, 3.0, 4.0])
    is_csr = False
    if case == "nan":
        vals[2] = np.nan
    elif case == "range":
        cols[1] = 7
    elif case == "dup":
        cols[3] = 0
    else:
        rows = np.array([0, 1, 3, 2], np.int64)           # decreasing pointer
        is_csr = True
    t = lambda a, dt: torch.as_tensor(a, dtype=dt, device="cuda")
    with pytest.raises(MCError) as e:
        SVT.from_device(3, 3, t(rows, torch.int64), t(cols, torch.int32),
                        t(vals, torch.float64), dict(i_max=5), is_csr=is_csr)
    assert e.value.status == status


def test_device_memory_comes_from_torch_allocator():
    import torch
    from paper_1810_06860_amd import SVT
    prob = synth.planted(900, 800, 6, 0.3, seed_data=91, seed_phi=191)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    s = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, dict(i_max=10))
    s.step()
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - before
    # at least M_Phi, the FP64 master iterate and its CSC copy
    assert held >= 3 * 8 * prob.nnz
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
