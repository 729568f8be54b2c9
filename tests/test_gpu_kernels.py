"""GPU parity of each kernel family against the oracle or a plain definition.

Sizes span several tiles and ragged tails; seeds are fixed.
"""

import numpy as np
import pytest
import scipy.sparse

import synth
from oracle import canonical_csr, gaussian_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_1810_06860_amd import kernels
    return kernels


def _coo(m, n, K_, seed, zipf=False):
    if zipf:
        p = synth.ratings(m, n, K_, 3, seed_data=seed)
        return p.rows, p.cols
    cells = synth.sample_cells(m, n, K_, seed)
    return synth.cells_to_coo(cells, n)


@pytest.mark.parametrize("rows,cols", [(1, 1), (7, 5), (1000, 21), (333, 111)])
def test_gaussian_matches_oracle_stream(K, rows, cols):
    g = K.gaussian(rows, cols, seed=12345, step=3, attempt=1)
    want = gaussian_block(rows, cols, 12345, 3, 1)
    # same counter stream; libm differences only in the last bits
    np.testing.assert_allclose(g, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("m,n,K_,zipf", [(40, 30, 200, False), (1, 50, 20, False),
                                         (60, 1, 10, False), (500, 500, 50000, False),
                                         (3000, 400, 60000, True)])
def test_layout_bit_exact(K, m, n, K_, zipf):
    rows, cols = _coo(m, n, K_, 17, zipf)
    rng = np.random.default_rng(5)
    perm = rng.permutation(rows.size)                # arbitrary input order
    rows, cols = rows[perm], cols[perm]
    got = K.layout(m, n, rows, cols)
    want = canonical_csr(m, n, rows, cols)
    for key in ("row_ptr", "col_idx", "order", "col_ptr", "row_idx", "perm"):
        assert np.array_equal(got[key], want[key]), key


def test_layout_rejects_duplicates_and_range(K):
    from paper_1810_06860_amd import MCError
    from paper_1810_06860_amd._ffi import MC_EDUP, MC_ERANGE
    with pytest.raises(MCError) as e:
        K.layout(4, 4, np.array([0, 1, 1]), np.array([0, 2, 2]))
    assert e.value.status == MC_EDUP
    with pytest.raises(MCError) as e:
        K.layout(4, 4, np.array([0, 4]), np.array([0, 0]))
    assert e.value.status == MC_ERANGE


@pytest.mark.parametrize("b", [1, 5, 16, 21, 24, 33, 40, 48, 52, 64, 70, 72, 80, 90, 97, 110, 112, 113, 128, 200, 300,
                               330, 400, 448, 520, 1100])
@pytest.mark.parametrize("transpose", [False, True])
def test_spmm_fp64(K, b, transpose):
    m, n = 700, 530
    rows, cols = _coo(m, n, 25000, 3)
    rng = np.random.default_rng(b)
    vals = rng.standard_normal(rows.size)
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(m, n))
    X = rng.standard_normal(((m if transpose else n), b))
    got = K.spmm(m, n, rows, cols, vals, X, transpose=transpose)
    want = (A.T @ X) if transpose else (A @ X)
    scale = (abs(A.T) if transpose else abs(A)) @ np.abs(X) + 1e-300
    assert np.max(np.abs(got - want) / scale) < 1e-14


@pytest.mark.parametrize("transpose", [False, True])
def test_spmm_long_rows_are_split(K, transpose):
    # Zipf rows and columns: some exceed the segment cap and go through the
    # partial-row fix-up path
    p = synth.ratings(4000, 1500, 300_000, 3, seed_data=8)
    rng = np.random.default_rng(1)
    vals = rng.standard_normal(p.nnz)
    A = scipy.sparse.csr_matrix((vals, (p.rows, p.cols)), shape=(p.m, p.n))
    b = 40
    X = rng.standard_normal(((p.m if transpose else p.n), b))
    got = K.spmm(p.m, p.n, p.rows, p.cols, vals, X, transpose=transpose)
    want = (A.T @ X) if transpose else (A @ X)
    scale = (abs(A.T) if transpose else abs(A)) @ np.abs(X) + 1e-300
    assert np.max(np.abs(got - want) / scale) < 1e-14


def test_spmm_fp32_error_bound(K):
    m, n, b = 600, 450, 24
    rows, cols = _coo(m, n, 30000, 9)
    rng = np.random.default_rng(2)
    vals = rng.standard_normal(rows.size)
    X = rng.standard_normal((n, b))
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(m, n))
    got = K.spmm(m, n, rows, cols, vals, X, precision="fp32")
    want = A @ X
    scale = abs(A) @ np.abs(X)
    nz = np.diff(A.indptr).max()
    u = 2.0 ** -24
    assert np.max(np.abs(got - want) / scale) < (nz + 2) * u * 1.01


@pytest.mark.parametrize("N,p,q,sym", [(1000, 21, 21, 1), (5000, 84, 84, 1),
                                       (777, 63, 21, 0), (33, 5, 7, 0),
                                       (20000, 330, 330, 1), (1, 3, 3, 1),
                                       (16, 64, 64, 1), (4099, 129, 17, 0),
                                       (70001, 81, 81, 1), (3001, 200, 65, 0),
                                       # the row-streaming form (one output block,
                                       # N >= 4096): each tile count of both kinds
                                       (5000, 3, 3, 1), (8192, 17, 17, 1), (4096, 40, 40, 1),
                                       (6000, 64, 64, 1), (140000, 75, 75, 1),
                                       (6001, 112, 112, 1), (4096, 16, 16, 0),
                                       (8192, 33, 17, 0), (9000, 48, 40, 0),
                                       (12345, 64, 50, 0), (9000, 75, 80, 0)])
def test_gram_fp64(K, N, p, q, sym):
    rng = np.random.default_rng(N + p)
    A = rng.standard_normal((N, p))
    B = None if sym else rng.standard_normal((N, q))
    got = K.gram(A, B)
    want = A.T @ (A if sym else B)
    scale = np.abs(A).T @ np.abs(A if sym else B)
    assert np.max(np.abs(got - want) / scale) < 1e-14
    if sym:
        assert np.array_equal(got, got.T)


@pytest.mark.parametrize("N,p,q,sym", [(1000, 21, 21, 1), (4099, 129, 17, 0),
                                       (70001, 81, 81, 1), (10700, 400, 400, 1),
                                       (9000, 75, 60, 0), (6001, 112, 112, 1)])
def test_gram_fp32(K, N, p, q, sym):
    # FP32 products accumulated in FP32 within a row split, splits summed in
    # FP64: error within N u32 of sum |a_i||b_j| (a loose form of the
    # recursive-summation bound)
    rng = np.random.default_rng(N + p + 1)
    A = rng.standard_normal((N, p)).astype(np.float32).astype(np.float64)
    B = None if sym else rng.standard_normal((N, q)).astype(np.float32).astype(np.float64)
    got = K.gram(A, B, precision="fp32")
    want = A.T @ (A if sym else B)
    scale = np.abs(A).T @ np.abs(A if sym else B)
    assert np.max(np.abs(got - want) / scale) < N * 2.0 ** -24
    if sym:
        assert np.array_equal(got, got.T)


@pytest.mark.parametrize("N,p,q,sym", [(4096, 16, 16, 1), (9001, 75, 75, 1),
                                       (140000, 48, 48, 1), (6001, 112, 112, 1),
                                       (8193, 64, 33, 0), (9000, 80, 75, 0)])
def test_gram_bf16(K, N, p, q, sym):
    # the BF16 matrix-core Gram: operands rounded to BF16 (exact products in
    # FP32), FP32 sums within a wavefront's rows, FP64 across workgroups;
    # against the FP64 product of the BF16-rounded operands
    rng = np.random.default_rng(N + p + 2)
    A = rng.standard_normal((N, p))
    B = None if sym else rng.standard_normal((N, q))

    def bf16(x):
        u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
        u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
        return u.astype(np.uint32).view(np.float32).astype(np.float64)

    got = K.gram(A, B, precision="bf16")
    Ab = bf16(A)
    Bb = Ab if sym else bf16(B)
    want = Ab.T @ Bb
    scale = np.abs(Ab).T @ np.abs(Bb)
    assert np.max(np.abs(got - want) / scale) < N * 2.0 ** -24
    # and it differs from the FP32 Gram by the BF16 rounding of the operands
    assert np.max(np.abs(got - A.T @ (A if sym else B)) / scale) > 1e-6
    if sym:
        assert np.array_equal(got, got.T)


@pytest.mark.parametrize("N,p,q", [(1, 1, 1), (63, 5, 7), (1000, 21, 21), (4097, 33, 81),
                                   (70001, 324, 81), (3000, 100, 129), (2000, 81, 300),
                                   (500, 17, 16), (777, 64, 48)])
def test_panel_matches_fp64_product(K, N, p, q):
    # C = beta C0 + alpha X W diag(s): FP64 accumulation, error within the
    # dot-product bound p u |X| |W|
    rng = np.random.default_rng(N + p + q)
    X = rng.standard_normal((N, p))
    W = rng.standard_normal((p, q))
    s = rng.uniform(0.5, 2.0, q)
    C0 = rng.standard_normal((N, q))
    got = K.panel(X, W, alpha=-0.75, colscale=s, beta=1.5, C0=C0)
    want = 1.5 * C0 + (-0.75 * (X @ W)) * s
    scale = 1.5 * np.abs(C0) + 0.75 * (np.abs(X) @ np.abs(W)) * s
    assert np.max(np.abs(got - want) / scale) < (p + 4) * 2.0 ** -53
    plain = K.panel(X, W)
    assert np.max(np.abs(plain - X @ W) / (np.abs(X) @ np.abs(W))) < (p + 2) * 2.0 ** -53
    # FP32 input rounding: the same product of the rounded X
    Xf = X.astype(np.float32).astype(np.float64)
    got32 = K.panel(X, W, precision="fp32")
    assert np.max(np.abs(got32 - Xf @ W) / (np.abs(Xf) @ np.abs(W))) < (p + 2) * 2.0 ** -53


@pytest.mark.parametrize("N,b,kappa", [(2000, 21, 1e2), (5000, 64, 1e5),
                                       (3000, 110, 1e3), (500, 7, 1e9),
                                       (4000, 128, 1e4), (2000, 140, 1e2)])
def test_cholqr2_orthonormal_same_range(K, N, b, kappa):
    rng = np.random.default_rng(b)
    U, _ = np.linalg.qr(rng.standard_normal((N, b)))
    V, _ = np.linalg.qr(rng.standard_normal((b, b)))
    H = (U * np.logspace(0, -np.log10(kappa), b)) @ V.T
    Q = K.cholqr2(H)
    assert np.linalg.norm(Q.T @ Q - np.eye(b)) < 1e-12
    Qr, _ = np.linalg.qr(H)
    assert np.linalg.norm(Q @ (Q.T @ Qr) - Qr) < 1e-8 * max(1.0, kappa * 1e-8)


@pytest.mark.parametrize("L,k", [(1, 1), (2, 2), (5, 3), (9, 9), (13, 5), (16, 16),
                                 (17, 8), (21, 5), (32, 32), (64, 64), (84, 11),
                                 (130, 40), (150, 20), (330, 110)])
def test_syev_matches_eigh(K, L, k):
    rng = np.random.default_rng(L)
    A = rng.standard_normal((4 * L, L)) * np.logspace(0, -3, L)
    G = A.T @ A
    ev, W, sweeps = K.syev(G, k)
    want, Vw = np.linalg.eigh(G)
    want = want[::-1][:k]
    assert np.allclose(ev, want, rtol=1e-12, atol=1e-14 * want[0])
    # eigenvectors: G W = W diag(ev), orthonormal columns
    assert np.linalg.norm(G @ W - W * ev) < 1e-12 * want[0] * np.sqrt(k)
    # rounding of ~L rotations per vector entry, per sweep
    assert np.linalg.norm(W.T @ W - np.eye(k)) < 2e-14 * L
    assert sweeps < 30


@pytest.mark.parametrize("L,k", [(142, 20), (143, 7), (200, 50), (480, 100),
                                 (600, 140), (900, 90), (1024, 60)])
def test_syev_large_multi_launch_path(K, L, k):
    # beyond one workgroup's LDS: one launch per Householder step over many
    # workgroups (a single step and its pending update at L = 142, 143), then
    # the trailing block in LDS
    rng = np.random.default_rng(L + 7)
    A = rng.standard_normal((3 * L, L)) * np.logspace(0, -4, L)
    A[:, 0] *= 50.0
    G = A.T @ A
    ev, W, sweeps = K.syev(G, k)
    want = np.linalg.eigh(G)[0][::-1][:k]
    assert np.allclose(ev, want, rtol=1e-12, atol=1e-14 * want[0])
    assert np.linalg.norm(G @ W - W * ev) < 1e-12 * want[0] * np.sqrt(k)
    assert np.linalg.norm(W.T @ W - np.eye(k)) < 2e-14 * L


def test_syev_large_clustered(K):
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((220, 220)))
    lam = np.concatenate([[9.0] * 4, [4.0] * 3, np.linspace(2.0, 0.1, 213)])
    G = (Q * lam) @ Q.T
    G = 0.5 * (G + G.T)
    ev, W, _ = K.syev(G, 10)
    np.testing.assert_allclose(ev[:7], [9.0] * 4 + [4.0] * 3, rtol=1e-12)
    assert np.linalg.norm(G @ W - W * ev) < 1e-12 * 9.0 * np.sqrt(10)
    assert np.linalg.norm(W.T @ W - np.eye(10)) < 2e-14 * 220


def test_syev_tiny_repeated_and_graded(K):
    # the one-wavefront Jacobi path (L <= 16): repeated eigenvalues, a graded
    # spectrum over 12 orders of magnitude, and a diagonal input
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    lam = np.array([5.0, 5.0, 5.0, 2.0, 2.0] + list(np.logspace(0, -12, 7)))
    G = (Q * lam) @ Q.T
    G = 0.5 * (G + G.T)
    ev, W, _ = K.syev(G, 6)
    np.testing.assert_allclose(ev[:5], [5.0, 5.0, 5.0, 2.0, 2.0], rtol=1e-13)
    assert np.linalg.norm(G @ W - W * ev) < 1e-13 * 5.0 * np.sqrt(6)
    assert np.linalg.norm(W.T @ W - np.eye(6)) < 1e-13
    D = np.diag([3.0, 1.0, 4.0, 1.5, 9.0, 2.6, 5.0])
    ev2, W2, _ = K.syev(D, 7)
    np.testing.assert_array_equal(ev2, [9.0, 5.0, 4.0, 3.0, 2.6, 1.5, 1.0])
    np.testing.assert_array_equal(np.abs(W2), np.eye(7)[:, [4, 6, 2, 0, 5, 3, 1]])


def test_syev_large_diagonal_and_rank_one(K):
    # the multi-launch path on inputs whose reflectors vanish (a diagonal
    # matrix) or whose spectrum is one value and a zero cluster (all ones)
    L = 300
    G = np.diag(np.arange(L, 0, -1.0))
    ev, W, _ = K.syev(G, 50)
    np.testing.assert_allclose(ev, np.arange(L, L - 50, -1.0), rtol=1e-14)
    np.testing.assert_allclose(np.abs(W), np.eye(L)[:, :50], atol=1e-13)
    G2 = np.ones((L, L))
    ev2, W2, _ = K.syev(G2, 4)
    np.testing.assert_allclose(ev2, [float(L), 0.0, 0.0, 0.0], atol=1e-11)
    np.testing.assert_allclose(np.abs(W2[:, 0]), np.full(L, L ** -0.5), rtol=1e-12)
    assert np.linalg.norm(W2.T @ W2 - np.eye(4)) < 2e-14 * L


def test_syev_degenerate_and_diagonal(K):
    G = np.diag(np.arange(40, 0, -1.0))
    ev, W, _ = K.syev(G, 10)
    assert np.array_equal(ev, np.arange(40, 30, -1.0))
    G2 = np.ones((20, 20))
    ev2, _, _ = K.syev(G2, 3)
    assert np.allclose(ev2, [20.0, 0.0, 0.0], atol=1e-12)


@pytest.mark.parametrize("r", [0, 1, 10, 37])
def test_sddmm_brute_force(K, r):
    m, n = 130, 90
    rows, cols = _coo(m, n, 3000, 4)
    rng = np.random.default_rng(r + 1)
    mv = rng.standard_normal(rows.size)
    y = rng.standard_normal(rows.size)
    U = rng.standard_normal((m, r))
    V = rng.standard_normal((n, r))
    sig = rng.random(r) + 0.5
    delta = 1.7
    x, ynew, ss = K.sddmm(m, n, rows, cols, mv, y, U, sig, V, delta)
    X = (U * sig) @ V.T
    want_x = X[rows, cols]
    np.testing.assert_allclose(x, want_x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ynew, y + delta * (mv - want_x), rtol=1e-13, atol=1e-13)
    assert ss == pytest.approx(np.sum((mv - want_x) ** 2), rel=1e-12)


@pytest.mark.parametrize("transpose", [False, True])
def test_spmm_empty_rows_and_columns(K, transpose):
    # rows 0..99 and columns 0..49 hold no entries; a single-entry row and a
    # single-entry column; outputs of empty rows must be exactly zero
    m, n = 400, 300
    rows, cols = _coo(m - 100, n - 50, 9000, 21)
    rows = rows + 100
    cols = cols + 50
    rows = np.concatenate([rows, [5]])
    cols = np.concatenate([cols, [7]])
    rng = np.random.default_rng(4)
    vals = rng.standard_normal(rows.size)
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(m, n))
    for b in (3, 37):
        X = rng.standard_normal(((m if transpose else n), b))
        got = K.spmm(m, n, rows, cols, vals, X, transpose=transpose)
        want = (A.T @ X) if transpose else (A @ X)
        scale = (abs(A.T) if transpose else abs(A)) @ np.abs(X) + 1e-300
        assert np.max(np.abs(got - want) / scale) < 1e-14
        empty = np.flatnonzero(np.asarray(abs(A.T if transpose else A).sum(axis=1)).ravel() == 0)
        assert empty.size > 0 and np.all(got[empty] == 0.0)


@pytest.mark.parametrize("m,n,b,precision", [
    (20000, 4000, 40, "fp64"), (20000, 4000, 55, "fp32"), (20000, 4000, 90, "fp32"),
    (20000, 4000, 300, "fp64"),
    (20000, 600, 40, "fp64"), (20000, 600, 300, "fp64")])
@pytest.mark.parametrize("transpose", [False, True])
def test_spmm_banded_large_panel(K, m, n, b, precision, transpose):
    # a gathered dimension of 20,000 rows and a panel above 2 MiB run the
    # banded schedule: rows of at least max(256, 4 cap) entries (256 at this
    # nnz) are split at eight equal ranges of the gathered index (one per XCD)
    # and summed by the fix-up.  Power-law rows: some short and whole, some
    # split; the wide cases have over a quarter of their entries in split rows.
    if not transpose:
        m, n = n, m
    p = synth.ratings(m, n, 400_000, 3, seed_data=31)
    rng = np.random.default_rng(b)
    vals = rng.standard_normal(p.nnz)
    A = scipy.sparse.csr_matrix((vals, (p.rows, p.cols)), shape=(m, n))
    Ao = A.T.tocsr() if transpose else A
    X = rng.standard_normal(((m if transpose else n), b))
    assert X.shape[0] * b * (8 if precision == "fp64" else 4) >= 2 << 20
    got = K.spmm(m, n, p.rows, p.cols, vals, X, transpose=transpose, precision=precision)
    want = Ao @ X
    scale = abs(Ao) @ np.abs(X) + 1e-300
    lens = np.diff(Ao.indptr)
    assert lens.max() >= 1024 and (lens < 256).any()
    if precision == "fp64":
        assert np.max(np.abs(got - want) / scale) < 1e-14
    else:
        u = 2.0 ** -24
        assert np.max(np.abs(got - want) / scale) < (lens.max() + 2) * u * 1.01
    empty = np.flatnonzero(lens == 0)
    assert np.all(got[empty] == 0.0)
