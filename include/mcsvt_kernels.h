/*
 * mcsvt_kernels.h -- kernel-level C ABI of libmcsvt (one device kernel
 * family per call, host buffers in and out).
 *
 * These entry points expose the building blocks of one fast-SVT step so that
 * each can be checked and timed on its own.  Each copies its host inputs to
 * the device, runs the same kernels mc_svt_step uses, copies the result back
 * and synchronises the stream.  Matrices are row-major.  Status codes and
 * mc_svt_last_error(NULL) behave as in mcsvt.h.
 */
#ifndef MCSVT_KERNELS_H
#define MCSVT_KERNELS_H

#include <stdint.h>

#include "mcsvt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Gaussian test matrix Omega of rSVD-BKI (Alg. 5): out (rows x cols) from the
 * Philox4x32-10 counter stream keyed by seed, counter (pair, step, attempt),
 * Box-Muller per element pair. */
mc_status mc_k_gaussian(int64_t rows, int64_t cols, uint64_t seed,
                        uint32_t step, uint32_t attempt, void* stream,
                        double* out);

/* Canonical CSR and CSC layout of Phi (Sec. II.C): entries sorted by
 * (row, col) and (col, row).  Outputs: row_ptr (m+1), col_idx (nnz),
 * order (nnz: CSR position -> input position), col_ptr (n+1),
 * row_idx (nnz), perm (nnz: CSC position -> CSR position).
 * Errors: MC_ERANGE, MC_EDUP, MC_EINVAL. */
mc_status mc_k_layout(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                      const int32_t* cols, void* stream, int32_t* row_ptr,
                      int32_t* col_idx, int32_t* order, int32_t* col_ptr,
                      int32_t* row_idx, int32_t* perm);

/* SpMM of the sparse A (COO input) with a dense panel -- the products
 * A Omega, A (A^T H) and A^T Q of the randomized SVDs (Alg. 4, Alg. 5):
 * transpose = 0: out (m x b) = A X with X (n x b); transpose = 1:
 * out (n x b) = A^T X with X (m x b).  precision as mc_precision (FP32 runs A and X in FP32 with FP32
 * accumulation; the result is returned in FP64). */
mc_status mc_k_spmm(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                    const int32_t* cols, const double* vals, int32_t transpose,
                    int32_t b, const double* X, int32_t precision, void* stream,
                    double* out);

/* C (p x q) = A^T B for A (N x p), B (N x q), the Gram matrix of eigSVD
 * (Alg. 3) and of the block orthonormalisation (Lemma 2); sym = 1 requires
 * A == B.  Host buffers; FP64 result in every precision.  MC_FP32_EIG64
 * rounds A and B to FP32 and accumulates in FP32; MC_BF16_EIG64 does the same
 * on the BF16 matrix cores (operands rounded to BF16, FP32 accumulation) for
 * the one-block shapes of a panel of at least 4096 rows (symmetric up to 112
 * wide, cross up to 80 x 80), and falls back to FP32 otherwise. */
mc_status mc_k_gram(int64_t N, int32_t p, int32_t q, const double* A,
                    const double* B, int32_t sym, int32_t precision,
                    void* stream, double* C);

/* Allocation-free form of mc_k_gram, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): C (p x q) = A^T B in FP64 with A (N x p, leading
 * dimension lda), B (N x q, ldb) and C (p x q, ldc) row-major DEVICE arrays
 * owned by the caller; sym = 1 requires p == q and reads A for B (B may then
 * be NULL).  Work is enqueued on `stream` (NULL: the default stream) and not
 * waited for.  The call allocates nothing: the split partial sums live in a
 * file-scope device array of 2^21 doubles (16 MiB) that each GPU the library
 * runs on holds until the process ends; its address is looked up once per
 * device, on the first call with that device current.  Calls on one GPU
 * share that array, so calls that overlap in time on one GPU (other streams,
 * other threads) race and must be serialised by the caller.
 * Errors: MC_EINVAL (sizes < 1, NULL A or C, NULL B without sym, sym with
 * p != q, a leading dimension below its row width), MC_ERANGE (p * q above
 * 2^21), MC_EDEVICE (the array's address could not be found, or a launch
 * failed). */
mc_status mc_k_gram_noalloc(int64_t N, int32_t p, int32_t q, const double* A,
                            int64_t lda, const double* B, int64_t ldb,
                            int32_t sym, void* stream, double* C, int64_t ldc);

/* Panel product C (N x q) = beta C0 + alpha X W diag(colscale) with X (N x p)
 * and W (p x q), all row-major host arrays; colscale (q) and C0 may be NULL
 * (then they are not applied / beta must be 0).  This is the product behind
 * H R^-1, H - Q (Q^T H), U = Q W and V = B^T W S^-1 (Alg. 3, Alg. 5).
 * precision MC_FP32 rounds X to FP32 first (the solver's FP32 panels); the
 * arithmetic is FP64 either way. */
mc_status mc_k_panel(int64_t N, int32_t p, int32_t q, const double* X,
                     const double* W, double alpha, const double* colscale,
                     double beta, const double* C0, int32_t precision,
                     void* stream, double* C);

/* Orthonormal basis of range(H) for H (N x b) by two passes of Cholesky QR
 * (with a diagonal shift on breakdown): Q (N x b).  This is the build's
 * range-preserving normalisation of a Krylov block in place of the pivoted
 * LU of Alg. 4 and Alg. 5 (Lemmas 2-3).  Errors: MC_EINVAL for b > N. */
mc_status mc_k_cholqr2(int64_t N, int32_t b, const double* H, void* stream,
                       double* Q);

/* The eig step of eigSVD (Alg. 3) and the top-k selection of Alg. 5.
 * Top-k symmetric eigensolver (FP64) of G (L x L), the solver's own dispatch:
 * one-wavefront Jacobi for L <= 16, Householder tridiagonalisation +
 * multisection + inverse iteration up to L = 1024 (k <= 140), block Jacobi
 * beyond.  The k largest eigenvalues, descending, in evals (k) and their
 * eigenvectors in W (L x k); *sweeps receives the number of block-Jacobi
 * sweeps (0 on the other paths). */
mc_status mc_k_syev(int32_t L, const double* G, int32_t k, void* stream,
                    double* evals, double* W, int32_t* sweeps);

/* Fused SDDMM + residual + update on Phi (Eq. (6), Alg. 6): given
 * U (m x r), sig (r), V (n x r), M_Phi and Y on Phi (COO order), returns
 * x (P_Phi(X), input order), y_new = y + delta (M - x) and
 * *sumsq = sum (M - x)^2. */
mc_status mc_k_sddmm(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                     const int32_t* cols, const double* mvals,
                     const double* y, int32_t r, const double* U,
                     const double* sig, const double* V, double delta,
                     void* stream, double* x, double* y_new, double* sumsq);

/* Banded work schedule of the SpMM for a CSR-like structure (host code only:
 * a scheduling aid of this library for the products of Alg. 5, with no
 * counterpart in the paper; no device is touched).  This is the schedule the SpMM uses once the dense
 * panel it gathers from outgrows one XCD's L2: the gathered index range
 * [0, gathered) is cut into `bands` equal ranges (a positive multiple of 8);
 * rows of at least max(256, 4 cap) entries are split at the range
 * boundaries, then into pieces of at most `cap` entries; shorter rows into
 * pieces of at most `cap`.  Band r belongs to XCD r % 8, which takes its
 * bands in increasing r; the shorter rows go to the XCDs with the fewest
 * segments.
 *
 * Inputs: ptr (rows + 1, ptr[0] = 0, non-decreasing) and idx (ptr[rows]
 * entries in [0, gathered), increasing within each row), both host arrays
 * owned by the caller.  Outputs, caller allocated: segs, 4 int32 per segment
 * (row, begin, end, slot) in launch order -- segment s runs in workgroup
 * s / 4 and workgroup w on XCD w % 8; row -1 marks padding and slot -1 a row
 * done in one segment; fix, 4 int32 per row done in several segments (row,
 * first slot, count, 0), whose partial rows occupy consecutive slots.
 * On entry *nseg and *nfix hold the capacities of segs and fix in records; on
 * return they hold the counts, and *nslot the number of partial rows.  If a
 * capacity is too small (NULL buffers with capacity 0 included) nothing is
 * written to the buffers, the counts are still returned and the status is
 * MC_ERANGE.  Errors: MC_EINVAL for bad sizes, a bad ptr, an index out of
 * range or not increasing within its row. */
mc_status mc_k_band_schedule(int64_t rows, const int32_t* ptr, const int32_t* idx,
                             int64_t gathered, int32_t cap, int32_t bands,
                             int32_t* segs, int64_t* nseg, int32_t* fix,
                             int64_t* nfix, int64_t* nslot);

#ifdef __cplusplus
}
#endif

#endif /* MCSVT_KERNELS_H */
