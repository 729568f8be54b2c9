/*
 * mcsvt.h -- C ABI of the MI355X fast-SVT matrix completion library.
 *
 * The library solves   min ||X||_*  s.t.  P_Phi(X) = P_Phi(M)   (Eq. (5))
 * with singular value thresholding (Eq. (6), Alg. 2) whose truncated SVD is
 * the block-Krylov randomized SVD rSVD-BKI (Alg. 5) with eigSVD (Alg. 3),
 * subspace recycling (Sec. IV.B) and the adaptive power parameter of the
 * fast SVT algorithm (Alg. 6, Sec. IV.C).  All arithmetic of a step runs in
 * HIP kernels on one gfx950 GPU; the host keeps only the scalar control of
 * Alg. 6 (rank search, p adaptation, recycling gate, stop test).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Indices are 0-based.  Matrices handed in or out are row-major.
 * - Host pointers are owned by the caller and only read (or written) during
 *   the call.  Device state is owned by the handle until mc_svt_destroy.
 * - Every call returns an mc_status; no C++ exception crosses the ABI.  The
 *   message of the last failure is returned by mc_svt_last_error (per
 *   handle, or per thread when the handle is NULL or was never created).
 * - All device work is queued on the HIP stream given to mc_svt_init (NULL
 *   = the default stream).  Calls that return host data synchronise that
 *   stream; mc_svt_step synchronises it twice per SVD call at most (the
 *   singular values for the rank search and the residual for the stop test).
 * - Calls on one handle are not thread-safe; distinct handles are.
 */
#ifndef MCSVT_H
#define MCSVT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCSVT_ABI_VERSION 2

typedef struct mc_svt* mc_svt_t;

typedef enum {
  MC_OK = 0,
  MC_EINVAL = 1,    /* bad argument: sizes <= 0, nnz = 0, NaN/Inf value,
                       parameter out of range, NULL pointer */
  MC_EDUP = 2,      /* the same cell (i, j) appears twice in Phi */
  MC_ERANGE = 3,    /* a row or column index is outside [0, m) x [0, n) */
  MC_ENOMEM = 4,    /* device allocation failed (or exceeded the budget) */
  MC_EDEVICE = 5,   /* a HIP runtime call failed */
  MC_ENUMERIC = 6,  /* NaN/Inf residual or singular values */
  MC_EDONE = 7,     /* mc_svt_step after the solve has converged */
  MC_ENOTCONV = 8   /* mc_svt_solve reached i_max without converging; the
                       factors of X^{i_max} are still available (Alg. 2) */
} mc_status;

/* Arithmetic of the sparse/dense products.  The small eigenproblem, the
 * Cholesky factors of the orthonormalisation and the residual sum are FP64
 * in every mode. */
typedef enum {
  MC_FP64 = 0,        /* everything in FP64 */
  MC_FP32_EIG64 = 1,  /* SpMM / SDDMM / Gram in FP32 (FP32 accumulation) */
  MC_BF16_EIG64 = 2   /* SpMM values and panels in BF16, FP32 accumulation */
} mc_precision;

/* Solver settings.  mc_svt_default_params fills the paper's defaults. */
typedef struct {
  double tau;       /* threshold; <= 0 -> 5 n (Sec. II.C) */
  double delta;     /* step size; <= 0 -> 1.2 m n / |Phi| */
  double eps;       /* stop when ||P_Phi(X - M)||_F / ||P_Phi(M)||_F < eps
                       (Alg. 2, Alg. 6) */
  double ritz_tol;  /* guarded recycling: a recycled SVD whose Ritz residual
                       max_j ||Y v_j - s_j u_j|| / s_j exceeds this is
                       discarded and rSVD-BKI runs instead; the rest of that
                       step and the next q_reuse * 2^(s-1) steps make no
                       recycled call (s: rejections since the last accepted
                       recycled SVD, exponent capped at 20).  0 -> the
                       paper's i_reuse / q_reuse gate alone.  Default 1e-4. */
  double c;         /* Y^0 = c delta P_Phi(M); <= 0 -> ceil(tau / (delta
                       ||P_Phi(M)||_2)) (Sec. II.C) */
  int32_t i_max;    /* maximum SVT steps (default 200) */
  int32_t l;        /* rank increment of the rank search (default 5) */
  int32_t s;        /* oversampling of rSVD-BKI (default 10, Sec. II.B) */
  int32_t p_init;   /* initial power parameter (default 3, Alg. 6) */
  int32_t p_min, p_max;  /* bounds of the adaptive p (default 1, 8) */
  int32_t adaptive_p;    /* 1: p+1 after a rise of the error, p-1 after ten
                            consecutive decreases (Sec. IV.C); 0: fixed */
  int32_t i_reuse;  /* first step allowed to recycle (Alg. 6) */
  int32_t q_reuse;  /* recycled calls per rSVD-BKI basis (default 10) */
  int32_t recycle;  /* 0 none, 1 reuse Q, 2 reuse U (Sec. IV.B) */
  int32_t k_max;    /* rank cap; 0 -> min(m, n) */
  int32_t precision;  /* mc_precision */
  int32_t use_graphs; /* 1 (default): replay each SVD call's kernel sequence
                         from a captured HIP graph (per shape); 0: launch
                         kernel by kernel.  Results are identical. */
  uint64_t seed;    /* key of the counter-based Gaussian test matrices */
} mc_svt_params;

/* What one SVT step did (Alg. 6, one iteration of the outer loop). */
typedef struct {
  int32_t i;          /* 1-based step index */
  int32_t r;          /* rank of X^i: #{S_j > tau} (Alg. 6) */
  int32_t k;          /* rank parameter of the last SVD call */
  int32_t p;          /* power parameter used in this step */
  int32_t fresh;      /* rSVD-BKI calls in this step */
  int32_t recycled;   /* recycled SVD calls in this step */
  int32_t rejected;   /* recycled calls discarded by the Ritz guard */
  int32_t converged;  /* 1 if res < eps */
  double res;         /* ||P_Phi(X^i - M)||_F / ||P_Phi(M)||_F */
  double sigma_max;   /* largest singular value computed this step */
} mc_svt_step_info;

typedef struct {
  int32_t iters, rank, converged;
  int32_t fresh, recycled, rejected;  /* totals over the solve */
  double res;       /* residual of the returned X */
  double c;         /* the constant of Y^0 actually used */
  double norm2;     /* ||P_Phi(M)||_2 as computed on the device */
  double mnorm;     /* ||P_Phi(M)||_F */
  int32_t shifts;   /* Cholesky factorisations of the block orthonormalisation
                       that needed a diagonal shift (shifted Cholesky QR), as of
                       the last rSVD-BKI call */
  int32_t redone;   /* rSVD-BKI calls redone with the third orthonormalisation
                       pass because a factorisation needed a shift */
} mc_svt_result;

/* Optional allocator hooks (e.g. a framework's caching allocator): every
 * device buffer of the library (the iterate, the panels of Alg. 5, the
 * workspaces) is then taken from and returned to the caller's allocator.
 * alloc returns device memory of at least `bytes` usable on `stream`, or
 * NULL (the library then fails with MC_ENOMEM); release may be called while
 * work that used the block is still queued on `stream` (stream-ordered
 * reuse, as a caching allocator gives).  Both must be thread-safe.  NULL
 * hooks restore hipMalloc / hipFree.  Errors: MC_EINVAL if only one is NULL. */
typedef void* (*mc_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*mc_free_fn)(void* ptr, size_t bytes, void* stream, void* ctx);
mc_status mc_set_allocator(mc_alloc_fn alloc, mc_free_fn release, void* ctx);

/* MCSVT_ABI_VERSION of the built library. */
int32_t mc_abi_version(void);
/* The paper's settings (Sec. II.C: tau = 5 n, l = 5; Sec. II.B: s = 10;
 * Alg. 6: p = 3; Sec. IV.C: the adaptive p) and the build's defaults
 * for the rest (eps 1e-4, i_max 200, q_reuse 10, no recycling, ritz_tol
 * 1e-4, FP64, graphs on). */
void mc_svt_default_params(mc_svt_params* p);

/* Device bytes one handle can hold for a problem of this size: the layouts
 * of Phi, the iterate, and the panels and workspaces of the largest SVD call
 * the solve can make -- rank search bounded by min(m, n, k_max) (min(m, n)
 * when k_max = 0; the rank search of Alg. 6), block width k + s, Krylov basis
 * (p_max + 1)(k + s) (Alg. 5).  The solver never grows its buffers past
 * these sizes, so this is an upper bound; the serving loop admits requests
 * by it.  Returns 0 for sizes < 1; params NULL -> defaults. */
size_t mc_svt_footprint(int64_t m, int64_t n, int64_t nnz,
                        const mc_svt_params* p);

/*
 * mc_svt_init -- set up one completion problem (the start of Alg. 6).
 *   m, n        matrix size (each >= 1; m*n may exceed 2^31)
 *   nnz         |Phi| (>= 1, < 2^31)
 *   rows        is_csr = 0: COO row index of each observed entry (nnz)
 *               is_csr = 1: CSR row pointer (m + 1), entries of a row in
 *                           any column order
 *   cols        column index of each observed entry (nnz)
 *   vals        M_Phi (nnz), finite
 *   params      settings, NULL -> defaults
 *   stream      hipStream_t for all device work, NULL -> default stream
 *   out         receives the handle; set to NULL on failure
 * Builds the canonical CSR and CSC layouts of Phi on the device (entries
 * sorted by (row, col) and (col, row)), computes ||P_Phi(M)||_F and
 * ||P_Phi(M)||_2, c, and Y^0 = c delta P_Phi(M).
 * Errors: MC_EINVAL, MC_ERANGE, MC_EDUP, MC_ENOMEM, MC_EDEVICE.
 */
mc_status mc_svt_init(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                      const int32_t* cols, const double* vals, int32_t is_csr,
                      const mc_svt_params* params, void* stream,
                      mc_svt_t* out);

/* mc_svt_init with Phi and M_Phi already in device memory (e.g. tensors of a
 * framework): rows (int64: COO row ids, nnz, or with is_csr the CSR row
 * pointer, m + 1), cols (int32, nnz) and vals (double, nnz) are device
 * pointers readable on `stream`, owned by the caller and only read during
 * the call (the layout is copied).  The same set-up as mc_svt_init (the start of
 * Alg. 6, Sec. II.C), with the checks made on the device.  Returns after the
 * stream has finished the set-up.  Errors: as mc_svt_init (a non-finite
 * value or a bad CSR pointer gives MC_EINVAL). */
mc_status mc_svt_init_dev(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                          const int32_t* cols, const double* vals, int32_t is_csr,
                          const mc_svt_params* params, void* stream,
                          mc_svt_t* out);

/* One step of Alg. 6: rank search with rSVD-BKI or a recycled basis, shrink,
 * residual, and the update Y^i = Y^{i-1} + delta P_Phi(M - X^i) (Eq. (6)).
 * The residual and the update come out of one pass over Phi, so the update
 * is also applied on the converging step, where Alg. 2 and Alg. 6 stop
 * before it: X^i is the paper's, Y is one update further (see
 * mc_svt_get_y).  Errors: MC_EDONE after convergence, MC_ENUMERIC,
 * MC_EDEVICE, MC_ENOMEM. */
mc_status mc_svt_step(mc_svt_t h, mc_svt_step_info* info);

/* Advance `count` independent solves by one step each (continuous batching
 * of completion requests).  Each handle's step runs on one of a fixed pool
 * of host worker threads (at most 16), so the device work of solves on
 * different streams overlaps and a solve waiting for its stream does not
 * hold back the others.  Handles must be distinct.  Results are those of
 * mc_svt_step on each handle alone.  info[j] (may be NULL) receives what
 * mc_svt_step would return; status[j] (may be NULL) the per-handle status,
 * MC_EDONE for a handle that had already converged.  Returns MC_OK if every
 * handle succeeded or was already converged, else the first error.
 * Calls of mc_svt_step_many must not overlap (one caller thread).  If the
 * runtime drops a handle's graph capture, that handle continues with direct
 * launches (same results). */
mc_status mc_svt_step_many(mc_svt_t* hs, int32_t count,
                           mc_svt_step_info* info, mc_status* status);

/* Advance `count` independent solves by one step each (Alg. 6) with their
 * sparse products batched: the fresh rSVD-BKI calls (Alg. 5) of all the
 * handles run in lock-step stages, and the sparse products of one stage --
 * one per solve -- go out in shared launches (one per lane form and value
 * type) on a stream of the library's, which waits for each participant's
 * stage work and is waited for by each participant's stream.  Every other
 * kernel of a solve stays on its own stream.  The products run the same
 * per-segment code as a solo launch, so results are bit-identical to
 * mc_svt_step on each handle alone with graphs off.  FP64 and FP32 handles
 * are batched (each type with its own kind); BF16 handles, rSVD-PI and
 * recycled calls launch their products alone.  Captured graphs are not
 * used for the batched calls.  All handles on the calling thread's device,
 * distinct; calls of mc_svt_step_group (and mc_svt_step_many on the same
 * handles) must not overlap.  info[j] / status[j] (may be NULL) as in
 * mc_svt_step_many; a handle that fails takes no further part in the call
 * and the others go on.  Returns MC_OK if every handle succeeded or was
 * already converged, else the first error. */
mc_status mc_svt_step_group(mc_svt_t* hs, int32_t count,
                            mc_svt_step_info* info, mc_status* status);

/* Steps until convergence or i_max (Alg. 6 outer loop); MC_ENOTCONV at
 * i_max, with X^{i_max} available as Alg. 2 returns it.  out may be NULL. */
mc_status mc_svt_solve(mc_svt_t h, mc_svt_result* out);

/* Summary of the solve so far (valid after init): iteration count, rank and
 * residual of Alg. 6, and the constants of its set-up (c, ||P_Phi(M)||_2,
 * Sec. II.C).  Errors: MC_EINVAL for a NULL argument. */
mc_status mc_svt_get_result(mc_svt_t h, mc_svt_result* out);

/* The factors of the current X^i = sum_{j <= r} (S_j - tau) u_j v_j^T (the
 * shrink of Eq. (6), Alg. 6): U (m x r, row stride ldu >= r), sig =
 * S_j - tau descending (r), V (n x r, row stride ldv >= r); caller-owned
 * host buffers sized for r_cap columns (any may be NULL to skip it).  *r
 * receives the rank.  Errors: MC_EINVAL if r > r_cap or a stride < r. */
mc_status mc_svt_get_factors(mc_svt_t h, double* U, double* sig, double* V,
                             int64_t ldu, int64_t ldv, int32_t r_cap,
                             int32_t* r);

/* P_Phi(X^i), the completed matrix at the observed cells (the term of the
 * stop test and the update, Alg. 6), in the caller's input order:
 * x_phi (nnz, caller-owned host buffer).  Errors: MC_EINVAL for NULL. */
mc_status mc_svt_get_observed(mc_svt_t h, double* x_phi);

/* The current iterate Y (Eq. (6)) on Phi, in the caller's input order: y
 * (nnz, caller-owned host buffer).  After the converging step this is one
 * update past the paper's Y^{i-1} (mc_svt_step applies it in the same pass
 * as the residual).  Errors: MC_EINVAL for NULL. */
mc_status mc_svt_get_y(mc_svt_t h, double* y);

/* Singular values (descending) of the last SVD call of the last step (the
 * S^{i-1} of Alg. 6); *k receives their count; S is a
 * caller-owned host buffer of k_cap values.  Errors: MC_EINVAL if k_cap is
 * too small. */
mc_status mc_svt_get_sigma(mc_svt_t h, double* S, int32_t k_cap, int32_t* k);

/* Event timing of the solve's kernel families on its own stream (a
 * measurement aid of this library with no counterpart in the paper; adds two
 * hipEventRecord calls per timed launch).  Families:
 *   0 SpMM Y X (CSR)       1 SpMM Y^T X (CSC)     2 fused SDDMM/update
 *   3 Gram / cross-Gram    4 panel GEMMs          5 Cholesky + inverse
 *   6 eigensolve (all its kernels and convergence checks)
 *   7 Gaussian test matrix
 * launches = timed launches, ms = summed event time, bytes / flops = summed
 * algorithmic traffic and arithmetic of those launches. */
typedef struct {
  int64_t launches;
  double ms;
  double bytes;
  double flops;
} mc_prof_entry;

#define MC_PROF_FAMILIES 8

/* on = 1 starts timing (totals reset), on = 0 stops it. */
mc_status mc_svt_profile(mc_svt_t h, int32_t on);
/* Synchronises the stream and returns the totals since the last start;
 * cap >= MC_PROF_FAMILIES entries. */
mc_status mc_svt_get_profile(mc_svt_t h, mc_prof_entry* out, int32_t cap);

/* Frees every device buffer of the handle (NULL is a no-op). */
mc_status mc_svt_destroy(mc_svt_t h);
/* Message of the last failure on h, or of the calling thread when h is NULL;
 * owned by the library, valid until the next call on the same handle or
 * thread. */
const char* mc_svt_last_error(mc_svt_t h);

/*
 * Standalone truncated SVD of a sparse matrix A (m x n), with the kernels of
 * the solver: the randomized SVDs of Sec. III.
 *
 *   MC_RSVD_PI   rSVD-PI (Alg. 4): H = A Omega, then p power iterations
 *                H <- A (A^T H), the block re-normalised after each one
 *                (Cholesky QR instead of the pivoted LU: only the range
 *                matters, Lemma 3), and eigSVD of B^T = A^T Q (Alg. 3) on the
 *                last block alone.  Needs k + s <= min(m, n).
 *   MC_RSVD_BKI  rSVD-BKI (Alg. 5): the p + 1 blocks H_0..H_p stacked and
 *                orthonormalised together before eigSVD.  Needs
 *                (p + 1)(k + s) <= min(m, n).
 *
 * Omega is the n x (k + s) Gaussian test matrix drawn from (seed, step,
 * attempt) by the library's counter-based generator, so a call is
 * reproducible and a caller holding the same generator can rebuild it.
 * Outputs are the top k triplets, singular values descending:
 *   U (m x k) and V (n x k), host, row-major; S (k) host.
 * Errors as for mc_svt_init (A is checked the same way), plus MC_EINVAL for
 * k < 1, s < 0, p < 0, an unknown method, or a basis wider than min(m, n).
 */
typedef enum { MC_RSVD_PI = 4, MC_RSVD_BKI = 5 } mc_rsvd_method;

typedef struct mc_rsvd* mc_rsvd_t;

/* One call: copies A (COO: rows int64, cols int32, vals; nnz entries) to the
 * device, runs one truncated SVD, returns U, S, V and frees everything. */
mc_status mc_rsvd_bki(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                      const int32_t* cols, const double* vals, int32_t k,
                      int32_t s, int32_t p, uint64_t seed, uint32_t step,
                      uint32_t attempt, int32_t precision, void* stream,
                      double* U, double* S, double* V);
mc_status mc_rsvd_pi(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                     const int32_t* cols, const double* vals, int32_t k,
                     int32_t s, int32_t p, uint64_t seed, uint32_t step,
                     uint32_t attempt, int32_t precision, void* stream,
                     double* U, double* S, double* V);

/* A resident on the device for repeated calls (the oversampling s, the
 * precision and the generator seed are fixed here).  The handle owns the
 * device copy of A until mc_rsvd_destroy; its work is queued on `stream`. */
mc_status mc_rsvd_init(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                       const int32_t* cols, const double* vals, int32_t s,
                       int32_t precision, uint64_t seed, void* stream,
                       mc_rsvd_t* out);
/* One truncated SVD by `method` (mc_rsvd_method) with test matrix
 * (seed, step, attempt).  S (k values) is required; U and V may be NULL, and
 * are then not copied back.  Returns after S (and U, V) are on the host. */
mc_status mc_rsvd_run(mc_rsvd_t h, int32_t method, int32_t k, int32_t p,
                      uint32_t step, uint32_t attempt, double* U, double* S,
                      double* V);
/* Per-family kernel times of mc_rsvd_run calls, as mc_svt_profile and
 * mc_svt_get_profile (calls run kernel by kernel while timing is on). */
mc_status mc_rsvd_profile(mc_rsvd_t h, int32_t on);
mc_status mc_rsvd_get_profile(mc_rsvd_t h, mc_prof_entry* out, int32_t cap);
/* Frees the device copy of A and the workspaces (NULL is a no-op). */
mc_status mc_rsvd_destroy(mc_rsvd_t h);
/* As mc_svt_last_error: per handle, or per thread when h is NULL. */
const char* mc_rsvd_last_error(mc_rsvd_t h);

#ifdef __cplusplus
}
#endif

#endif /* MCSVT_H */
