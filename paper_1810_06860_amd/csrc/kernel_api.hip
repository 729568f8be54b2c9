// extern "C" kernel-level entry points declared in include/mcsvt_kernels.h.
#include <cmath>
#include <string>
#include <vector>

#include "mcsvt_kernels.h"
#include "solver.hpp"

namespace {

template <class F>
mc_status kguard(F&& f) {
  try {
    f();
    return MC_OK;
  } catch (const mcsvt::Error& e) {
    mcsvt_set_thread_error(e.what());
    return (mc_status)e.status;
  } catch (const std::exception& e) {
    mcsvt_set_thread_error(e.what());
    return MC_EDEVICE;
  }
}

template <class T>
T* upload(mcsvt::DevBuf<T>& d, const T* h, int64_t n, hipStream_t st) {
  d.reserve(std::max<int64_t>(n, 1), st);
  if (n > 0) MC_HIP(hipMemcpyAsync(d.p, h, n * sizeof(T), hipMemcpyHostToDevice, st));
  return d.p;
}

template <class T>
void download(T* h, const T* d, int64_t n, hipStream_t st) {
  if (n > 0) MC_HIP(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, st));
}

void build(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
           const int32_t* cols, mcsvt::Layout& L, hipStream_t st) {
  MC_REQUIRE(m >= 1 && n >= 1 && nnz >= 1 && rows && cols, mcsvt::kEINVAL,
             "bad sizes or NULL argument");
  mcsvt::DevBuf<int64_t> dr;
  mcsvt::DevBuf<int32_t> dc;
  upload(dr, rows, nnz, st);
  upload(dc, cols, nnz, st);
  const int s = mcsvt::build_layout(m, n, nnz, dr.p, dc.p, nullptr, L, st);
  if (s == mcsvt::kERANGE) throw mcsvt::Error(s, "index out of range");
  if (s == mcsvt::kEDUP) throw mcsvt::Error(s, "duplicate cell");
  if (s != mcsvt::kOK) throw mcsvt::Error(s, "invalid input");
}

}  // namespace

extern "C" {

mc_status mc_k_gaussian(int64_t rows, int64_t cols, uint64_t seed, uint32_t step,
                        uint32_t attempt, void* stream, double* out) {
  return kguard([&] {
    MC_REQUIRE(rows >= 0 && cols >= 0 && out, mcsvt::kEINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    mcsvt::DevBuf<double> d;
    d.reserve(std::max<int64_t>(rows * cols, 1), st);
    mcsvt::launch_gaussian<double>(d.p, rows, cols, cols, seed, step, attempt, st);
    download(out, d.p, rows * cols, st);
    MC_HIP(hipStreamSynchronize(st));
  });
}

mc_status mc_k_layout(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                      const int32_t* cols, void* stream, int32_t* row_ptr,
                      int32_t* col_idx, int32_t* order, int32_t* col_ptr,
                      int32_t* row_idx, int32_t* perm) {
  return kguard([&] {
    hipStream_t st = (hipStream_t)stream;
    mcsvt::Layout L;
    build(m, n, nnz, rows, cols, L, st);
    download(row_ptr, L.row_ptr.p, m + 1, st);
    download(col_idx, L.col_idx.p, nnz, st);
    download(order, L.order.p, nnz, st);
    download(col_ptr, L.col_ptr.p, n + 1, st);
    download(row_idx, L.row_idx.p, nnz, st);
    download(perm, L.perm.p, nnz, st);
    MC_HIP(hipStreamSynchronize(st));
  });
}

mc_status mc_k_spmm(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                    const int32_t* cols, const double* vals, int32_t transpose,
                    int32_t b, const double* X, int32_t precision, void* stream,
                    double* out) {
  return kguard([&] {
    MC_REQUIRE(vals && X && out && b >= 1, mcsvt::kEINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    mcsvt::Layout L;
    build(m, n, nnz, rows, cols, L, st);
    mcsvt::DevBuf<double> dv, dval, dX, dout, part;
    upload(dv, vals, nnz, st);
    dval.reserve(nnz, st);
    const mcsvt::Schedule& S = transpose ? L.sched_csc : L.sched_csr;
    const int32_t* idx = transpose ? L.row_idx.p : L.col_idx.p;
    mcsvt::launch_gather(nnz, L.order.p, dv.p, dval.p, st);
    if (transpose) {
      mcsvt::DevBuf<double> tmp;
      tmp.reserve(nnz, st);
      mcsvt::launch_gather(nnz, L.perm.p, dval.p, tmp.p, st);
      MC_HIP(hipMemcpyAsync(dval.p, tmp.p, nnz * sizeof(double), hipMemcpyDeviceToDevice, st));
      MC_HIP(hipStreamSynchronize(st));
    }
    const int64_t rows_out = transpose ? n : m;
    const int64_t rows_in = transpose ? m : n;
    upload(dX, X, rows_in * b, st);
    dout.reserve(rows_out * b, st);
    if (precision == MC_FP64) {
      part.reserve(std::max<int64_t>(1, S.nslot) * b, st);
      mcsvt::launch_spmm<double, double, double, double>(S, idx, dval.p, dX.p, b,
                                                         dout.p, b, b, part.p, st);
    } else {
      mcsvt::DevBuf<float> fv, fX, fout, fpart;
      fv.reserve(nnz, st);
      fX.reserve(rows_in * b, st);
      fout.reserve(rows_out * b, st);
      fpart.reserve(std::max<int64_t>(1, S.nslot) * b, st);
      mcsvt::launch_cast<double, float>(nnz, dval.p, fv.p, st);
      mcsvt::launch_cast<double, float>(rows_in * b, dX.p, fX.p, st);
      mcsvt::launch_spmm<float, float, float, float>(S, idx, fv.p, fX.p, b, fout.p,
                                                     b, b, fpart.p, st);
      mcsvt::launch_cast<float, double>(rows_out * b, fout.p, dout.p, st);
      MC_HIP(hipStreamSynchronize(st));
    }
    download(out, dout.p, rows_out * b, st);
    MC_HIP(hipStreamSynchronize(st));
  });
}

mc_status mc_k_gram(int64_t N, int32_t p, int32_t q, const double* A,
                    const double* B, int32_t sym, int32_t precision, void* stream,
                    double* C) {
  return kguard([&] {
    MC_REQUIRE(N >= 1 && p >= 1 && q >= 1 && A && C && (sym || B), mcsvt::kEINVAL,
               "bad arguments");
    MC_REQUIRE(!sym || p == q, mcsvt::kEINVAL, "sym needs p == q");
    hipStream_t st = (hipStream_t)stream;
    mcsvt::DevBuf<double> dA, dB, dC, part;
    upload(dA, A, N * p, st);
    const double* pB = dA.p;
    if (!sym) pB = upload(dB, B, N * q, st);
    dC.reserve((int64_t)p * q, st);
    const int64_t cap = mcsvt::gram_splits(N, p, q, sym) * p * q;
    if (precision == MC_FP64) {
      part.reserve(cap, st);
      mcsvt::launch_gram<double, double>(N, p, q, dA.p, p, pB, sym ? p : q, dC.p, q,
                                         sym, part.p, cap, st);
    } else {
      mcsvt::DevBuf<float> fA, fB, fpart;
      fA.reserve(N * p, st);
      mcsvt::launch_cast<double, float>(N * p, dA.p, fA.p, st);
      const float* fpB = fA.p;
      if (!sym) {
        fB.reserve(N * q, st);
        mcsvt::launch_cast<double, float>(N * q, pB, fB.p, st);
        fpB = fB.p;
      }
      fpart.reserve(cap, st);
      if (precision == MC_BF16_EIG64 && mcsvt::gram_bf16_fits(N, p, q, sym))
        mcsvt::launch_gram_bf16(N, p, q, fA.p, p, fpB, sym ? p : q, dC.p, q, sym, fpart.p,
                                cap, st);
      else
        mcsvt::launch_gram<float, float>(N, p, q, fA.p, p, fpB, sym ? p : q, dC.p, q,
                                         sym, fpart.p, cap, st);
      MC_HIP(hipStreamSynchronize(st));
    }
    download(C, dC.p, (int64_t)p * q, st);
    MC_HIP(hipStreamSynchronize(st));
  });
}

mc_status mc_k_panel(int64_t N, int32_t p, int32_t q, const double* X,
                     const double* W, double alpha, const double* colscale,
                     double beta, const double* C0, int32_t precision,
                     void* stream, double* C) {
  return kguard([&] {
    MC_REQUIRE(N >= 1 && p >= 1 && q >= 1 && X && W && C, mcsvt::kEINVAL,
               "bad arguments");
    MC_REQUIRE(beta == 0.0 || C0, mcsvt::kEINVAL, "beta != 0 needs C0");
    hipStream_t st = (hipStream_t)stream;
    mcsvt::DevBuf<double> dX, dW, ds, dC0, dC;
    upload(dX, X, N * p, st);
    upload(dW, W, (int64_t)p * q, st);
    const double* pS = colscale ? upload(ds, colscale, q, st) : nullptr;
    const double* pC0 = C0 ? upload(dC0, C0, N * q, st) : nullptr;
    dC.reserve(N * q, st);
    if (precision == MC_FP64) {
      mcsvt::launch_panel_gemm<double, double>(N, p, q, dX.p, p, dW.p, q, alpha, pS, beta,
                                               pC0, q, dC.p, q, st);
    } else {
      mcsvt::DevBuf<float> fX;
      fX.reserve(N * p, st);
      mcsvt::launch_cast<double, float>(N * p, dX.p, fX.p, st);
      mcsvt::launch_panel_gemm<float, double>(N, p, q, fX.p, p, dW.p, q, alpha, pS, beta,
                                              pC0, q, dC.p, q, st);
      MC_HIP(hipStreamSynchronize(st));
    }
    download(C, dC.p, N * q, st);
    MC_HIP(hipStreamSynchronize(st));
  });
}

mc_status mc_k_cholqr2(int64_t N, int32_t b, const double* H, void* stream,
                       double* Q) {
  return kguard([&] {
    MC_REQUIRE(N >= 1 && b >= 1 && b <= N && H && Q, mcsvt::kEINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    mcsvt::DevBuf<double> dH, d2, G, Rinv, work, part;
    mcsvt::DevBuf<int> shifted;
    upload(dH, H, N * b, st);
    d2.reserve(N * b, st);
    G.reserve((int64_t)b * b, st);
    Rinv.reserve((int64_t)b * b, st);
    work.reserve(2 * (int64_t)b * b, st);
    shifted.reserve(1, st);
    MC_HIP(hipMemsetAsync(shifted.p, 0, sizeof(int), st));
    const int64_t cap = mcsvt::gram_splits(N, b, b, 1) * b * b;
    part.reserve(cap, st);
    mcsvt::DevBuf<int> flag;
    flag.reserve(1, st);
    mcsvt::launch_set_int(flag.p, 0, st);
    double* in = dH.p;
    double* outp = d2.p;
    // two passes, then a third one gated on a shifted factorisation
    for (int pass = 0; pass < 3; ++pass) {
      const int* gate = pass == 2 ? flag.p : nullptr;
      mcsvt::launch_gram<double, double>(N, b, b, in, b, in, b, G.p, b, 1, part.p,
                                         cap, st, gate);
      mcsvt::launch_chol_inv(b, G.p, b, Rinv.p, b, work.p, N, shifted.p, st, flag.p,
                             gate);
      mcsvt::launch_panel_gemm<double, double>(N, b, b, in, b, Rinv.p, b, 1.0,
                                               nullptr, 0.0, nullptr, 0, outp, b, st,
                                               gate);
      if (pass < 2) std::swap(in, outp);
    }
    // after the loop `in` holds pass 2's result; pass 3 (if it ran) wrote outp
    mcsvt::launch_copy_gated<double>(N, b, outp, b, in, b, flag.p, st);
    download(Q, in, N * b, st);
    MC_HIP(hipStreamSynchronize(st));
  });
}

mc_status mc_k_syev(int32_t L, const double* G, int32_t k, void* stream,
                    double* evals, double* W, int32_t* sweeps) {
  return kguard([&] {
    MC_REQUIRE(L >= 1 && k >= 1 && k <= L && G && evals && W, mcsvt::kEINVAL,
               "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    mcsvt::DevBuf<double> dG, S, D, Wk;
    upload(dG, G, (int64_t)L * L, st);
    S.reserve(k, st);
    D.reserve(L, st);
    Wk.reserve((int64_t)L * k, st);
    mcsvt::EigSolver eig;
    eig.solve_topk(L, dG.p, L, k, S.p, D.p, Wk.p, k, st);
    download(evals, D.p, k, st);
    download(W, Wk.p, (int64_t)L * k, st);
    MC_HIP(hipStreamSynchronize(st));
    if (sweeps) *sweeps = eig.device_sweeps(st);
  });
}

mc_status mc_k_sddmm(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                     const int32_t* cols, const double* mvals, const double* y,
                     int32_t r, const double* U, const double* sig,
                     const double* V, double delta, void* stream, double* x,
                     double* y_new, double* sumsq) {
  return kguard([&] {
    MC_REQUIRE(mvals && y && x && y_new && sumsq && r >= 0, mcsvt::kEINVAL,
               "bad arguments");
    MC_REQUIRE(r == 0 || (U && sig && V), mcsvt::kEINVAL, "NULL factors");
    hipStream_t st = (hipStream_t)stream;
    mcsvt::Layout L;
    build(m, n, nnz, rows, cols, L, st);
    mcsvt::DevBuf<double> dm, dy, m_csr, y_csr, ycsc, dU, dV, dsig, part, scal, dx;
    upload(dm, mvals, nnz, st);
    upload(dy, y, nnz, st);
    m_csr.reserve(nnz, st);
    y_csr.reserve(nnz, st);
    ycsc.reserve(nnz, st);
    mcsvt::launch_gather(nnz, L.order.p, dm.p, m_csr.p, st);
    mcsvt::launch_gather(nnz, L.order.p, dy.p, y_csr.p, st);
    const int rr = std::max(r, 1);
    dU.reserve(m * rr, st);
    dV.reserve(n * rr, st);
    dsig.reserve(rr, st);
    if (r > 0) {
      upload(dU, U, m * r, st);
      upload(dV, V, n * r, st);
      upload(dsig, sig, r, st);
    }
    part.reserve(mcsvt::sddmm_partials(L), st);
    scal.reserve(1, st);
    dx.reserve(nnz, st);
    if (r > 0) {
      mcsvt::launch_eval_observed<double>(L, dU.p, r, dV.p, r, dsig.p, r, dx.p, st);
    } else {
      MC_HIP(hipMemsetAsync(dx.p, 0, nnz * sizeof(double), st));
    }
    mcsvt::launch_sddmm_update<double, double, double, double>(
        L, m_csr.p, y_csr.p, (double*)nullptr, ycsc.p, (double*)nullptr,
        (double*)nullptr, dU.p, r, dV.p, r, dsig.p, r, delta, 1, part.p, scal.p, st);
    mcsvt::launch_scatter(nnz, L.order.p, y_csr.p, dy.p, st);
    download(x, dx.p, nnz, st);
    download(y_new, dy.p, nnz, st);
    download(sumsq, scal.p, 1, st);
    MC_HIP(hipStreamSynchronize(st));
  });
}

mc_status mc_k_band_schedule(int64_t rows, const int32_t* ptr, const int32_t* idx,
                             int64_t gathered, int32_t cap, int32_t bands,
                             int32_t* segs, int64_t* nseg, int32_t* fix,
                             int64_t* nfix, int64_t* nslot) {
  return kguard([&] {
    MC_REQUIRE(rows >= 1 && ptr && nseg && nfix && nslot && gathered >= 1 &&
                   gathered <= INT32_MAX && cap >= 1 && bands >= mcsvt::kBands &&
                   bands % mcsvt::kBands == 0 && *nseg >= 0 && *nfix >= 0,
               mcsvt::kEINVAL, "bad sizes or NULL argument");
    MC_REQUIRE(ptr[0] == 0, mcsvt::kEINVAL, "ptr[0] must be 0");
    MC_REQUIRE(ptr[rows] == 0 || idx, mcsvt::kEINVAL, "NULL idx");
    for (int64_t i = 0; i < rows; ++i) {
      MC_REQUIRE(ptr[i + 1] >= ptr[i], mcsvt::kEINVAL, "ptr decreases");
      for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e)
        MC_REQUIRE(idx[e] >= 0 && idx[e] < gathered &&
                       (e == ptr[i] || idx[e] > idx[e - 1]),
                   mcsvt::kEINVAL, "index out of range or not increasing in its row");
    }
    std::vector<int4> s, f;
    int32_t slot = 0;
    mcsvt::band_schedule(ptr, idx, rows, gathered, cap, bands, s, f, slot);
    const bool fits = (int64_t)s.size() <= *nseg && (int64_t)f.size() <= *nfix &&
                      (segs || s.empty()) && (fix || f.empty());
    *nseg = (int64_t)s.size();
    *nfix = (int64_t)f.size();
    *nslot = slot;
    MC_REQUIRE(fits, mcsvt::kERANGE, "output capacity too small");
    for (size_t q = 0; q < s.size(); ++q) {
      segs[4 * q] = s[q].x;
      segs[4 * q + 1] = s[q].y;
      segs[4 * q + 2] = s[q].z;
      segs[4 * q + 3] = s[q].w;
    }
    for (size_t q = 0; q < f.size(); ++q) {
      fix[4 * q] = f[q].x;
      fix[4 * q + 1] = f[q].y;
      fix[4 * q + 2] = f[q].z;
      fix[4 * q + 3] = f[q].w;
    }
  });
}

}  // extern "C"
