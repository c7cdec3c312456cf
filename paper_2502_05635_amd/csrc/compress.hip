// Kernel compression (paper Sec. "SVD analysis of electron-hole kernel",
// Eq. svd_diag_offdiag): K = K_diag + K_off with K_diag the literal matrix
// diagonal; K_off is replaced by its rank-r truncated SVD, returned as
// S = U diag(s) (the S~ = U~ M~ of Eq. svd_acc) and V^H.
//
// K_off is Hermitian, so its SVD follows from the eigendecomposition
// K_off = Q diag(l) Q^H: s = |l|, U = Q sign(l), V = Q, hence
// S = Q diag(l) and V^H = Q^H restricted to the kept columns.  The
// eigendecomposition runs in FP64 on the device (rocSOLVER, divide and
// conquer); ordering and the rank rule run on the host.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace {

constexpr double MULTIPLET_TOL = 1e-9;

template <typename T>
struct Cx;
template <>
struct Cx<double> {
  using type = double2;
};
template <>
struct Cx<float> {
  using type = float2;
};

// A (column-major, c128) <- K_off: A[c + r n] = K_off(c, r) = conj(K(r, c));
// kdiag[r] <- K(r, r).  One row r of K per blockIdx.y, coalesced over c.
template <typename T>
__global__ void prep_kernel(const typename Cx<T>::type* __restrict__ K, int64_t ld, int64_t n, double2* __restrict__ A,
                            double2* __restrict__ kdiag) {
  const int64_t r = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const auto v = K[r * ld + c];
    double2 o = make_double2((double)v.x, -(double)v.y);
    if (c == r) {
      kdiag[r] = make_double2((double)v.x, (double)v.y);
      o = make_double2(0.0, 0.0);
    }
    A[c + r * n] = o;
  }
}

// Diagonal in the output precision.
template <typename T>
__global__ void kdiag_out_kernel(const double2* __restrict__ in, int64_t n, typename Cx<T>::type* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    typename Cx<T>::type v;
    v.x = (T)in[i].x;
    v.y = (T)in[i].y;
    out[i] = v;
  }
}

// Per-row sums of K_off (for the R^2 rule's mean), fixed order per row.
__global__ void rowsum_kernel(const double2* __restrict__ A, int64_t n, double2* __restrict__ out) {
  __shared__ double sr[256], si[256];
  const int64_t col = blockIdx.x;  // a column of A is a row of K_off^T
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double2 v = A[i + col * n];
    a += v.x;
    b += v.y;
  }
  sr[threadIdx.x] = a;
  si[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sr[threadIdx.x] += sr[threadIdx.x + w];
      si[threadIdx.x] += si[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[col] = make_double2(sr[0], si[0]);
}

// us[i][c] = lam[c] Q[i][perm[c]];  w[c][i] = conj(Q[i][perm[c]]).
template <typename T>
__global__ void gather_kernel(const double2* __restrict__ Q, int64_t n, const int* __restrict__ perm,
                              const double* __restrict__ lam, int64_t rank, typename Cx<T>::type* __restrict__ us,
                              typename Cx<T>::type* __restrict__ w) {
  const int64_t c = blockIdx.y;
  const int64_t col = perm[c];
  const double l = lam[c];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 q = Q[i + col * n];
    typename Cx<T>::type a, b;
    a.x = (T)(l * q.x);
    a.y = (T)(l * q.y);
    b.x = (T)q.x;
    b.y = (T)(-q.y);
    us[i * rank + c] = a;
    w[c * n + i] = b;
  }
}

}  // namespace

namespace tdg {

void release_blas(tdg_ctx ctx) {
  if (ctx->blas) {
    rocblas_destroy_handle((rocblas_handle)ctx->blas);
    ctx->blas = nullptr;
  }
}

// Rank rule on singular values s (descending).  dev2 = sum |K_off - mean|^2.
int64_t choose_rank(const std::vector<double>& s, int mode, double value, double dev2) {
  const int64_t n = (int64_t)s.size();
  int64_t r = 0;
  if (mode == TDG_TRUNC_REL_CUT) {
    for (int64_t i = 0; i < n; ++i)
      if (s[i] > value * s[0]) ++r;
  } else if (mode == TDG_TRUNC_FRACTION) {
    r = std::max<int64_t>(1, (int64_t)std::llround(value * (double)n));
  } else if (mode == TDG_TRUNC_RANK) {
    r = (int64_t)value;
  } else {
    // smallest r with 1 - sum_{i >= r} s_i^2 / dev2 >= value
    std::vector<double> tail(n + 1, 0.0);
    for (int64_t i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
    r = n;
    for (int64_t i = 0; i <= n; ++i)
      if (1.0 - tail[i] / dev2 >= value) {
        r = i;
        break;
      }
  }
  r = std::min(std::max<int64_t>(r, 0), n);
  while (r > 0 && r < n && s[r - 1] - s[r] <= MULTIPLET_TOL * s[0]) ++r;
  return r;
}

}  // namespace tdg

using namespace tdg;

extern "C" int tdg_kernel_compress(tdg_ctx ctx, const void* K, int64_t ld, int32_t dtype, const tdg_trunc* trunc,
                                   tdg_lowrank* out) {
  if (!ctx) return TDG_E_INVAL;
  if (!K || !trunc || !out) return fail(ctx, TDG_E_INVAL, "NULL argument");
  if (dtype != TDG_C128 && dtype != TDG_C64) return fail(ctx, TDG_E_INVAL, "dtype %d", dtype);
  if (out->dtype != TDG_C128 && out->dtype != TDG_C64 && out->dtype != TDG_BF16X2)
    return fail(ctx, TDG_E_INVAL, "output dtype %d", out->dtype);
  const int64_t n = out->n;
  if (n < 2 || n > 200000) return fail(ctx, TDG_E_INVAL, "n = %lld outside [2, 200000]", (long long)n);
  if (ld < n) return fail(ctx, TDG_E_INVAL, "ld < n");
  if (out->max_rank < 1 || out->max_rank > n) return fail(ctx, TDG_E_INVAL, "max_rank outside [1, n]");
  if (!out->kdiag || !out->us || !out->w) return fail(ctx, TDG_E_INVAL, "output factor pointer is NULL");
  if (out->dtype == TDG_BF16X2 && ((n % 4) != 0 || (((uintptr_t)out->us | (uintptr_t)out->w) & 15)))
    return fail(ctx, TDG_E_UNSUPPORTED, "BF16X2 factors need n %% 4 == 0 and 16-byte aligned buffers");
  if (trunc->mode < TDG_TRUNC_REL_CUT || trunc->mode > TDG_TRUNC_R2)
    return fail(ctx, TDG_E_INVAL, "truncation mode %d", trunc->mode);
  if (!std::isfinite(trunc->value) || trunc->value < 0.0) return fail(ctx, TDG_E_INVAL, "truncation value");
  if ((double)n * (double)n * 16.0 > 256e9)
    return fail(ctx, TDG_E_UNSUPPORTED, "dense FP64 eigendecomposition of n = %lld does not fit", (long long)n);
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));

  void *A = nullptr, *D = nullptr, *I = nullptr, *M = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_SOLVER_A, (size_t)n * n * sizeof(double2), &A));
  TDG_TRY(ws_reserve(ctx, WS_SOLVER_D, (size_t)2 * n * sizeof(double), &D));
  TDG_TRY(ws_reserve(ctx, WS_SOLVER_I, (size_t)n * (sizeof(int) + sizeof(double)) + 256, &I));
  TDG_TRY(ws_reserve(ctx, WS_MISC, (size_t)n * sizeof(double2), &M));
  void* KD = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_TMP2, (size_t)n * sizeof(double2), &KD));

  const int bx = (int)std::min<int64_t>((n + 255) / 256, 64);
  if (n > 65535) return fail(ctx, TDG_E_UNSUPPORTED, "n = %lld exceeds the launch grid", (long long)n);
  if (dtype == TDG_C128)
    hipLaunchKernelGGL(prep_kernel<double>, dim3(bx, (unsigned)n), dim3(256), 0, ctx->stream, (const double2*)K, ld, n,
                       (double2*)A, (double2*)KD);
  else
    hipLaunchKernelGGL(prep_kernel<float>, dim3(bx, (unsigned)n), dim3(256), 0, ctx->stream, (const float2*)K, ld, n,
                       (double2*)A, (double2*)KD);
  if (out->dtype == TDG_C128)
    hipLaunchKernelGGL(kdiag_out_kernel<double>, dim3(bx), dim3(256), 0, ctx->stream, (const double2*)KD, n,
                       (double2*)out->kdiag);
  else
    hipLaunchKernelGGL(kdiag_out_kernel<float>, dim3(bx), dim3(256), 0, ctx->stream, (const double2*)KD, n,
                       (float2*)out->kdiag);
  TDG_TRY(launch_check(ctx, "compress prep"));
  hipLaunchKernelGGL(rowsum_kernel, dim3((unsigned)n), dim3(256), 0, ctx->stream, (const double2*)A, n, (double2*)M);
  TDG_TRY(launch_check(ctx, "compress row sums"));

  if (!ctx->blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocblas_create_handle");
    ctx->blas = h;
  }
  rocblas_handle h = (rocblas_handle)ctx->blas;
  if (rocblas_set_stream(h, ctx->stream) != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocblas_set_stream");
  double* dvals = (double*)D;
  double* evals_off = dvals + n;
  int* info = (int*)I;
  rocblas_status st = rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)n,
                                       (rocblas_double_complex*)A, (rocblas_int)n, dvals, evals_off, info);
  if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocsolver_zheevd status %d", (int)st);
  TDG_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "eigensolver sync"));
  int hinfo = 0;
  std::vector<double> lam(n);
  std::vector<double2> rows(n);
  TDG_TRY(hip_check(ctx, hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost), "info copy"));
  if (hinfo != 0) return fail(ctx, TDG_E_SOLVER, "rocsolver_zheevd info = %d", hinfo);
  TDG_TRY(hip_check(ctx, hipMemcpy(lam.data(), dvals, n * sizeof(double), hipMemcpyDeviceToHost), "eigenvalue copy"));
  TDG_TRY(hip_check(ctx, hipMemcpy(rows.data(), M, n * sizeof(double2), hipMemcpyDeviceToHost), "row sum copy"));

  // order by |l| descending (stable on the ascending eigenvalue order)
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return std::fabs(lam[a]) > std::fabs(lam[b]); });
  std::vector<double> s(n);
  double fro2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    s[i] = std::fabs(lam[order[i]]);
    fro2 += s[i] * s[i];
  }
  double sr = 0.0, si = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    sr += rows[i].x;
    si += rows[i].y;
  }
  const double nn = (double)n * (double)n;
  const double dev2 = fro2 - (sr * sr + si * si) / nn;  // sum |y - mean|^2 = sum |y|^2 - n^2 |mean|^2
  const int64_t r = choose_rank(s, trunc->mode, trunc->value, dev2);
  out->rank = r;
  double tail = 0.0;
  for (int64_t i = r; i < n; ++i) tail += s[i] * s[i];
  out->tail_fro = std::sqrt(tail);
  out->tail_spec = r < n ? s[r] : 0.0;
  if (out->sigma) std::copy(s.begin(), s.end(), out->sigma);
  if (r < 1) return fail(ctx, TDG_E_INVAL, "truncation keeps no singular value");
  if (r > out->max_rank)
    return fail(ctx, TDG_E_INVAL, "rank %lld exceeds max_rank %lld", (long long)r, (long long)out->max_rank);

  std::vector<int> perm(r);
  std::vector<double> kept(r);
  for (int64_t c = 0; c < r; ++c) {
    perm[c] = order[c];
    kept[c] = lam[order[c]];
  }
  int* dperm = (int*)((char*)I + 256);
  double* dkept = (double*)M;  // row sums are no longer needed
  TDG_TRY(hip_check(ctx, hipMemcpy(dperm, perm.data(), r * sizeof(int), hipMemcpyHostToDevice), "perm upload"));
  TDG_TRY(hip_check(ctx, hipMemcpy(dkept, kept.data(), r * sizeof(double), hipMemcpyHostToDevice), "lambda upload"));
  if (r > 65535) return fail(ctx, TDG_E_UNSUPPORTED, "rank exceeds the launch grid");
  if (out->dtype == TDG_C128) {
    hipLaunchKernelGGL(gather_kernel<double>, dim3(bx, (unsigned)r), dim3(256), 0, ctx->stream, (const double2*)A, n,
                       dperm, dkept, r, (double2*)out->us, (double2*)out->w);
  } else if (out->dtype == TDG_C64) {
    hipLaunchKernelGGL(gather_kernel<float>, dim3(bx, (unsigned)r), dim3(256), 0, ctx->stream, (const double2*)A, n,
                       dperm, dkept, r, (float2*)out->us, (float2*)out->w);
  } else {
    // gather in FP64, then split into hi / lo planes (us row stride: rank rounded up to 4)
    void *tus = nullptr, *tw = nullptr;
    TDG_TRY(ws_reserve(ctx, WS_TMP1, (size_t)n * r * sizeof(double2), &tus));
    TDG_TRY(ws_reserve(ctx, WS_TMP3, (size_t)n * r * sizeof(double2), &tw));
    hipLaunchKernelGGL(gather_kernel<double>, dim3(bx, (unsigned)r), dim3(256), 0, ctx->stream, (const double2*)A, n,
                       dperm, dkept, r, (double2*)tus, (double2*)tw);
    TDG_TRY(launch_check(ctx, "compress gather"));
    const int64_t ld_us = (r + 3) / 4 * 4;
    split_bf16x2(ctx->stream, tus, 1, r, n, r, out->us, ld_us);
    split_bf16x2(ctx->stream, tw, 1, n, r, n, out->w, n);
  }
  TDG_TRY(launch_check(ctx, "compress gather"));
  return hip_check(ctx, hipStreamSynchronize(ctx->stream), "compress sync");
}
