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

// Per-row sums of K_off (re, im, |.|^2) in FP64 for the rank rules, and the
// diagonal of K.  One row of K per block, coalesced over columns.
template <typename T>
__global__ void __launch_bounds__(256) koff_stats_kernel(const typename Cx<T>::type* __restrict__ K, int64_t ld,
                                                         int64_t n, double2* __restrict__ kdiag,
                                                         double* __restrict__ stats) {
  __shared__ double sh[3][256];
  const int64_t r = blockIdx.x;
  double a = 0.0, b = 0.0, m = 0.0;
  for (int64_t c = threadIdx.x; c < n; c += 256) {
    const auto v = K[r * ld + c];
    const double x = (double)v.x, y = (double)v.y;
    if (c == r) {
      kdiag[r] = make_double2(x, y);
      continue;
    }
    a += x;
    b += y;
    m += x * x + y * y;
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) stats[3 * r + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void to_c64_kernel(const double2* __restrict__ in, int64_t total, float2* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// Y = KX - diag(K) X for an n-row column-major block (K_off X from K X).
template <typename T>
__global__ void diag_sub_kernel(const typename Cx<T>::type* __restrict__ KX, const double2* __restrict__ X,
                                const double2* __restrict__ kd, int64_t n, int64_t total, double2* __restrict__ Y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 d = kd[i % n];
    const double2 x = X[i];
    const auto p = KX[i];
    Y[i] = make_double2((double)p.x - (d.x * x.x - d.y * x.y), (double)p.y - (d.x * x.y + d.y * x.x));
  }
}

// T <- (T + T^H) / 2 for a column-major l x l matrix; one thread per pair.
__global__ void hermitize_kernel(double2* __restrict__ T, int64_t l) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i > j || j >= l) return;
  if (i == j) {
    T[i + j * l].y = 0.0;
    return;
  }
  const double2 a = T[i + j * l], b = T[j + i * l];
  const double2 m = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  T[i + j * l] = m;
  T[j + i * l] = make_double2(m.x, -m.y);
}

// Hermitian dilation H = [[0, A], [A^H, 0]] (column-major c128, 2 nk x 2 nk)
// of channel (p, q) of K: A[i][j] = K[i P + p][j P + q].  Its eigenvalues are
// +-s_i; the eigenvector of +s_i is (u_i, v_i) / sqrt(2).
template <typename T>
__global__ void dilation_kernel(const typename Cx<T>::type* __restrict__ K, int64_t ld, int64_t nk, int P, int p,
                                int q, double2* __restrict__ H) {
  const int64_t c = blockIdx.y, m = 2 * nk;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    double2 v = make_double2(0.0, 0.0);
    if (r < nk && c >= nk) {
      const auto a = K[(r * P + p) * ld + (c - nk) * P + q];
      v = make_double2((double)a.x, (double)a.y);
    } else if (r >= nk && c < nk) {
      const auto a = K[(c * P + p) * ld + (r - nk) * P + q];
      v = make_double2((double)a.x, -(double)a.y);
    }
    H[r + c * m] = v;
  }
}

// Row sums of channel (p, q), FP64, for the R^2 rule's mean.
template <typename T>
__global__ void channel_rowsum_kernel(const typename Cx<T>::type* __restrict__ K, int64_t ld, int64_t nk, int P,
                                      int p, int q, double2* __restrict__ out) {
  __shared__ double sr[256], si[256];
  const int64_t r = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t c = threadIdx.x; c < nk; c += 256) {
    const auto v = K[(r * P + p) * ld + c * P + q];
    a += (double)v.x;
    b += (double)v.y;
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
  if (threadIdx.x == 0) out[r] = make_double2(sr[0], si[0]);
}

// Diagonal channel p, row-major [nk][nk], in the output precision.
template <typename T, typename TO>
__global__ void diag_channel_kernel(const typename Cx<T>::type* __restrict__ K, int64_t ld, int64_t nk, int P, int p,
                                    typename Cx<TO>::type* __restrict__ out) {
  const int64_t r = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nk; c += (int64_t)gridDim.x * blockDim.x) {
    const auto v = K[(r * P + p) * ld + c * P + p];
    typename Cx<TO>::type o;
    o.x = (TO)v.x;
    o.y = (TO)v.y;
    out[r * nk + c] = o;
  }
}

// Factors of channel (p, q) from the dilation's eigenvectors Q (ascending
// eigenvalues; s_j belongs to column 2 nk - 1 - j): S^{pq}[i][j] = s_j sqrt2 Q_top,
// V^{pq H}[j][i] = conj(sqrt2 Q_bottom) for j < r, zero for r <= j < rmax.
template <typename TO>
__global__ void channel_factor_kernel(const double2* __restrict__ Q, int64_t nk, int P, int p, int slot, int64_t rmax,
                                      int64_t r, const double* __restrict__ sig, typename Cx<TO>::type* __restrict__ S,
                                      typename Cx<TO>::type* __restrict__ W) {
  const int64_t j = blockIdx.y, ls = (int64_t)(P - 1) * rmax, m = 2 * nk;
  const double sq2 = 1.4142135623730951;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (int64_t)gridDim.x * blockDim.x) {
    typename Cx<TO>::type a, b;
    a.x = a.y = b.x = b.y = (TO)0;
    if (j < r) {
      const int64_t col = m - 1 - j;
      const double2 u = Q[i + col * m], v = Q[nk + i + col * m];
      a.x = (TO)(sig[j] * sq2 * u.x);
      a.y = (TO)(sig[j] * sq2 * u.y);
      b.x = (TO)(sq2 * v.x);
      b.y = (TO)(-sq2 * v.y);
    }
    S[(i * P + p) * ls + slot * rmax + j] = a;
    W[(((int64_t)p * (P - 1) + slot) * rmax + j) * nk + i] = b;
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

int blas_handle(tdg_ctx ctx, void** out_handle) {
  rocblas_handle* out = (rocblas_handle*)out_handle;
  if (!ctx->blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocblas_create_handle");
    ctx->blas = h;
  }
  *out = (rocblas_handle)ctx->blas;
  if (rocblas_set_stream(*out, ctx->stream) != rocblas_status_success)
    return fail(ctx, TDG_E_SOLVER, "rocblas_set_stream");
  return TDG_OK;
}

// Writes kdiag (from its FP64 copy KD) and the factors S = Q[:, perm] diag(kept),
// V^H = Q[:, perm]^H from the column-major n-row matrix Q, in out->dtype.
static int write_factors(tdg_ctx ctx, const double2* KD, const double2* Q, int64_t n, int64_t r,
                         const std::vector<int>& perm, const std::vector<double>& kept, tdg_lowrank* out) {
  const int bx = (int)std::min<int64_t>((n + 255) / 256, 64);
  if (out->dtype == TDG_C128)
    hipLaunchKernelGGL(kdiag_out_kernel<double>, dim3(bx), dim3(256), 0, ctx->stream, KD, n, (double2*)out->kdiag);
  else
    hipLaunchKernelGGL(kdiag_out_kernel<float>, dim3(bx), dim3(256), 0, ctx->stream, KD, n, (float2*)out->kdiag);
  TDG_TRY(launch_check(ctx, "compress diagonal"));
  if (r > 65535) return fail(ctx, TDG_E_UNSUPPORTED, "rank exceeds the launch grid");
  void* I = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_SOLVER_I, (size_t)r * (sizeof(int) + sizeof(double)) + 256, &I));
  int* dperm = (int*)I;
  double* dkept = (double*)((char*)I + (((size_t)r * sizeof(int) + 255) / 256) * 256);
  TDG_TRY(hip_check(ctx, hipMemcpy(dperm, perm.data(), r * sizeof(int), hipMemcpyHostToDevice), "perm upload"));
  TDG_TRY(hip_check(ctx, hipMemcpy(dkept, kept.data(), r * sizeof(double), hipMemcpyHostToDevice), "lambda upload"));
  if (out->dtype == TDG_C128) {
    hipLaunchKernelGGL(gather_kernel<double>, dim3(bx, (unsigned)r), dim3(256), 0, ctx->stream, Q, n, dperm, dkept, r,
                       (double2*)out->us, (double2*)out->w);
  } else if (out->dtype == TDG_C64) {
    hipLaunchKernelGGL(gather_kernel<float>, dim3(bx, (unsigned)r), dim3(256), 0, ctx->stream, Q, n, dperm, dkept, r,
                       (float2*)out->us, (float2*)out->w);
  } else {
    // gather in FP64, then split into hi / lo planes (us row stride: rank rounded up to 4)
    void *tus = nullptr, *tw = nullptr;
    TDG_TRY(ws_reserve(ctx, WS_TMP1, (size_t)n * r * sizeof(double2), &tus));
    TDG_TRY(ws_reserve(ctx, WS_TMP3, (size_t)n * r * sizeof(double2), &tw));
    hipLaunchKernelGGL(gather_kernel<double>, dim3(bx, (unsigned)r), dim3(256), 0, ctx->stream, Q, n, dperm, dkept, r,
                       (double2*)tus, (double2*)tw);
    TDG_TRY(launch_check(ctx, "compress gather"));
    const int64_t ld_us = (r + 3) / 4 * 4;
    split_bf16x2(ctx->stream, tus, 1, r, n, r, out->us, ld_us);
    split_bf16x2(ctx->stream, tw, 1, n, r, n, out->w, n);
  }
  TDG_TRY(launch_check(ctx, "compress gather"));
  return hip_check(ctx, hipStreamSynchronize(ctx->stream), "compress sync");
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
  TDG_TRY(launch_check(ctx, "compress prep"));
  hipLaunchKernelGGL(rowsum_kernel, dim3((unsigned)n), dim3(256), 0, ctx->stream, (const double2*)A, n, (double2*)M);
  TDG_TRY(launch_check(ctx, "compress row sums"));

  rocblas_handle h = nullptr;
  TDG_TRY(blas_handle(ctx, (void**)&h));
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
  return write_factors(ctx, (const double2*)KD, (const double2*)A, n, r, perm, kept, out);
}

// Rank rule on the l Ritz values s (descending) of an n x n K_off with
// ||K_off||_F^2 = fro2 and sum |K_off - mean|^2 = dev2.  Returns -1 when the
// rule's rank cannot be decided within the l values.
static int64_t choose_rank_ritz(const std::vector<double>& s, int64_t n, int mode, double value, double fro2,
                                double dev2) {
  const int64_t l = (int64_t)s.size();
  int64_t r = -1;
  if (mode == TDG_TRUNC_REL_CUT) {
    r = 0;
    for (int64_t i = 0; i < l; ++i)
      if (s[i] > value * s[0]) ++r;
    if (r == l && l < n) return -1;  // values beyond the range block may still pass the cut
  } else if (mode == TDG_TRUNC_FRACTION) {
    r = std::max<int64_t>(1, (int64_t)std::llround(value * (double)n));
  } else if (mode == TDG_TRUNC_RANK) {
    r = (int64_t)value;
  } else {
    double kept = 0.0;
    for (int64_t i = 0; i <= l; ++i) {
      if (1.0 - std::max(0.0, fro2 - kept) / dev2 >= value) {
        r = i;
        break;
      }
      if (i < l) kept += s[i] * s[i];
    }
    if (r < 0) return -1;
  }
  if (r > l) return -1;
  while (r > 0 && r < l && s[r - 1] - s[r] <= MULTIPLET_TOL * s[0]) ++r;
  return r;
}

extern "C" int tdg_kernel_compress_randomized(tdg_ctx ctx, const void* K, int64_t ld, int32_t dtype,
                                              const tdg_trunc* trunc, const void* omega, int64_t l,
                                              int32_t power_iters, tdg_lowrank* out) {
  if (!ctx) return TDG_E_INVAL;
  if (!K || !trunc || !out || !omega) return fail(ctx, TDG_E_INVAL, "NULL argument");
  if (dtype != TDG_C128 && dtype != TDG_C64) return fail(ctx, TDG_E_INVAL, "dtype %d", dtype);
  if (out->dtype != TDG_C128 && out->dtype != TDG_C64 && out->dtype != TDG_BF16X2)
    return fail(ctx, TDG_E_INVAL, "output dtype %d", out->dtype);
  const int64_t n = out->n;
  if (n < 2 || n > 200000) return fail(ctx, TDG_E_INVAL, "n = %lld outside [2, 200000]", (long long)n);
  if (ld < n) return fail(ctx, TDG_E_INVAL, "ld < n");
  if (l < 1 || l > n || l > 32768) return fail(ctx, TDG_E_INVAL, "l = %lld outside [1, min(n, 32768)]", (long long)l);
  if (power_iters < 0 || power_iters > 16) return fail(ctx, TDG_E_INVAL, "power_iters outside [0, 16]");
  if (out->max_rank < 1 || out->max_rank > n) return fail(ctx, TDG_E_INVAL, "max_rank outside [1, n]");
  if (!out->kdiag || !out->us || !out->w) return fail(ctx, TDG_E_INVAL, "output factor pointer is NULL");
  if (out->dtype == TDG_BF16X2 && ((n % 4) != 0 || (((uintptr_t)out->us | (uintptr_t)out->w) & 15)))
    return fail(ctx, TDG_E_UNSUPPORTED, "BF16X2 factors need n %% 4 == 0 and 16-byte aligned buffers");
  if (trunc->mode < TDG_TRUNC_REL_CUT || trunc->mode > TDG_TRUNC_R2)
    return fail(ctx, TDG_E_INVAL, "truncation mode %d", trunc->mode);
  if (!std::isfinite(trunc->value) || trunc->value < 0.0) return fail(ctx, TDG_E_INVAL, "truncation value");
  if (dtype == TDG_C64 && (((uintptr_t)K & 7) != 0)) return fail(ctx, TDG_E_INVAL, "C64 kernel must be 8-byte aligned");
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));

  const size_t nl = (size_t)n * (size_t)l;
  void *Y = nullptr, *Z = nullptr, *F = nullptr, *T = nullptr, *D = nullptr, *ST = nullptr, *KD = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_RSVD_Y, nl * sizeof(double2), &Y));
  TDG_TRY(ws_reserve(ctx, WS_RSVD_Z, nl * sizeof(double2), &Z));
  if (dtype == TDG_C64) TDG_TRY(ws_reserve(ctx, WS_RSVD_F, 2 * nl * sizeof(float2), &F));
  const size_t t_bytes = ((size_t)l * l * sizeof(double2) + 255) / 256 * 256;
  TDG_TRY(ws_reserve(ctx, WS_RSVD_T, t_bytes + (size_t)l * sizeof(double2), &T));
  TDG_TRY(ws_reserve(ctx, WS_SOLVER_D, (size_t)2 * l * sizeof(double), &D));
  TDG_TRY(ws_reserve(ctx, WS_MISC, (size_t)3 * n * sizeof(double) + 256, &ST));
  TDG_TRY(ws_reserve(ctx, WS_TMP2, (size_t)n * sizeof(double2), &KD));
  double2* tau = (double2*)((char*)T + t_bytes);
  int* info = (int*)((char*)ST + (size_t)3 * n * sizeof(double));

  // kdiag and the exact statistics of K_off
  if (dtype == TDG_C128)
    hipLaunchKernelGGL(koff_stats_kernel<double>, dim3((unsigned)n), dim3(256), 0, ctx->stream, (const double2*)K, ld, n,
                       (double2*)KD, (double*)ST);
  else
    hipLaunchKernelGGL(koff_stats_kernel<float>, dim3((unsigned)n), dim3(256), 0, ctx->stream, (const float2*)K, ld, n,
                       (double2*)KD, (double*)ST);
  TDG_TRY(launch_check(ctx, "compress statistics"));

  rocblas_handle h = nullptr;
  TDG_TRY(blas_handle(ctx, (void**)&h));
  const unsigned eb = (unsigned)std::min<size_t>((nl + 255) / 256, 8192);

  // dst = K_off src for an n x l column-major block (K row-major: K = (K as column-major)^T)
  auto apply_koff = [&](const double2* src, double2* dst) -> int {
    rocblas_status st;
    if (dtype == TDG_C128) {
      const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
      st = rocblas_zgemm_64(h, rocblas_operation_transpose, rocblas_operation_none, n, l, n, &one,
                            (const rocblas_double_complex*)K, ld, (const rocblas_double_complex*)src, n, &zero,
                            (rocblas_double_complex*)dst, n);
      if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocblas_zgemm status %d", (int)st);
      hipLaunchKernelGGL(diag_sub_kernel<double>, dim3(eb), dim3(256), 0, ctx->stream, (const double2*)dst, src,
                         (const double2*)KD, n, (int64_t)nl, dst);
    } else {
      float2* xf = (float2*)F;
      float2* yf = xf + nl;
      hipLaunchKernelGGL(to_c64_kernel, dim3(eb), dim3(256), 0, ctx->stream, src, (int64_t)nl, xf);
      TDG_TRY(launch_check(ctx, "compress conversion"));
      const rocblas_float_complex one(1.0f, 0.0f), zero(0.0f, 0.0f);
      st = rocblas_cgemm_64(h, rocblas_operation_transpose, rocblas_operation_none, n, l, n, &one,
                            (const rocblas_float_complex*)K, ld, (const rocblas_float_complex*)xf, n, &zero,
                            (rocblas_float_complex*)yf, n);
      if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocblas_cgemm status %d", (int)st);
      hipLaunchKernelGGL(diag_sub_kernel<float>, dim3(eb), dim3(256), 0, ctx->stream, (const float2*)yf, src,
                         (const double2*)KD, n, (int64_t)nl, dst);
    }
    return launch_check(ctx, "compress diagonal removal");
  };
  // Q <- orthonormal basis of the columns of Y, in place (Householder QR)
  auto orthonormalise = [&](double2* A) -> int {
    rocblas_status st = rocsolver_zgeqrf(h, (rocblas_int)n, (rocblas_int)l, (rocblas_double_complex*)A, (rocblas_int)n,
                                         (rocblas_double_complex*)tau);
    if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocsolver_zgeqrf status %d", (int)st);
    st = rocsolver_zungqr(h, (rocblas_int)n, (rocblas_int)l, (rocblas_int)l, (rocblas_double_complex*)A, (rocblas_int)n,
                          (rocblas_double_complex*)tau);
    if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocsolver_zungqr status %d", (int)st);
    return TDG_OK;
  };

  double2* y = (double2*)Y;
  double2* z = (double2*)Z;
  TDG_TRY(apply_koff((const double2*)omega, y));
  for (int it = 0; it < power_iters; ++it) {
    TDG_TRY(orthonormalise(y));
    TDG_TRY(apply_koff(y, z));
    std::swap(y, z);
  }
  TDG_TRY(orthonormalise(y));
  TDG_TRY(apply_koff(y, z));
  {
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    rocblas_status st = rocblas_zgemm_64(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, l, l, n,
                                         &one, (const rocblas_double_complex*)y, n, (const rocblas_double_complex*)z,
                                         n, &zero, (rocblas_double_complex*)T, l);
    if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocblas_zgemm status %d", (int)st);
  }
  hipLaunchKernelGGL(hermitize_kernel, dim3((unsigned)((l + 255) / 256), (unsigned)l), dim3(256), 0, ctx->stream,
                     (double2*)T, l);
  TDG_TRY(launch_check(ctx, "compress hermitize"));
  double* dvals = (double*)D;
  rocblas_status st = rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)l,
                                       (rocblas_double_complex*)T, (rocblas_int)l, dvals, dvals + l, info);
  if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocsolver_zheevd status %d", (int)st);
  {  // U = Q W for every Ritz vector (the rank rule picks the columns)
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    st = rocblas_zgemm_64(h, rocblas_operation_none, rocblas_operation_none, n, l, l, &one,
                          (const rocblas_double_complex*)y, n, (const rocblas_double_complex*)T, l, &zero,
                          (rocblas_double_complex*)z, n);
    if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocblas_zgemm status %d", (int)st);
  }
  TDG_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "randomized compression sync"));
  int hinfo = 0;
  TDG_TRY(hip_check(ctx, hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost), "info copy"));
  if (hinfo != 0) return fail(ctx, TDG_E_SOLVER, "rocsolver_zheevd info = %d", hinfo);
  std::vector<double> lam(l), stats((size_t)3 * n);
  TDG_TRY(hip_check(ctx, hipMemcpy(lam.data(), dvals, l * sizeof(double), hipMemcpyDeviceToHost), "eigenvalue copy"));
  TDG_TRY(hip_check(ctx, hipMemcpy(stats.data(), ST, stats.size() * sizeof(double), hipMemcpyDeviceToHost),
                    "statistics copy"));

  std::vector<int> order(l);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return std::fabs(lam[a]) > std::fabs(lam[b]); });
  std::vector<double> s(l);
  for (int64_t i = 0; i < l; ++i) s[i] = std::fabs(lam[order[i]]);
  double sr = 0.0, si = 0.0, fro2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    sr += stats[3 * i];
    si += stats[3 * i + 1];
    fro2 += stats[3 * i + 2];
  }
  const double dev2 = fro2 - (sr * sr + si * si) / ((double)n * (double)n);
  const int64_t r = choose_rank_ritz(s, n, trunc->mode, trunc->value, fro2, dev2);
  if (out->sigma) std::copy(s.begin(), s.end(), out->sigma);
  if (r < 0) return fail(ctx, TDG_E_INVAL, "the rank rule is not decided within l = %lld Ritz values", (long long)l);
  out->rank = r;
  double kept2 = 0.0;
  for (int64_t i = 0; i < r; ++i) kept2 += s[i] * s[i];
  out->tail_fro = std::sqrt(std::max(0.0, fro2 - kept2));
  out->tail_spec = r < l ? s[r] : (l < n ? std::nan("") : 0.0);
  if (r < 1) return fail(ctx, TDG_E_INVAL, "truncation keeps no singular value");
  if (r > out->max_rank)
    return fail(ctx, TDG_E_INVAL, "rank %lld exceeds max_rank %lld", (long long)r, (long long)out->max_rank);
  std::vector<int> perm(r);
  std::vector<double> kept(r);
  for (int64_t c = 0; c < r; ++c) {
    perm[c] = order[c];
    kept[c] = lam[order[c]];
  }
  return write_factors(ctx, (const double2*)KD, z, n, r, perm, kept, out);
}

extern "C" int tdg_kernel_compress_channels(tdg_ctx ctx, const void* K, int64_t ld, int32_t dtype,
                                            const tdg_trunc* trunc, tdg_channels* out) {
  if (!ctx) return TDG_E_INVAL;
  if (!K || !trunc || !out) return fail(ctx, TDG_E_INVAL, "NULL argument");
  if (dtype != TDG_C128 && dtype != TDG_C64) return fail(ctx, TDG_E_INVAL, "dtype %d", dtype);
  if (out->dtype != TDG_C128 && out->dtype != TDG_C64)
    return fail(ctx, TDG_E_UNSUPPORTED, "channel-wise factors are TDG_C128 or TDG_C64");
  const int64_t nk = out->nk, rmax = out->rmax;
  const int P = out->npair;
  if (P < 2 || P > TDG_NB_MAX * TDG_NB_MAX) return fail(ctx, TDG_E_INVAL, "npair = %d", P);
  if (nk < 2 || nk > 32767) return fail(ctx, TDG_E_INVAL, "nk = %lld outside [2, 32767]", (long long)nk);
  if (rmax < 4 || rmax % 4 != 0 || rmax > nk) return fail(ctx, TDG_E_INVAL, "rmax must be a multiple of 4 in [4, nk]");
  const int64_t n = nk * P;
  if (ld < n) return fail(ctx, TDG_E_INVAL, "ld < nk * npair");
  if (!out->diag || !out->s || !out->w) return fail(ctx, TDG_E_INVAL, "output pointer is NULL");
  if (trunc->mode < TDG_TRUNC_REL_CUT || trunc->mode > TDG_TRUNC_R2)
    return fail(ctx, TDG_E_INVAL, "truncation mode %d", trunc->mode);
  if (!std::isfinite(trunc->value) || trunc->value < 0.0) return fail(ctx, TDG_E_INVAL, "truncation value");
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));

  const int64_t m = 2 * nk;
  void *H = nullptr, *D = nullptr, *I = nullptr, *M = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_SOLVER_A, (size_t)m * m * sizeof(double2), &H));
  TDG_TRY(ws_reserve(ctx, WS_SOLVER_D, (size_t)2 * m * sizeof(double), &D));
  TDG_TRY(ws_reserve(ctx, WS_SOLVER_I, (size_t)nk * sizeof(double) + 256, &I));
  TDG_TRY(ws_reserve(ctx, WS_MISC, (size_t)nk * sizeof(double2), &M));
  rocblas_handle h = nullptr;
  TDG_TRY(blas_handle(ctx, (void**)&h));
  const int bx = (int)std::min<int64_t>((m + 255) / 256, 64);
  const bool o64 = out->dtype == TDG_C128;
  int* info = (int*)I;
  double* dsig = (double*)((char*)I + 256);
  std::vector<double> lam(m);
  std::vector<double2> rows(nk);

  for (int p = 0; p < P; ++p) {
    // the diagonal channel is kept whole
    auto* dst = (char*)out->diag + (size_t)p * nk * nk * (o64 ? 16 : 8);
    if (dtype == TDG_C128) {
      if (o64)
        hipLaunchKernelGGL((diag_channel_kernel<double, double>), dim3(bx, (unsigned)nk), dim3(256), 0, ctx->stream,
                           (const double2*)K, ld, nk, P, p, (double2*)dst);
      else
        hipLaunchKernelGGL((diag_channel_kernel<double, float>), dim3(bx, (unsigned)nk), dim3(256), 0, ctx->stream,
                           (const double2*)K, ld, nk, P, p, (float2*)dst);
    } else {
      if (o64)
        hipLaunchKernelGGL((diag_channel_kernel<float, double>), dim3(bx, (unsigned)nk), dim3(256), 0, ctx->stream,
                           (const float2*)K, ld, nk, P, p, (double2*)dst);
      else
        hipLaunchKernelGGL((diag_channel_kernel<float, float>), dim3(bx, (unsigned)nk), dim3(256), 0, ctx->stream,
                           (const float2*)K, ld, nk, P, p, (float2*)dst);
    }
    TDG_TRY(launch_check(ctx, "diagonal channel copy"));
    if (out->ranks) out->ranks[p * P + p] = nk;
    if (out->sigma) std::fill(out->sigma + ((size_t)p * P + p) * nk, out->sigma + ((size_t)p * P + p + 1) * nk, 0.0);

    for (int q = 0; q < P; ++q) {
      if (q == p) continue;
      const int slot = q < p ? q : q - 1;
      if (dtype == TDG_C128) {
        hipLaunchKernelGGL(dilation_kernel<double>, dim3(bx, (unsigned)m), dim3(256), 0, ctx->stream,
                           (const double2*)K, ld, nk, P, p, q, (double2*)H);
        hipLaunchKernelGGL(channel_rowsum_kernel<double>, dim3((unsigned)nk), dim3(256), 0, ctx->stream,
                           (const double2*)K, ld, nk, P, p, q, (double2*)M);
      } else {
        hipLaunchKernelGGL(dilation_kernel<float>, dim3(bx, (unsigned)m), dim3(256), 0, ctx->stream, (const float2*)K,
                           ld, nk, P, p, q, (double2*)H);
        hipLaunchKernelGGL(channel_rowsum_kernel<float>, dim3((unsigned)nk), dim3(256), 0, ctx->stream,
                           (const float2*)K, ld, nk, P, p, q, (double2*)M);
      }
      TDG_TRY(launch_check(ctx, "channel dilation"));
      double* dvals = (double*)D;
      rocblas_status st = rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)m,
                                           (rocblas_double_complex*)H, (rocblas_int)m, dvals, dvals + m, info);
      if (st != rocblas_status_success) return fail(ctx, TDG_E_SOLVER, "rocsolver_zheevd status %d", (int)st);
      TDG_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "channel eigensolver sync"));
      int hinfo = 0;
      TDG_TRY(hip_check(ctx, hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost), "info copy"));
      if (hinfo != 0) return fail(ctx, TDG_E_SOLVER, "rocsolver_zheevd info = %d (channel %d,%d)", hinfo, p, q);
      TDG_TRY(hip_check(ctx, hipMemcpy(lam.data(), dvals, m * sizeof(double), hipMemcpyDeviceToHost), "eigenvalues"));
      TDG_TRY(hip_check(ctx, hipMemcpy(rows.data(), M, nk * sizeof(double2), hipMemcpyDeviceToHost), "row sums"));
      // singular values, descending: the nk largest eigenvalues of the dilation
      std::vector<double> sv(nk);
      double fro2 = 0.0, sr = 0.0, si = 0.0;
      for (int64_t j = 0; j < nk; ++j) {
        sv[j] = std::fabs(lam[m - 1 - j]);
        fro2 += sv[j] * sv[j];
      }
      for (int64_t i = 0; i < nk; ++i) {
        sr += rows[i].x;
        si += rows[i].y;
      }
      const double dev2 = fro2 - (sr * sr + si * si) / ((double)nk * (double)nk);
      const int64_t r = choose_rank(sv, trunc->mode, trunc->value, dev2);
      if (out->ranks) out->ranks[p * P + q] = r;
      if (out->sigma) std::copy(sv.begin(), sv.end(), out->sigma + ((size_t)p * P + q) * nk);
      if (r > rmax)
        return fail(ctx, TDG_E_INVAL, "channel (%d,%d) rank %lld exceeds rmax %lld", p, q, (long long)r, (long long)rmax);
      if (r > 0)
        TDG_TRY(hip_check(ctx, hipMemcpy(dsig, sv.data(), r * sizeof(double), hipMemcpyHostToDevice), "sigma upload"));
      const int fb = (int)std::min<int64_t>((nk + 255) / 256, 64);
      if (o64)
        hipLaunchKernelGGL(channel_factor_kernel<double>, dim3(fb, (unsigned)rmax), dim3(256), 0, ctx->stream,
                           (const double2*)H, nk, P, p, slot, rmax, r, dsig, (double2*)out->s, (double2*)out->w);
      else
        hipLaunchKernelGGL(channel_factor_kernel<float>, dim3(fb, (unsigned)rmax), dim3(256), 0, ctx->stream,
                           (const double2*)H, nk, P, p, slot, rmax, r, dsig, (float2*)out->s, (float2*)out->w);
      TDG_TRY(launch_check(ctx, "channel factors"));
    }
  }
  return hip_check(ctx, hipStreamSynchronize(ctx->stream), "channel compression sync");
}
