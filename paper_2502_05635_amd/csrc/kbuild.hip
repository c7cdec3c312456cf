// Kernel build: direct electron-hole kernel of a lattice model (paper
// Eq. sigma-from-k with the single-G limit of Eq. bse-direct-def).
//
//   K_{(n m k),(n' m' k')} = -W(|fold(k - k')|) / (nk a^2) <n k|n' k'> <m' k'|m k>
//
// W is the 2D Rytova-Keldysh interaction 2pi / (q (1 + r0 q)); the divergent
// q = 0 term is replaced by its average over the grid cell (paper Appendix B).
// On a uniform grid q depends only on the index difference, so W (with the
// -1/(nk a^2) prefactor) is tabulated once per difference on the device (the
// q = 0 cell average, a single number, comes from the host) and the build
// kernel combines it with band overlaps.
#include <cmath>
#include <vector>

#include "internal.h"

namespace tdg {

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on the
// three-term Legendre recurrence, starting from the asymptotic root guess.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // refresh the derivative at the converged root
        p0 = 1.0;
        p1 = z;
        for (int j = 2; j <= n; ++j) {
          double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Average of W(q) = 2pi/(q(1 + r0 q)) over the square [-h, h]^2: integrate
// q dq in polar coordinates over the eight triangles of the square,
//   (1/4h^2) * 8 int_0^{pi/4} int_0^{h sec t} W(q) q dq dt
//   = (4 pi / (r0 h^2)) int_0^{pi/4} ln(1 + r0 h sec t) dt.
double cell_average_w0(double h, double r0, int nquad) {
  std::vector<double> x, w;
  gauss_legendre(nquad, x, w);
  double s = 0.0;
  for (int i = 0; i < nquad; ++i) {
    double t = 0.125 * M_PI * (x[i] + 1.0);
    double sec = 1.0 / std::cos(t);
    double inner = r0 > 0.0 ? std::log1p(r0 * h * sec) / r0 : h * sec;  // int_0^{h sec t} dq/(1 + r0 q)
    s += w[i] * inner;
  }
  s *= 0.125 * M_PI;
  return 4.0 * M_PI / (h * h) * s;
}

}  // namespace tdg

using namespace tdg;

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

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// <n k | n' k'> = sum_alpha conj(C_k[alpha][n]) C_k'[alpha][n']
__device__ inline double2 overlap(const double2* ck, const double2* ckp, int nb, int n, int np) {
  double2 s = make_double2(0.0, 0.0);
  for (int a = 0; a < nb; ++a) {
    double2 u = ck[a * nb + n], v = ckp[a * nb + np];
    s.x += u.x * v.x + u.y * v.y;
    s.y += u.x * v.y - u.y * v.x;
  }
  return s;
}

__device__ inline void pair_bands(int block, int nb, int nv, int p, int& a, int& b) {
  if (block == TDG_BLOCK_ALL) {
    a = p / nb;
    b = p % nb;
  } else {
    a = nv + p / nv;
    b = p % nv;
  }
}

// wt[d1 nk2 + d2] = scale W(q) for the index difference (d1, d2), folded into
// [-N/2, N/2) per direction; w0 replaces W at q = 0.
__global__ void __launch_bounds__(256) wtable_kernel(double* __restrict__ wt, int nk1, int nk2, double a, double r0,
                                                     double w0, double scale) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nk1 * nk2) return;
  const int d1 = i / nk2, d2 = i % nk2;
  const int m1 = (2 * d1 < nk1) ? d1 : d1 - nk1;
  const int m2 = (2 * d2 < nk2) ? d2 : d2 - nk2;
  const double qx = 2.0 * M_PI / (nk1 * a) * m1, qy = 2.0 * M_PI / (nk2 * a) * m2;
  const double q = sqrt(qx * qx + qy * qy);
  const double w = (m1 == 0 && m2 == 0) ? w0 : 2.0 * M_PI / (q * (1.0 + r0 * q));
  wt[i] = scale * w;
}

// One thread per (k, k') block of P x P kernel elements; k' runs along x so
// neighbouring threads write neighbouring column blocks of the same rows.
template <typename T>
__global__ void __launch_bounds__(256) build_kernel_k(const double* __restrict__ wtab, const double2* __restrict__ evec,
                                                      int nk1, int nk2, int nb, int nv, int block, int npair,
                                                      typename Cx<T>::type* __restrict__ K, int64_t ld) {
  const int nk = nk1 * nk2;
  const int kp = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (kp >= nk) return;
  const int i1 = k / nk2, i2 = k % nk2, j1 = kp / nk2, j2 = kp % nk2;
  const int d1 = (i1 - j1 + nk1) % nk1, d2 = (i2 - j2 + nk2) % nk2;
  const double w = wtab[d1 * nk2 + d2];
  const double2* ck = evec + (size_t)k * nb * nb;
  const double2* ckp = evec + (size_t)kp * nb * nb;
  for (int p = 0; p < npair; ++p) {
    int a, b;
    pair_bands(block, nb, nv, p, a, b);
    typename Cx<T>::type* row = K + (size_t)((int64_t)k * npair + p) * ld + (size_t)kp * npair;
    for (int q = 0; q < npair; ++q) {
      int a2, b2;
      pair_bands(block, nb, nv, q, a2, b2);
      // <a k|a2 k'> <b2 k'|b k> = O(a, a2) conj(O(b, b2))
      double2 v = cmulc(overlap(ck, ckp, nb, a, a2), overlap(ck, ckp, nb, b, b2));
      row[q].x = (T)(w * v.x);
      row[q].y = (T)(w * v.y);
    }
  }
}

extern "C" int tdg_kernel_dim(const tdg_model* model, int32_t block, int64_t* n_out) {
  if (!model || !n_out) return TDG_E_INVAL;
  int p = pairs_per_k(model, block);
  if (p <= 0 || model->nk1 <= 0 || model->nk2 <= 0) return TDG_E_INVAL;
  *n_out = (int64_t)model->nk1 * model->nk2 * p;
  return TDG_OK;
}

extern "C" int tdg_kernel_build(tdg_ctx ctx, const tdg_model* model, const tdg_coulomb* coul, int32_t dtype,
                                void* K, int64_t ld) {
  if (!ctx) return TDG_E_INVAL;
  TDG_TRY(validate_model(ctx, model));
  if (!coul) return fail(ctx, TDG_E_INVAL, "coulomb parameters are NULL");
  if (!(coul->r0_bohr >= 0.0)) return fail(ctx, TDG_E_INVAL, "r0 must be >= 0");
  const int npair = pairs_per_k(model, coul->block);
  if (npair <= 0) return fail(ctx, TDG_E_INVAL, "unknown block %d", coul->block);
  if (model->nk1 != model->nk2)
    return fail(ctx, TDG_E_UNSUPPORTED, "the q = 0 cell average is implemented for square grids only");
  if (dtype != TDG_C128 && dtype != TDG_C64 && dtype != TDG_BF16X2) return fail(ctx, TDG_E_INVAL, "dtype %d", dtype);
  const int nk = model->nk1 * model->nk2;
  const int64_t n = (int64_t)nk * npair;
  if (!K) return fail(ctx, TDG_E_INVAL, "K is NULL");
  if (ld < n) return fail(ctx, TDG_E_INVAL, "ld = %lld < N = %lld", (long long)ld, (long long)n);
  if (dtype == TDG_BF16X2 && ((ld % 4) != 0 || ((uintptr_t)K & 15)))
    return fail(ctx, TDG_E_INVAL, "BF16X2 storage needs ld %% 4 == 0 and a 16-byte aligned buffer");
  if (nk > 65535) return fail(ctx, TDG_E_UNSUPPORTED, "nk = %d exceeds the launch grid", nk);
  const int nquad = coul->nquad > 0 ? coul->nquad : 64;
  if (nquad > 4096) return fail(ctx, TDG_E_INVAL, "nquad = %d too large", nquad);
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));

  // W table by index difference, with the -1/(nk a^2) prefactor folded in
  const double a = model->a_bohr;
  void* wdev = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_WTAB, (size_t)nk * sizeof(double), &wdev));
  hipLaunchKernelGGL(wtable_kernel, dim3((nk + 255) / 256), dim3(256), 0, ctx->stream, (double*)wdev, model->nk1,
                     model->nk2, a, coul->r0_bohr, cell_average_w0(M_PI / (model->nk1 * a), coul->r0_bohr, nquad),
                     -1.0 / ((double)nk * a * a));
  TDG_TRY(launch_check(ctx, "W table launch"));
  dim3 grid((nk + 255) / 256, nk);
  if (dtype == TDG_BF16X2) {
    // build in complex64, then split into the hi / lo planes
    void* tmp = nullptr;
    TDG_TRY(ws_reserve(ctx, WS_TMP1, (size_t)n * n * sizeof(float2), &tmp));
    hipLaunchKernelGGL(build_kernel_k<float>, grid, dim3(256), 0, ctx->stream, (const double*)wdev,
                       (const double2*)model->evec, model->nk1, model->nk2, model->nb, model->nv, coul->block, npair,
                       (float2*)tmp, n);
    TDG_TRY(launch_check(ctx, "build_kernel launch"));
    if (n > 65535) return fail(ctx, TDG_E_UNSUPPORTED, "N exceeds the conversion grid");
    split_bf16x2(ctx->stream, tmp, 0, n, n, n, K, ld);
    return launch_check(ctx, "bf16 split launch");
  }
  if (dtype == TDG_C128)
    hipLaunchKernelGGL(build_kernel_k<double>, grid, dim3(256), 0, ctx->stream, (const double*)wdev,
                       (const double2*)model->evec, model->nk1, model->nk2, model->nb, model->nv, coul->block, npair,
                       (double2*)K, ld);
  else
    hipLaunchKernelGGL(build_kernel_k<float>, grid, dim3(256), 0, ctx->stream, (const double*)wdev,
                       (const double2*)model->evec, model->nk1, model->nk2, model->nb, model->nv, coul->block, npair,
                       (float2*)K, ld);
  return launch_check(ctx, "build_kernel launch");
}
