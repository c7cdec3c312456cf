// Intraband part of the field coupling (paper Eq. tdagw, with the position
// operator r in the smooth gauge of Appendix A.1).
//
// The interband part of r is the dipole matrix d, which the stage kernels
// apply k-locally.  The intraband part acts on rho as a covariant derivative
// in k, [r_intra, rho]_k = i (rho)_{;k}, so with e = +1 the equation of motion
// gains -E(t) e.(rho)_{;k}.  On the uniform periodic grid the derivative is a
// central difference taken after carrying the neighbours into the gauge of k:
//
//   (rho)_{;a}(k) = [ L_a(k) rho(k + b_a) L_a(k)^H
//                     - L_a(k - b_a)^H rho(k - b_a) L_a(k - b_a) ] / (2 |b_a|),
//
// |b_a| = 2 pi / (N_a a).  The link L_a(k) transports the valence and the
// conduction subspace separately from k + b_a to k: it is the unitary polar
// factor of each diagonal block of the overlap M = evec_k^H evec_{k + b_a}
// and zero between the blocks.  Unitary links conserve sum_k Tr rho_k and
// leave rho_eq unchanged.
#include <hip/hip_ext.h>

#include <cmath>
#include <vector>

#include "covariant.h"
#include "internal.h"

namespace {

constexpr int SB = TDG_NB_MAX - 1;  // largest diagonal block (nv >= 1 and nb - nv >= 1)

__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// conj(a) * b
__device__ inline double2 zmulc(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__device__ inline double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// y <- x^{-1} (s x s) by Gauss-Jordan elimination with partial pivoting.
// Returns false if a pivot is below `tiny` in magnitude.
__device__ bool zinverse(const double2 (&x)[SB][SB], double2 (&y)[SB][SB], int s, double tiny) {
  double2 a[SB][SB];
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      a[i][j] = x[i][j];
      y[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
  for (int c = 0; c < s; ++c) {
    int p = c;
    double best = zabs2(a[c][c]);
    for (int r = c + 1; r < s; ++r)
      if (zabs2(a[r][c]) > best) {
        best = zabs2(a[r][c]);
        p = r;
      }
    if (!(best > tiny * tiny)) return false;
    if (p != c)
      for (int j = 0; j < s; ++j) {
        double2 t = a[c][j];
        a[c][j] = a[p][j];
        a[p][j] = t;
        t = y[c][j];
        y[c][j] = y[p][j];
        y[p][j] = t;
      }
    // row c /= pivot
    const double2 pv = a[c][c];
    const double inv = 1.0 / zabs2(pv);
    const double2 rp = make_double2(pv.x * inv, -pv.y * inv);
    for (int j = 0; j < s; ++j) {
      a[c][j] = zmul(a[c][j], rp);
      y[c][j] = zmul(y[c][j], rp);
    }
    for (int r = 0; r < s; ++r) {
      if (r == c) continue;
      const double2 f = a[r][c];
      for (int j = 0; j < s; ++j) {
        const double2 ta = zmul(f, a[c][j]), ty = zmul(f, y[c][j]);
        a[r][j].x -= ta.x;
        a[r][j].y -= ta.y;
        y[r][j].x -= ty.x;
        y[r][j].y -= ty.y;
      }
    }
  }
  return true;
}

// Unitary polar factor of the s x s matrix x (in place) by Newton's iteration
// X <- (zeta X + X^{-H} / zeta) / 2, with the Frobenius-norm scaling
// zeta = sqrt(|X^{-1}|_F / |X|_F) while the relative change exceeds 1e-2 and
// zeta = 1 after that (N. J. Higham, SIAM J. Sci. Stat. Comput. 7 (1986)).
// Returns 0, 1 if x is singular to working accuracy, 2 without convergence.
__device__ int polar_factor(double2 (&x)[SB][SB], int s) {
  double n0 = 0.0;
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) n0 += zabs2(x[i][j]);
  if (!(n0 > 0.0)) return 1;
  bool scaled = true, polish = false;
  for (int it = 0; it < 100; ++it) {
    double2 y[SB][SB];
    if (!zinverse(x, y, s, it == 0 ? 1e-10 * sqrt(n0) : 1e-300)) return 1;
    double nx = 0.0, ny = 0.0;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        nx += zabs2(x[i][j]);
        ny += zabs2(y[i][j]);
      }
    const double zeta = scaled ? sqrt(sqrt(ny / nx)) : 1.0;
    double diff = 0.0, norm = 0.0;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        // (X^{-H})_ij = conj((X^{-1})_ji)
        const double2 v = make_double2(0.5 * (zeta * x[i][j].x + y[j][i].x / zeta),
                                       0.5 * (zeta * x[i][j].y - y[j][i].y / zeta));
        diff += zabs2(make_double2(v.x - x[i][j].x, v.y - x[i][j].y));
        norm += zabs2(v);
        x[i][j] = v;
      }
    if (polish) return 0;
    if (scaled) {
      if (diff <= 1e-4 * norm) scaled = false;
    } else if (diff <= 1e-24 * norm) {
      polish = true;  // one more unscaled step squares the remaining error
    }
  }
  return 2;
}

// One thread per (axis a, k point): L_a(k) into links[a][k] ([nb][nb], row-major)
// and a status word (0 ok, 1 singular block, 2 no convergence) into status[a][k].
__global__ void __launch_bounds__(64) links_kernel(const double2* __restrict__ evec, int nk1, int nk2, int nb,
                                                   int nv, double2* __restrict__ links, int* __restrict__ status) {
  const int nk = nk1 * nk2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * nk) return;
  const int a = i / nk, k = i - a * nk;
  const int i1 = k / nk2, i2 = k - i1 * nk2;
  const int f = (a == 0) ? ((i1 + 1) % nk1) * nk2 + i2 : i1 * nk2 + (i2 + 1) % nk2;
  const double2* u = evec + (size_t)k * nb * nb;  // u[alpha * nb + n] = <alpha|n k>
  const double2* w = evec + (size_t)f * nb * nb;
  double2* out = links + (size_t)i * nb * nb;
  for (int e = 0; e < nb * nb; ++e) out[e] = make_double2(0.0, 0.0);
  int rc = 0;
  for (int blk = 0; blk < 2; ++blk) {
    const int o = blk ? nv : 0, s = blk ? nb - nv : nv;
    double2 x[SB][SB];
    for (int n = 0; n < s; ++n)
      for (int m = 0; m < s; ++m) {
        double2 acc = make_double2(0.0, 0.0);
        for (int al = 0; al < nb; ++al) {
          const double2 p = zmulc(u[al * nb + o + n], w[al * nb + o + m]);
          acc.x += p.x;
          acc.y += p.y;
        }
        x[n][m] = acc;
      }
    const int r = polar_factor(x, s);
    if (r > rc) rc = r;
    for (int n = 0; n < s; ++n)
      for (int m = 0; m < s; ++m) out[(o + n) * nb + o + m] = x[n][m];
  }
  status[i] = rc;
}

// out(b, k, e) = sum_a e_a c_a [ L_a(k) y(k+b_a) L_a(k)^H - L_a(k-b_a)^H y(k-b_a) L_a(k-b_a) ]_e,
// c_a = 1 / (2 |b_a|), for y and out addressed as b*sb + k*sk + e*se.  One thread
// per (k, element, instance), instances fastest; the links' block structure
// limits the sums to the blocks of the row and the column band.
__global__ void __launch_bounds__(256) covariant_derivative_kernel(
    const double2* __restrict__ y, int64_t sb, int64_t sk, int64_t se, const double2* __restrict__ links,
    const tdg_field* __restrict__ fields, int nk1, int nk2, int nb, int nv, int batch, double c1, double c2,
    double2* __restrict__ out) {
  const int nk = nk1 * nk2, nb2 = nb * nb;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (int64_t)nk * nb2 * batch) return;
  const int b = (int)(j % batch);
  const int e = (int)((j / batch) % nb2);
  const int k = (int)(j / ((int64_t)batch * nb2));
  const int n = e / nb, m = e - n * nb;
  const tdg_field F = fields[b];
  const double2* yb = y + (int64_t)b * sb;
  double2 acc = make_double2(0.0, 0.0);
  for (int a = 0; a < 2; ++a) {
    const double ea = a == 0 ? F.ex : F.ey;
    if (ea == 0.0) continue;
    int kf, kb;
    tdg::covariant_neighbours(k, a, nk1, nk2, kf, kb);
    const double2* lf = links + ((size_t)a * nk + k) * nb2;   // L_a(k)
    const double2* lb = links + ((size_t)a * nk + kb) * nb2;  // L_a(k - b_a)
    const double2* yf = yb + (int64_t)kf * sk;
    const double2* yk = yb + (int64_t)kb * sk;
    const double2 t = tdg::covariant_axis_element(
        n, m, nb, nv, [&](int r, int c) { return yf[(int64_t)(r * nb + c) * se]; },
        [&](int r, int c) { return yk[(int64_t)(r * nb + c) * se]; }, [&](int r, int c) { return lf[r * nb + c]; },
        [&](int r, int c) { return lb[r * nb + c]; });
    const double c = ea * (a == 0 ? c1 : c2);
    acc.x += c * t.x;
    acc.y += c * t.y;
  }
  out[(int64_t)b * sb + (int64_t)k * sk + (int64_t)e * se] = acc;
}

}  // namespace

namespace tdg {

void covariant_derivative(hipStream_t stream, const tdg_model* model, const void* y, int64_t sb, int64_t sk,
                          int64_t se, const tdg_field* fields, int batch, void* out, hipEvent_t ea, hipEvent_t eb) {
  const int nk = model->nk1 * model->nk2, nb = model->nb;
  const int64_t total = (int64_t)nk * nb * nb * batch;
  if (total == 0) return;
  const double c1 = model->nk1 * model->a_bohr / (4.0 * M_PI);  // 1 / (2 |b_1|)
  const double c2 = model->nk2 * model->a_bohr / (4.0 * M_PI);
  hipExtLaunchKernelGGL(covariant_derivative_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0u, stream, ea,
                        eb, 0u, (const double2*)y, sb, sk, se, (const double2*)model->links, fields, model->nk1,
                        model->nk2, nb, model->nv, batch, c1, c2, (double2*)out);
}

}  // namespace tdg

using namespace tdg;

extern "C" int tdg_links_build(tdg_ctx ctx, const tdg_model* model, void* links) {
  if (!ctx) return TDG_E_INVAL;
  TDG_TRY(validate_model(ctx, model));
  if (!links) return fail(ctx, TDG_E_INVAL, "links is NULL");
  if ((uintptr_t)links & 15) return fail(ctx, TDG_E_INVAL, "links must be 16-byte aligned");
  const int nk = model->nk1 * model->nk2;
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
  void* st = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_MISC, (size_t)2 * nk * sizeof(int), &st));
  hipLaunchKernelGGL(links_kernel, dim3((2 * nk + 63) / 64), dim3(64), 0, ctx->stream, (const double2*)model->evec,
                     model->nk1, model->nk2, model->nb, model->nv, (double2*)links, (int*)st);
  TDG_TRY(launch_check(ctx, "links_kernel launch"));
  std::vector<int> status((size_t)2 * nk);
  TDG_TRY(hip_check(ctx, hipMemcpyAsync(status.data(), st, status.size() * sizeof(int), hipMemcpyDeviceToHost,
                                        ctx->stream),
                    "links status copy"));
  TDG_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "links build sync"));
  for (int i = 0; i < 2 * nk; ++i)
    if (status[i] != 0)
      return fail(ctx, TDG_E_NUMERIC,
                  "link %s at k = %d: %s", i < nk ? "x" : "y", i % nk,
                  status[i] == 1 ? "a subspace overlap with the neighbour is singular (grid too coarse for transport)"
                                 : "the polar iteration did not converge");
  return TDG_OK;
}
