// TD-aGW propagation on the device: RK4 integration of
//
//   i d rho_k/dt = [ eps_k + dSigma_k - E(t) e.d_k , rho_k ]          (paper Eq. tdagw)
//   dSigma = K drho                                                   (Eq. sigma-from-k)
//   dSigma = K_diag o drho + S (V^H drho)                             (Eq. svd_acc)
//
// Per RK4 stage one "stage" kernel runs per (k point, instance): it forms the
// k point's P kernel rows dotted with the gathered drho (dense: rows of K;
// low rank: rows of S dotted with z = V^H drho from the projection kernel),
// builds H_k, evaluates f = -i [H_k, rho_k], advances the RK4 stage and
// writes the next stage's drho gather.  Launch boundaries are the global
// synchronisation every stage needs (each stage contracts all of drho).
// Observables of rho(t_n) are formed per k in the first stage of step n and
// reduced over k in fixed order by a separate kernel every few steps.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace {

constexpr int THREADS = 256;
constexpr int WAVES = THREADS / 64;
constexpr int NB2_MAX = TDG_NB_MAX * TDG_NB_MAX;
constexpr int ROWS = 4;  // kernel rows contracted together (shared drho loads)
constexpr size_t OBS_PART_BUDGET = size_t(64) << 20;

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

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

__device__ inline double field_value(const tdg_field& f, double t) {
  const double d = t - f.t0;
  return f.e0 * exp(-d * d / (2.0 * f.tau * f.tau)) * cos(f.omega * t);
}

// ---- row dot products ------------------------------------------------------
// acc_r = sum_j A[r][j] x[j] for r < nvalid (rows lda apart), this thread's
// share of the columns; the block reduction below completes the sums.

__device__ inline void rows_dot(const float2* __restrict__ A, int64_t lda, int nvalid, int ncols,
                                const float2* __restrict__ x, float (&ar)[ROWS], float (&ai)[ROWS]) {
  if (((lda | (int64_t)(uintptr_t)A / 8 | (int64_t)(uintptr_t)x / 8) & 1) == 0) {
    // two complex numbers per 16-byte load
    const int npair = ncols >> 1;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    for (int j = threadIdx.x; j < npair; j += THREADS) {
      const float4 xv = x4[j];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        if (r < nvalid) {
          const float4 a = reinterpret_cast<const float4*>(A + r * lda)[j];
          ar[r] += a.x * xv.x - a.y * xv.y + a.z * xv.z - a.w * xv.w;
          ai[r] += a.x * xv.y + a.y * xv.x + a.z * xv.w + a.w * xv.z;
        }
      }
    }
    if ((ncols & 1) && threadIdx.x == 0) {
      const float2 xv = x[ncols - 1];
      for (int r = 0; r < nvalid; ++r) {
        const float2 a = A[r * lda + ncols - 1];
        ar[r] += a.x * xv.x - a.y * xv.y;
        ai[r] += a.x * xv.y + a.y * xv.x;
      }
    }
  } else {
    for (int j = threadIdx.x; j < ncols; j += THREADS) {
      const float2 xv = x[j];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        if (r < nvalid) {
          const float2 a = A[r * lda + j];
          ar[r] += a.x * xv.x - a.y * xv.y;
          ai[r] += a.x * xv.y + a.y * xv.x;
        }
      }
    }
  }
}

__device__ inline void rows_dot(const double2* __restrict__ A, int64_t lda, int nvalid, int ncols,
                                const double2* __restrict__ x, double (&ar)[ROWS], double (&ai)[ROWS]) {
  for (int j = threadIdx.x; j < ncols; j += THREADS) {
    const double2 xv = x[j];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if (r < nvalid) {
        const double2 a = A[r * lda + j];
        ar[r] += a.x * xv.x - a.y * xv.y;
        ai[r] += a.x * xv.y + a.y * xv.x;
      }
    }
  }
}

// Sum each thread's ROWS complex partials over the block; out[2r], out[2r+1]
// receive row r (as double).  Wave shuffles, then a fixed-order sum over waves.
template <typename T>
__device__ inline void block_reduce(T (&ar)[ROWS], T (&ai)[ROWS], double* red, double* out) {
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    for (int off = 32; off > 0; off >>= 1) {
      ar[r] += __shfl_xor(ar[r], off, 64);
      ai[r] += __shfl_xor(ai[r], off, 64);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      red[wave * 2 * ROWS + 2 * r] = (double)ar[r];
      red[wave * 2 * ROWS + 2 * r + 1] = (double)ai[r];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * ROWS) {
    double s = 0.0;
    for (int w = 0; w < WAVES; ++w) s += red[w * 2 * ROWS + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

struct StageParams {
  const void* A;      // dense: K [N][lda]; low rank: S [N][lda = rank]
  int64_t lda;
  int ncols;          // N (dense) or rank (low rank)
  const void* vec;    // contracted vector per instance: drho gather (dense) or z (low rank)
  int64_t vstride;
  const void* kdiag;  // low rank: K_diag [N]; dense: NULL
  const void* xcur;   // drho gather of this stage [B][xstride]
  void* xnext;        // drho gather of the next stage
  int64_t xstride;
  double2* rho_n;     // rho(t_n) [B][nk][nb][nb]
  double2* rho_s;     // state of this stage
  double2* acc;       // RK4 sum of stage derivatives
  const double* eps;
  const double2* dip;
  const double2* vel;
  const tdg_field* fields;
  double* obs_part;   // [slot][B][nk][5] or NULL
  int obs_slot;
  int nk, nb, nv, npair, block, batch;
  int step, stage;
  double dt;
};

// Per-k observables of s_rho into obs_part (threads t < nb^2 participate).
__device__ inline void per_k_observables(const StageParams& sp, const double2* s_rho, double (*s_obs)[NB2_MAX],
                                         const tdg_field& F, int k, int b) {
  const int nb = sp.nb, nb2 = nb * nb, t = threadIdx.x;
  if (t < nb2) {
    const int n = t / nb, m = t % nb;
    const size_t base = (size_t)k * nb2 + t;
    const size_t plane = (size_t)sp.nk * nb2;
    const double2 d = make_double2(F.ex * sp.dip[base].x + F.ey * sp.dip[plane + base].x,
                                   F.ex * sp.dip[base].y + F.ey * sp.dip[plane + base].y);
    const double2 v = make_double2(F.ex * sp.vel[base].x + F.ey * sp.vel[plane + base].x,
                                   F.ex * sp.vel[base].y + F.ey * sp.vel[plane + base].y);
    const double2 rmn = s_rho[m * nb + n];
    const double2 rnm = s_rho[t];
    s_obs[0][t] = d.x * rmn.x - d.y * rmn.y;  // Re(d_nm rho_mn)
    s_obs[1][t] = v.x * rmn.x - v.y * rmn.y;
    s_obs[2][t] = (n == m && n == sp.nv) ? rnm.x : 0.0;
    s_obs[3][t] = (n == m) ? rnm.x : 0.0;
    const double hx = rnm.x - rmn.x, hy = rnm.y + rmn.y;
    s_obs[4][t] = sqrt(hx * hx + hy * hy);
  }
  __syncthreads();
  if (t == 0) {
    double o[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < nb2; ++i) {
      o[0] += s_obs[0][i];
      o[1] += s_obs[1][i];
      o[2] += s_obs[2][i];
      o[3] += s_obs[3][i];
      const double h = s_obs[4][i];
      if (h > o[4] || h != h) o[4] = h;
    }
    o[3] = fabs(o[3] - (double)sp.nv);
    double* dst = sp.obs_part + (((size_t)sp.obs_slot * sp.batch + b) * sp.nk + k) * 5;
    for (int c = 0; c < 5; ++c) dst[c] = o[c];
  }
}

template <typename T>
__global__ void __launch_bounds__(THREADS) stage_kernel(StageParams sp) {
  using C = typename Cx<T>::type;
  const int k = blockIdx.x, b = blockIdx.y;
  const tdg_field F = sp.fields[b];
  const int64_t nsb = (int64_t)F.nsteps;
  if (sp.step > nsb) return;                     // instance finished
  if (sp.stage != 0 && sp.step >= nsb) return;

  __shared__ double2 s_rho[NB2_MAX];
  __shared__ double2 s_h[NB2_MAX];
  __shared__ double s_y[2 * NB2_MAX];
  __shared__ double s_red[WAVES * 2 * ROWS];
  __shared__ double s_obs[5][NB2_MAX];

  const int nb = sp.nb, nb2 = nb * nb, P = sp.npair, t = threadIdx.x;
  const size_t kb = ((size_t)b * sp.nk + k) * nb2;
  if (t < nb2) s_rho[t] = sp.rho_s[kb + t];
  __syncthreads();
  if (sp.stage == 0 && sp.obs_part) per_k_observables(sp, s_rho, s_obs, F, k, b);
  if (sp.step == nsb) return;                    // final time: observables only

  // ---- contraction: y_p = sum_j A[k P + p][j] vec[j] ----------------------
  const C* A = reinterpret_cast<const C*>(sp.A);
  const C* vec = reinterpret_cast<const C*>(sp.vec) + (size_t)b * sp.vstride;
  for (int r0 = 0; r0 < P; r0 += ROWS) {
    const int nvalid = min(ROWS, P - r0);
    T ar[ROWS], ai[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) ar[r] = ai[r] = (T)0;
    rows_dot(A + ((int64_t)k * P + r0) * sp.lda, sp.lda, nvalid, sp.ncols, vec, ar, ai);
    block_reduce<T>(ar, ai, s_red, s_y + 2 * r0);
  }
  const C* xcur = reinterpret_cast<const C*>(sp.xcur) + (size_t)b * sp.xstride;
  if (sp.kdiag && t < P) {
    const C kd = reinterpret_cast<const C*>(sp.kdiag)[(size_t)k * P + t];
    const C xv = xcur[(size_t)k * P + t];
    const T re = kd.x * xv.x - kd.y * xv.y, im = kd.x * xv.y + kd.y * xv.x;
    s_y[2 * t] += (double)re;
    s_y[2 * t + 1] += (double)im;
  }
  __syncthreads();

  // ---- H_k = eps_k + dSigma_k - E(t) e.d_k ----------------------------------
  const double cs = (sp.stage == 0) ? 0.0 : (sp.stage == 3 ? 1.0 : 0.5);
  const double tt = (double)sp.step * sp.dt + cs * sp.dt;
  const double ef = field_value(F, tt);
  if (t < nb2) {
    const int n = t / nb, m = t % nb;
    double2 ds = make_double2(0.0, 0.0);
    if (sp.block == TDG_BLOCK_ALL) {
      ds = make_double2(s_y[2 * t], s_y[2 * t + 1]);
    } else if (n >= sp.nv && m < sp.nv) {
      const int p = (n - sp.nv) * sp.nv + m;
      ds = make_double2(s_y[2 * p], s_y[2 * p + 1]);
    } else if (n < sp.nv && m >= sp.nv) {
      const int p = (m - sp.nv) * sp.nv + n;
      ds = make_double2(s_y[2 * p], -s_y[2 * p + 1]);
    }
    const size_t base = (size_t)k * nb2 + t;
    const size_t plane = (size_t)sp.nk * nb2;
    const double2 d0 = sp.dip[base], d1 = sp.dip[plane + base];
    double2 h = make_double2(ds.x - ef * (F.ex * d0.x + F.ey * d1.x), ds.y - ef * (F.ex * d0.y + F.ey * d1.y));
    if (n == m) h.x += sp.eps[(size_t)k * nb + n];
    s_h[t] = h;
  }
  __syncthreads();

  // ---- f = -i [H, rho], RK4 stage update, next drho gather ----------------
  if (t < nb2) {
    const int n = t / nb, m = t % nb;
    double2 c = make_double2(0.0, 0.0);
    for (int l = 0; l < nb; ++l) {
      const double2 hr = cmul(s_h[n * nb + l], s_rho[l * nb + m]);
      const double2 rh = cmul(s_rho[n * nb + l], s_h[l * nb + m]);
      c.x += hr.x - rh.x;
      c.y += hr.y - rh.y;
    }
    const double2 f = make_double2(c.y, -c.x);  // -i c
    const size_t g = kb + t;
    const double2 r0 = sp.rho_n[g];
    double2 next;
    if (sp.stage == 0) {
      sp.acc[g] = f;
      next = make_double2(r0.x + 0.5 * sp.dt * f.x, r0.y + 0.5 * sp.dt * f.y);
    } else if (sp.stage == 1) {
      const double2 a = sp.acc[g];
      sp.acc[g] = make_double2(a.x + 2.0 * f.x, a.y + 2.0 * f.y);
      next = make_double2(r0.x + 0.5 * sp.dt * f.x, r0.y + 0.5 * sp.dt * f.y);
    } else if (sp.stage == 2) {
      const double2 a = sp.acc[g];
      sp.acc[g] = make_double2(a.x + 2.0 * f.x, a.y + 2.0 * f.y);
      next = make_double2(r0.x + sp.dt * f.x, r0.y + sp.dt * f.y);
    } else {
      const double2 a = sp.acc[g];
      const double w = sp.dt / 6.0;
      next = make_double2(r0.x + w * (a.x + f.x), r0.y + w * (a.y + f.y));
      sp.rho_n[g] = next;
    }
    sp.rho_s[g] = next;
    int p = -1;
    if (sp.block == TDG_BLOCK_ALL)
      p = t;
    else if (n >= sp.nv && m < sp.nv)
      p = (n - sp.nv) * sp.nv + m;
    if (p >= 0) {
      const double dre = next.x - ((n == m && n < sp.nv) ? 1.0 : 0.0);
      C xv;
      xv.x = (T)dre;
      xv.y = (T)next.y;
      reinterpret_cast<C*>(sp.xnext)[(size_t)b * sp.xstride + (size_t)k * P + p] = xv;
    }
  }
}

// Low-rank projection z_j = sum_i W[j][i] x_i (W = V^H), ROWS rows per block.
template <typename T>
__global__ void __launch_bounds__(THREADS) project_kernel(const void* __restrict__ W, int64_t n, int rank,
                                                          const void* __restrict__ x, int64_t xstride, void* z,
                                                          int64_t zstride, const tdg_field* fields, int step) {
  using C = typename Cx<T>::type;
  const int b = blockIdx.y;
  if (step >= (int64_t)fields[b].nsteps) return;
  __shared__ double s_red[WAVES * 2 * ROWS];
  __shared__ double s_out[2 * ROWS];
  const int r0 = blockIdx.x * ROWS;
  const int nvalid = min(ROWS, rank - r0);
  T ar[ROWS], ai[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) ar[r] = ai[r] = (T)0;
  rows_dot(reinterpret_cast<const C*>(W) + (int64_t)r0 * n, n, nvalid, (int)n,
           reinterpret_cast<const C*>(x) + (size_t)b * xstride, ar, ai);
  block_reduce<T>(ar, ai, s_red, s_out);
  if (threadIdx.x < nvalid) {
    C v;
    v.x = (T)s_out[2 * threadIdx.x];
    v.y = (T)s_out[2 * threadIdx.x + 1];
    reinterpret_cast<C*>(z)[(size_t)b * zstride + r0 + threadIdx.x] = v;
  }
}

// rho_n <- rho_eq (optional), rho_s <- rho_n, x <- (rho_n - rho_eq)[pairs].
template <typename T>
__global__ void init_kernel(double2* rho_n, double2* rho_s, void* x, int64_t xstride, int nk, int nb, int nv,
                            int npair, int block, int init_eq) {
  using C = typename Cx<T>::type;
  const int k = blockIdx.x, b = blockIdx.y, t = threadIdx.x, nb2 = nb * nb;
  if (t >= nb2) return;
  const int n = t / nb, m = t % nb;
  const size_t g = ((size_t)b * nk + k) * nb2 + t;
  const double occ = (n == m && n < nv) ? 1.0 : 0.0;
  double2 r = init_eq ? make_double2(occ, 0.0) : rho_n[g];
  rho_n[g] = r;
  rho_s[g] = r;
  int p = -1;
  if (block == TDG_BLOCK_ALL)
    p = t;
  else if (n >= nv && m < nv)
    p = (n - nv) * nv + m;
  if (p >= 0) {
    C xv;
    xv.x = (T)(r.x - occ);
    xv.y = (T)r.y;
    reinterpret_cast<C*>(x)[(size_t)b * xstride + (size_t)k * npair + p] = xv;
  }
}

// Observables of an arbitrary state (tdg_observables).
__global__ void obs_state_kernel(StageParams sp) {
  const int k = blockIdx.x, b = blockIdx.y;
  __shared__ double2 s_rho[NB2_MAX];
  __shared__ double s_obs[5][NB2_MAX];
  const int nb2 = sp.nb * sp.nb;
  if (threadIdx.x < nb2) s_rho[threadIdx.x] = sp.rho_s[((size_t)b * sp.nk + k) * nb2 + threadIdx.x];
  __syncthreads();
  per_k_observables(sp, s_rho, s_obs, sp.fields[b], k, b);
}

// Fixed-order reduction of per-k observables: sums (P, J, occ) / nk and
// maxima (tr, herm), for steps step0 .. step0 + gridDim.x - 1.
__global__ void __launch_bounds__(THREADS) obs_reduce_kernel(const double* __restrict__ part, int nk, int batch,
                                                             int step0, const tdg_field* fields, tdg_obs obs,
                                                             double* out5) {
  const int slot = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  const int step = step0 + slot;
  if (out5 == nullptr && step > (int64_t)fields[b].nsteps) return;
  __shared__ double s[5][THREADS];
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const double* p = part + ((size_t)slot * batch + b) * (size_t)nk * 5;
  for (int k = t; k < nk; k += THREADS) {
    const double* q = p + (size_t)k * 5;
    a[0] += q[0];
    a[1] += q[1];
    a[2] += q[2];
    for (int c = 3; c < 5; ++c)
      if (q[c] > a[c] || q[c] != q[c]) a[c] = q[c];
  }
  for (int c = 0; c < 5; ++c) s[c][t] = a[c];
  __syncthreads();
  for (int w = THREADS / 2; w > 0; w >>= 1) {
    if (t < w) {
      for (int c = 0; c < 3; ++c) s[c][t] += s[c][t + w];
      for (int c = 3; c < 5; ++c) {
        const double o = s[c][t + w];
        if (o > s[c][t] || o != o) s[c][t] = o;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const double inv = 1.0 / (double)nk;
    if (out5) {
      double* o = out5 + (size_t)b * 5;
      o[0] = s[0][0] * inv;
      o[1] = s[1][0] * inv;
      o[2] = s[2][0] * inv;
      o[3] = s[3][0];
      o[4] = s[4][0];
    } else {
      const size_t i = (size_t)b * obs.stride + step;
      obs.P[i] = s[0][0] * inv;
      obs.J[i] = s[1][0] * inv;
      obs.occ[i] = s[2][0] * inv;
      if (obs.tr) obs.tr[i] = s[3][0];
      if (obs.herm) obs.herm[i] = s[4][0];
    }
  }
}

}  // namespace

using namespace tdg;

static int validate_fields(tdg_ctx ctx, const tdg_field* fields, int batch, int64_t* max_steps) {
  if (!fields) return fail(ctx, TDG_E_INVAL, "fields is NULL");
  if (batch < 1 || batch > 65535) return fail(ctx, TDG_E_INVAL, "batch = %d outside [1, 65535]", batch);
  int64_t mx = 0;
  for (int b = 0; b < batch; ++b) {
    const tdg_field& f = fields[b];
    if (!(f.tau > 0.0)) return fail(ctx, TDG_E_INVAL, "instance %d: tau must be positive", b);
    if (!(f.nsteps >= 0.0) || f.nsteps != std::floor(f.nsteps) || f.nsteps > 2e9)
      return fail(ctx, TDG_E_INVAL, "instance %d: nsteps must be a non-negative integer", b);
    if (!std::isfinite(f.e0) || !std::isfinite(f.omega) || !std::isfinite(f.t0) || !std::isfinite(f.ex) ||
        !std::isfinite(f.ey))
      return fail(ctx, TDG_E_INVAL, "instance %d: non-finite field parameter", b);
    mx = std::max(mx, (int64_t)f.nsteps);
  }
  *max_steps = mx;
  return TDG_OK;
}

static int upload_fields(tdg_ctx ctx, const tdg_field* fields, int batch, tdg_field** dev) {
  void* p = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_FIELDS, sizeof(tdg_field) * batch, &p));
  TDG_TRY(hip_check(ctx, hipMemcpyAsync(p, fields, sizeof(tdg_field) * batch, hipMemcpyHostToDevice, ctx->stream),
                    "field upload"));
  // the host array need not outlive this call
  TDG_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "field upload sync"));
  *dev = (tdg_field*)p;
  return TDG_OK;
}

extern "C" int tdg_propagate(tdg_ctx ctx, const tdg_operator* op, const tdg_model* model, const tdg_field* fields,
                             int32_t batch, double dt, void* rho, int32_t init_eq, const tdg_obs* obs) {
  if (!ctx) return TDG_E_INVAL;
  TDG_TRY(validate_model(ctx, model));
  if (!op) return fail(ctx, TDG_E_INVAL, "operator is NULL");
  if (op->dtype != TDG_C128 && op->dtype != TDG_C64) return fail(ctx, TDG_E_INVAL, "operator dtype %d", op->dtype);
  const int npair = pairs_per_k(model, op->block);
  if (npair <= 0) return fail(ctx, TDG_E_INVAL, "unknown block %d", op->block);
  const int nk = model->nk1 * model->nk2;
  const int64_t n = (int64_t)nk * npair;
  if (op->n != n) return fail(ctx, TDG_E_INVAL, "operator n = %lld, model gives N = %lld", (long long)op->n, (long long)n);
  if (n > (int64_t)1 << 30) return fail(ctx, TDG_E_UNSUPPORTED, "N = %lld too large", (long long)n);
  const size_t elt = op->dtype == TDG_C128 ? 16 : 8;
  const void* A = nullptr;
  int64_t lda = 0;
  int ncols = 0;
  if (op->kind == TDG_OP_DENSE) {
    if (!op->K) return fail(ctx, TDG_E_INVAL, "dense operator without K");
    if (op->ld < n) return fail(ctx, TDG_E_INVAL, "K ld = %lld < N", (long long)op->ld);
    A = op->K;
    lda = op->ld;
    ncols = (int)n;
  } else if (op->kind == TDG_OP_LOWRANK) {
    if (!op->kdiag || !op->us || !op->w) return fail(ctx, TDG_E_INVAL, "low-rank operator with NULL factor");
    if (op->rank < 1 || op->rank > n) return fail(ctx, TDG_E_INVAL, "rank %lld outside [1, N]", (long long)op->rank);
    A = op->us;
    lda = op->rank;
    ncols = (int)op->rank;
  } else {
    return fail(ctx, TDG_E_INVAL, "operator kind %d", op->kind);
  }
  if (((uintptr_t)A | (uintptr_t)op->kdiag | (uintptr_t)op->w) & (elt == 16 ? 15 : 7))
    return fail(ctx, TDG_E_INVAL, "operator arrays must be aligned to their complex element size");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, TDG_E_INVAL, "dt must be positive");
  if (!rho || ((uintptr_t)rho & 15)) return fail(ctx, TDG_E_INVAL, "rho NULL or not 16-byte aligned");
  int64_t max_steps = 0;
  TDG_TRY(validate_fields(ctx, fields, batch, &max_steps));
  if (!obs || !obs->P || !obs->J || !obs->occ) return fail(ctx, TDG_E_INVAL, "observable arrays are NULL");
  if (obs->stride < max_steps + 1)
    return fail(ctx, TDG_E_INVAL, "obs stride %lld < max nsteps + 1 = %lld", (long long)obs->stride,
                (long long)(max_steps + 1));
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));

  const int nb2 = model->nb * model->nb;
  const size_t state_bytes = (size_t)batch * nk * nb2 * sizeof(double2);
  const int64_t xstride = (n + 1) & ~int64_t(1);
  const int64_t zstride = (op->rank + 1) & ~int64_t(1);
  void *rho_s, *acc, *x0, *x1, *z = nullptr, *part;
  TDG_TRY(ws_reserve(ctx, WS_RHO_S, state_bytes, &rho_s));
  TDG_TRY(ws_reserve(ctx, WS_ACC, state_bytes, &acc));
  TDG_TRY(ws_reserve(ctx, WS_X0, (size_t)batch * xstride * elt, &x0));
  TDG_TRY(ws_reserve(ctx, WS_X1, (size_t)batch * xstride * elt, &x1));
  if (op->kind == TDG_OP_LOWRANK) TDG_TRY(ws_reserve(ctx, WS_Z, (size_t)batch * zstride * elt, &z));
  const size_t part_per_step = (size_t)batch * nk * 5 * sizeof(double);
  int chunk = (int)std::min<size_t>(256, std::max<size_t>(1, OBS_PART_BUDGET / part_per_step));
  TDG_TRY(ws_reserve(ctx, WS_OBS_PART, part_per_step * chunk, &part));
  tdg_field* dfields = nullptr;
  TDG_TRY(upload_fields(ctx, fields, batch, &dfields));

  const dim3 kgrid(nk, batch);
  const int init_threads = ((nb2 + 63) / 64) * 64;
  if (op->dtype == TDG_C128)
    hipLaunchKernelGGL(init_kernel<double>, kgrid, dim3(init_threads), 0, ctx->stream, (double2*)rho, (double2*)rho_s,
                       x0, xstride, nk, model->nb, model->nv, npair, op->block, init_eq);
  else
    hipLaunchKernelGGL(init_kernel<float>, kgrid, dim3(init_threads), 0, ctx->stream, (double2*)rho, (double2*)rho_s,
                       x0, xstride, nk, model->nb, model->nv, npair, op->block, init_eq);
  TDG_TRY(launch_check(ctx, "init launch"));

  StageParams sp;
  sp.A = A;
  sp.lda = lda;
  sp.ncols = ncols;
  sp.kdiag = op->kind == TDG_OP_LOWRANK ? op->kdiag : nullptr;
  sp.xstride = xstride;
  sp.rho_n = (double2*)rho;
  sp.rho_s = (double2*)rho_s;
  sp.acc = (double2*)acc;
  sp.eps = model->eps;
  sp.dip = (const double2*)model->dip;
  sp.vel = (const double2*)model->vel;
  sp.fields = dfields;
  sp.obs_part = (double*)part;
  sp.nk = nk;
  sp.nb = model->nb;
  sp.nv = model->nv;
  sp.npair = npair;
  sp.block = op->block;
  sp.batch = batch;
  sp.dt = dt;
  tdg_obs ob = *obs;

  void* xc = x0;
  void* xn = x1;
  int slot = 0;
  int64_t chunk_start = 0;
  const dim3 pgrid((unsigned)((op->rank + ROWS - 1) / ROWS), batch);
  for (int64_t step = 0; step <= max_steps; ++step) {
    for (int s = 0; s < 4; ++s) {
      if (step == max_steps && s > 0) break;
      if (op->kind == TDG_OP_LOWRANK && step < max_steps) {
        prof_begin(ctx, TDG_KCLASS_PROJECT);
        if (op->dtype == TDG_C128)
          hipLaunchKernelGGL(project_kernel<double>, pgrid, dim3(THREADS), 0, ctx->stream, op->w, n, (int)op->rank,
                             xc, xstride, z, zstride, dfields, (int)step);
        else
          hipLaunchKernelGGL(project_kernel<float>, pgrid, dim3(THREADS), 0, ctx->stream, op->w, n, (int)op->rank,
                             xc, xstride, z, zstride, dfields, (int)step);
        prof_end(ctx, TDG_KCLASS_PROJECT);
      }
      sp.vec = op->kind == TDG_OP_LOWRANK ? z : xc;
      sp.vstride = op->kind == TDG_OP_LOWRANK ? zstride : xstride;
      sp.xcur = xc;
      sp.xnext = xn;
      sp.step = (int)step;
      sp.stage = s;
      sp.obs_slot = slot;
      prof_begin(ctx, TDG_KCLASS_STAGE);
      if (op->dtype == TDG_C128)
        hipLaunchKernelGGL(stage_kernel<double>, kgrid, dim3(THREADS), 0, ctx->stream, sp);
      else
        hipLaunchKernelGGL(stage_kernel<float>, kgrid, dim3(THREADS), 0, ctx->stream, sp);
      prof_end(ctx, TDG_KCLASS_STAGE);
      std::swap(xc, xn);
    }
    ++slot;
    if (slot == chunk || step == max_steps) {
      hipLaunchKernelGGL(obs_reduce_kernel, dim3(slot, batch), dim3(THREADS), 0, ctx->stream, (const double*)part, nk,
                         batch, (int)chunk_start, dfields, ob, (double*)nullptr);
      chunk_start += slot;
      slot = 0;
    }
    if ((step & 63) == 0) TDG_TRY(launch_check(ctx, "propagation launch"));
  }
  return launch_check(ctx, "propagation launch");
}

extern "C" int tdg_observables(tdg_ctx ctx, const tdg_model* model, const void* rho, int32_t batch,
                               const tdg_field* fields, double* out) {
  if (!ctx) return TDG_E_INVAL;
  TDG_TRY(validate_model(ctx, model));
  if (!rho || ((uintptr_t)rho & 15) || !out) return fail(ctx, TDG_E_INVAL, "rho or out NULL / misaligned");
  int64_t mx = 0;
  TDG_TRY(validate_fields(ctx, fields, batch, &mx));
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
  const int nk = model->nk1 * model->nk2;
  void* part = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_OBS_PART, (size_t)batch * nk * 5 * sizeof(double), &part));
  tdg_field* dfields = nullptr;
  TDG_TRY(upload_fields(ctx, fields, batch, &dfields));
  StageParams sp = {};
  sp.rho_s = (double2*)rho;
  sp.dip = (const double2*)model->dip;
  sp.vel = (const double2*)model->vel;
  sp.fields = dfields;
  sp.obs_part = (double*)part;
  sp.obs_slot = 0;
  sp.nk = nk;
  sp.nb = model->nb;
  sp.nv = model->nv;
  sp.batch = batch;
  hipLaunchKernelGGL(obs_state_kernel, dim3(nk, batch), dim3(64), 0, ctx->stream, sp);
  TDG_TRY(launch_check(ctx, "observables launch"));
  tdg_obs none = {};
  hipLaunchKernelGGL(obs_reduce_kernel, dim3(1, batch), dim3(THREADS), 0, ctx->stream, (const double*)part, nk, batch,
                     0, dfields, none, out);
  return launch_check(ctx, "observables reduce launch");
}

extern "C" int tdg_check_numeric(tdg_ctx ctx, const tdg_obs* obs, int32_t batch, const tdg_field* fields,
                                 double tr_tol, double herm_tol) {
  if (!ctx) return TDG_E_INVAL;
  if (!obs || !obs->P || !obs->J || !obs->occ) return fail(ctx, TDG_E_INVAL, "observable arrays are NULL");
  int64_t mx = 0;
  TDG_TRY(validate_fields(ctx, fields, batch, &mx));
  if (obs->stride < mx + 1) return fail(ctx, TDG_E_INVAL, "obs stride too small");
  TDG_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "check sync"));
  const size_t cnt = (size_t)batch * obs->stride;
  std::vector<double> h(cnt);
  double* arrs[5] = {obs->P, obs->J, obs->occ, obs->tr, obs->herm};
  const char* names[5] = {"P", "J", "occ", "trace deviation", "Hermiticity residual"};
  for (int a = 0; a < 5; ++a) {
    if (!arrs[a]) continue;
    TDG_TRY(hip_check(ctx, hipMemcpy(h.data(), arrs[a], cnt * sizeof(double), hipMemcpyDeviceToHost), "check copy"));
    const double tol = a == 3 ? tr_tol : (a == 4 ? herm_tol : INFINITY);
    for (int b = 0; b < batch; ++b)
      for (int64_t s = 0; s <= (int64_t)fields[b].nsteps; ++s) {
        const double v = h[(size_t)b * obs->stride + s];
        if (!std::isfinite(v) || std::fabs(v) > tol)
          return fail(ctx, TDG_E_NUMERIC, "%s = %g at instance %d, step %lld", names[a], v, b, (long long)s);
      }
  }
  return TDG_OK;
}
