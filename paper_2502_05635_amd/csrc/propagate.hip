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
// Every global load a block needs is issued before its first use, so a
// block's lifetime is about one memory round trip plus on-chip work.
// Observables of rho(t_n) are formed per k in the first stage of step n and
// reduced over k in fixed order by a separate kernel every few steps.
//
// Instances are integrated in order of decreasing length: the host sorts
// them, so at every step the instances still running are a prefix and the
// grid covers exactly those.  The working state lives in that sorted order
// and is scattered back to the caller's order at the end.
#include <algorithm>
#include <functional>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include <hip/hip_ext.h>

#include "bf16x2.h"
#include "xcd.h"
#include "covariant.h"
#include "internal.h"

// operand types of the direct-to-LDS load builtin: a global source, an LDS destination
typedef __attribute__((address_space(1))) void lds_dma_src;
typedef __attribute__((address_space(3))) void lds_dma_dst;
// s_waitcnt immediate for vmcnt(0) alone (gfx9 encoding: vmcnt in bits 3:0 and
// 15:14 = 0, expcnt in 6:4 and lgkmcnt in 11:8 at their maxima, i.e. no wait)
constexpr int WAIT_VMCNT0 = 0x0F70;

namespace {

constexpr int THREADS = 256;  // dense stage kernel and auxiliary kernels
constexpr int NB2_MAX = TDG_NB_MAX * TDG_NB_MAX;
constexpr int ROWS = 4;  // kernel rows contracted together (shared drho loads)
constexpr int ZSPLIT_MAX = 4;  // low rank: largest number of projection column slices
constexpr int PROJ_THREADS = 256;
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

// E_b at the four stage times of steps step0 .. step0 + count - 1, as
// tab[(slot * batch + b) * 4 + stage].  The stage kernels load their value
// instead of evaluating exp and cos (a long dependent FP64 chain) at the end
// of their critical path.
__global__ void field_table_kernel(const tdg_field* __restrict__ fields, int batch, int step0, int count, double dt,
                                   double* __restrict__ tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count * batch * 4) return;
  const int s = i & 3, b = (i >> 2) % batch, slot = (i >> 2) / batch;
  const double cs = (s == 0) ? 0.0 : (s == 3 ? 1.0 : 0.5);
  tab[i] = field_value(fields[b], (double)(step0 + slot) * dt + cs * dt);
}

// Host records copied to the device inside kernel arguments: the launch takes
// its own copy of the arguments, so nothing waits for the copy and the host
// array may go away as soon as the launch is queued.
constexpr int ARG_WORDS = 512;  // 2 KiB of payload per launch
struct ArgPayload {
  uint32_t w[ARG_WORDS];
};
__global__ void __launch_bounds__(256) arg_copy_kernel(ArgPayload p, uint32_t* __restrict__ dst, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = p.w[i];
}

// Barrier for the per-k epilogue, which only the block's first wave runs
// (nb^2 <= 64 elements): wave-level ordering of its LDS accesses.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- row dot products ------------------------------------------------------
// acc_r = sum_j A[r][j] x[j] for r < nvalid (rows lda apart), this thread's
// share of the columns; the block reduction below completes the sums.  The
// column loop is unrolled UNROLL times with all loads issued before the
// arithmetic, so each wave keeps UNROLL * (ROWS + 1) 16-byte loads in flight.
template <int NT, int UNROLL>
__device__ inline void rows_dot(const float2* __restrict__ A, int64_t lda, int nvalid, int ncols,
                                const float2* __restrict__ x, float (&ar)[ROWS], float (&ai)[ROWS]) {
  if (((lda | (int64_t)(uintptr_t)A / 8 | (int64_t)(uintptr_t)x / 8) & 1) == 0) {
    // two complex numbers per 16-byte load
    const int npair = ncols >> 1;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    for (int j0 = threadIdx.x; j0 < npair; j0 += NT * UNROLL) {
      float4 xv[UNROLL], a[UNROLL][ROWS];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int j = j0 + u * NT;
        if (j < npair) {
          xv[u] = x4[j];
#pragma unroll
          for (int r = 0; r < ROWS; ++r)
            if (r < nvalid) a[u][r] = reinterpret_cast<const float4*>(A + r * lda)[j];
        }
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        if (j0 + u * NT < npair) {
#pragma unroll
          for (int r = 0; r < ROWS; ++r) {
            if (r < nvalid) {
              ar[r] += a[u][r].x * xv[u].x - a[u][r].y * xv[u].y + a[u][r].z * xv[u].z - a[u][r].w * xv[u].w;
              ai[r] += a[u][r].x * xv[u].y + a[u][r].y * xv[u].x + a[u][r].z * xv[u].w + a[u][r].w * xv[u].z;
            }
          }
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
    for (int j = threadIdx.x; j < ncols; j += NT) {
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

template <int NT, int UNROLL>
__device__ inline void rows_dot(const double2* __restrict__ A, int64_t lda, int nvalid, int ncols,
                                const double2* __restrict__ x, double (&ar)[ROWS], double (&ai)[ROWS]) {
  for (int j0 = threadIdx.x; j0 < ncols; j0 += NT * UNROLL) {
    double2 xv[UNROLL], a[UNROLL][ROWS];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int j = j0 + u * NT;
      if (j < ncols) {
        xv[u] = x[j];
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
          if (r < nvalid) a[u][r] = A[r * lda + j];
      }
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      if (j0 + u * NT < ncols) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          if (r < nvalid) {
            ar[r] += a[u][r].x * xv[u].x - a[u][r].y * xv[u].y;
            ai[r] += a[u][r].x * xv[u].y + a[u][r].y * xv[u].x;
          }
        }
      }
    }
  }
}

// One 32-bit word of lane l ^ 1, l ^ 2 (quad permutes), of the mirrored lane
// in the 8-lane half row, or of the mirrored lane in the 16-lane row (DPP).
template <int CTRL>
__device__ inline int dpp_word(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(dpp_word<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_word<CTRL>((int)(b & 0xffffffffLL)), hi = dpp_word<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float lane_value(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ inline double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum of v over the 64 lanes of a full wave, returned to every lane: within
// each 16-lane row by four DPP steps (quad permutes [1,0,3,2] and [2,3,0,1],
// half-row mirror, row mirror), then the four row sums in row order.
template <typename T>
__device__ inline T wave_sum(T v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}

// Sum each thread's ROWS complex partials over the block; out[2r], out[2r+1]
// receive row r (as double).  Wave sums (every lane of the block calls it),
// then a fixed-order sum over waves.
template <typename T, int NT>
__device__ inline void block_reduce(T (&ar)[ROWS], T (&ai)[ROWS], double* red, double* out) {
  constexpr int WAVES = NT / 64;
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    ar[r] = wave_sum(ar[r]);
    ai[r] = wave_sum(ai[r]);
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
  const void* vec;    // contracted vector per instance: drho gather (dense) or z slices (low rank)
  int64_t vstride;
  int zsplit;         // low rank: number of projection column slices summed by the stage kernel
  int64_t zsplit_stride;  // elements between consecutive slices of z
  const void* kdiag;  // low rank: K_diag [N]; dense: NULL
  const void* chS;    // channel-wise: off-diagonal channel factors S, row (k, p) = [(P-1) rmax]
  int chLS;           // channel-wise: (P-1) rmax
  const void* xcur;   // drho gather of this stage [B][xstride]
  void* xnext;        // drho gather of the next stage
  int64_t xstride;
  double2* rho_n;     // rho(t_n), sorted instance order [B][nk][nb][nb]
  double2* rho_s;     // state of this stage
  double2* acc;       // RK4 sum of stage derivatives
  const double* eps;
  const double2* dip;
  const double2* vel;
  const tdg_field* fields;  // sorted instance order
  double* obs_part;   // [slot][B][nk][5] or NULL
  int obs_slot;
  int nk, nb, nv, npair, block, batch;
  int n_dyn;          // blocks with blockIdx.y < n_dyn integrate; the others only record observables
  int step, stage;
  double dt;
  double2* rho_s_out;    // where the next stage state goes: rho_s itself, or (with links) the other buffer
  const double2* links;  // intraband term: links L_a(k) [2][nk][nb][nb], the covariant difference of
                         // rho_s formed in the epilogue from the neighbours' states; NULL = none
  int nk1, nk2;
  double cov_c1, cov_c2;  // 1 / (2 |b_a|) per grid axis
  int tr_signed;          // per-k trace partial signed (summed over k) instead of |.| (maximised)
  const double* ftab;     // field at the stage times, [obs slot][B][4] (field_table_kernel)
};

// Per-k observables of s_rho (LDS) into obs_part; de, ve are this thread's
// element of e.d and e.v (threads t < nb^2 participate).  Called by the first
// wave of a block only.
__device__ inline void obs_partial(const StageParams& sp, const double2* s_rho, double (*s_obs)[NB2_MAX],
                                   double2 de, double2 ve, int k, int b) {
  const int nb = sp.nb, nb2 = nb * nb, t = threadIdx.x;
  if (t < nb2) {
    const int n = t / nb, m = t % nb;
    const double2 rmn = s_rho[m * nb + n];
    const double2 rnm = s_rho[t];
    s_obs[0][t] = de.x * rmn.x - de.y * rmn.y;  // Re(d_nm rho_mn)
    s_obs[1][t] = ve.x * rmn.x - ve.y * rmn.y;
    s_obs[2][t] = (n == m && n == sp.nv) ? rnm.x : 0.0;
    s_obs[3][t] = (n == m) ? rnm.x : 0.0;
    const double hx = rnm.x - rmn.x, hy = rnm.y + rmn.y;
    s_obs[4][t] = sqrt(hx * hx + hy * hy);
  }
  wave_sync();
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
    o[3] = sp.tr_signed ? o[3] - (double)sp.nv : fabs(o[3] - (double)sp.nv);
    double* dst = sp.obs_part + (((size_t)sp.obs_slot * sp.batch + b) * sp.nk + k) * 5;
    for (int c = 0; c < 5; ++c) dst[c] = o[c];
  }
}

__device__ inline double2 proj_e(double ex, double ey, double2 a, double2 b) {
  return make_double2(ex * a.x + ey * b.x, ex * a.y + ey * b.y);
}
__device__ inline double2 proj_e(const tdg_field& F, double2 a, double2 b) { return proj_e(F.ex, F.ey, a, b); }

// Stage kernel: one block per (k point, instance).  LOWRANK selects the
// low-rank expansion (rows of S against z, plus K_diag o x); it is a template
// parameter so the two paths are distinct kernels in traces.  NT threads per
// block (a k point's rows are split over the block's columns), U-fold unrolled
// row streams (low rank: 2 U columns of S per thread and pass), WPE = minimum
// waves per SIMD requested from the compiler.
template <typename T, int MODE, int NT, int U, int WPE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
stage_kernel(StageParams sp) {
  using C = typename Cx<T>::type;
  constexpr bool LOWRANK = MODE == 1, CHANNEL = MODE == 2;
  constexpr int WAVES = NT / 64;
  const int k = blockIdx.x, b = blockIdx.y;
  const bool dyn = b < sp.n_dyn;
  const int nb = sp.nb, nb2 = nb * nb, P = sp.npair, t = threadIdx.x;
  const size_t kb = ((size_t)b * sp.nk + k) * nb2;
  const size_t base = (size_t)k * nb2 + t;
  const size_t plane = (size_t)sp.nk * nb2;

  __shared__ double2 s_rho[NB2_MAX];
  __shared__ double2 s_h[NB2_MAX];
  __shared__ double s_y[2 * NB2_MAX + 2 * ROWS];
  __shared__ double s_red[WAVES * 2 * ROWS];
  __shared__ double s_obs[5][NB2_MAX];
  // intraband term: entry (4 a + w) nb^2 + e holds element e of, for axis a,
  // w = 0: y(k + b_a), 1: y(k - b_a), 2: L_a(k), 3: L_a(k - b_a)
  __shared__ __align__(16) double2 s_cov[8 * NB2_MAX];

  // ---- loads: the low-rank kernel issues every load of the block before any
  // use (its lifetime is latency-bound); the dense kernel loads the per-k
  // state after its row stream (bandwidth-bound, registers kept for the stream)
  double2 r_s = make_double2(0.0, 0.0), r_n = r_s, r_acc = r_s, d0 = r_s, d1 = r_s, v0 = r_s, v1 = r_s;
  double e_nn = 0.0;
  auto load_state = [&]() {
    if (t < nb2) {
      r_s = sp.rho_s[kb + t];
      d0 = sp.dip[base];
      d1 = sp.dip[plane + base];
      if (sp.stage == 0) {
        v0 = sp.vel[base];
        v1 = sp.vel[plane + base];
      }
      if (dyn) {
        r_n = sp.rho_n[kb + t];
        if (sp.stage != 0) r_acc = sp.acc[kb + t];
        if (t / nb == t % nb) e_nn = sp.eps[(size_t)k * nb + t / nb];
      }
    }
  };
  // E(t) of this stage and the polarisation, for the epilogue only, read by
  // vector loads issued after the state loads.  As scalar loads they formed a
  // pointer chase (argument, table, value) ahead of the first vector load, and
  // scalar loads complete out of order, so each use waited for all of them.
  // The offset is a zero held in a vector register, opaque to the compiler,
  // which then cannot treat the addresses as uniform.
  double ef = 0.0, fex = 0.0, fey = 0.0;
  auto load_field = [&]() {
    int vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    fex = (&sp.fields[b].ex)[vzero];
    fey = (&sp.fields[b].ey)[vzero];
    if (dyn) ef = sp.ftab[((size_t)sp.obs_slot * sp.batch + b) * 4 + sp.stage + vzero];
  };
  // intraband term: the first wave copies the neighbours' state elements and
  // the links into LDS with direct-to-LDS loads issued now (lane l of the copy
  // starting at entry c0 writes entry c0 + l); nothing is held in registers,
  // and the epilogue waits for them before reading.  The states are read from
  // rho_s while this kernel writes the next stage state to the other buffer.
  if (sp.links && dyn && t < 64) {
    const int count = 8 * nb2;
    for (int c0 = 0; c0 < count; c0 += 64) {
      const int i = c0 + t;
      if (i < count) {
        const int q = i / nb2, e = i - q * nb2, a = q >> 2, w = q & 3;
        int kf, kr;
        tdg::covariant_neighbours(k, a, sp.nk1, sp.nk2, kf, kr);
        const double2* src = w == 0   ? sp.rho_s + ((size_t)b * sp.nk + kf) * nb2 + e
                             : w == 1 ? sp.rho_s + ((size_t)b * sp.nk + kr) * nb2 + e
                             : w == 2 ? sp.links + ((size_t)a * sp.nk + k) * nb2 + e
                                      : sp.links + ((size_t)a * sp.nk + kr) * nb2 + e;
        __builtin_amdgcn_global_load_lds((lds_dma_src*)src, (lds_dma_dst*)(s_cov + c0), 16, 0, 0);
      }
    }
  }
  if (LOWRANK) {
    load_state();
    load_field();
  }
  const C* A = reinterpret_cast<const C*>(sp.A);
  const C* vec = reinterpret_cast<const C*>(sp.vec) + (size_t)b * sp.vstride;
  const C* xcur = reinterpret_cast<const C*>(sp.xcur) + (size_t)b * sp.xstride;
  C kd_t, x_t;
  if (LOWRANK && dyn && t < P) {
    kd_t = reinterpret_cast<const C*>(sp.kdiag)[(size_t)k * P + t];
    x_t = xcur[(size_t)k * P + t];
  }

  // ---- contraction: y_p = sum_j A[k P + p][j] vec[j] ----------------------
  if (CHANNEL && dyn) {
    // pair p of k: its diagonal channel's row k against x_p (channel-major
    // drho), plus its off-diagonal channels' S rows against z_p
    const C* S = reinterpret_cast<const C*>(sp.chS);
    for (int p = 0; p < P; ++p) {
      T ar[ROWS], ai[ROWS];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) ar[r] = ai[r] = (T)0;
      rows_dot<NT, U>(A + ((int64_t)p * sp.nk + k) * sp.lda, sp.lda, 1, sp.ncols, xcur + (size_t)p * sp.nk, ar, ai);
      rows_dot<NT, U>(S + ((int64_t)k * P + p) * sp.chLS, sp.chLS, 1, sp.chLS, vec + (size_t)p * sp.chLS, ar, ai);
      block_reduce<T, NT>(ar, ai, s_red, s_y + 2 * p);
    }
  } else if (dyn) {
    for (int r0 = 0; r0 < P; r0 += ROWS) {
      const int nvalid = min(ROWS, P - r0);
      T ar[ROWS], ai[ROWS];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) ar[r] = ai[r] = (T)0;
      const C* Ar = A + ((int64_t)k * P + r0) * sp.lda;
      if (LOWRANK) {
        // rows of S against z = sum of the projection's column slices (at most
        // ZSPLIT_MAX); each thread sums the slices of its own columns.  2 U
        // columns per thread and pass, every load of the pass issued first.
        constexpr int CP = 2 * U;
        for (int j0 = t; j0 < sp.ncols; j0 += CP * NT) {
          C zv[CP][ZSPLIT_MAX], av[CP][ROWS];
#pragma unroll
          for (int u = 0; u < CP; ++u) {
            const int j = j0 + u * NT;
            if (j < sp.ncols) {
#pragma unroll
              for (int q = 0; q < ZSPLIT_MAX; ++q)
                if (q < sp.zsplit) zv[u][q] = vec[(size_t)q * sp.zsplit_stride + j];
#pragma unroll
              for (int r = 0; r < ROWS; ++r)
                if (r < nvalid) av[u][r] = Ar[r * sp.lda + j];
            }
          }
#pragma unroll
          for (int u = 0; u < CP; ++u) {
            if (j0 + u * NT < sp.ncols) {
              T zr = (T)0, zi = (T)0;
#pragma unroll
              for (int q = 0; q < ZSPLIT_MAX; ++q)
                if (q < sp.zsplit) {
                  zr += zv[u][q].x;
                  zi += zv[u][q].y;
                }
#pragma unroll
              for (int r = 0; r < ROWS; ++r) {
                if (r < nvalid) {
                  ar[r] += av[u][r].x * zr - av[u][r].y * zi;
                  ai[r] += av[u][r].x * zi + av[u][r].y * zr;
                }
              }
            }
          }
        }
      } else {
        rows_dot<NT, U>(Ar, sp.lda, nvalid, sp.ncols, vec, ar, ai);
      }
      block_reduce<T, NT>(ar, ai, s_red, s_y + 2 * r0);
    }
  }
  if (!LOWRANK) {
    load_state();
    load_field();
  }
  // the per-k epilogue runs in the first wave (nb^2 <= 64 elements, P <= 64 pairs)
  if (t >= 64) return;
  // the direct-to-LDS copies of the intraband neighbours have landed once
  // this wave's vector memory counter is zero
  if (sp.links && dyn) __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
  if (t < nb2) s_rho[t] = r_s;
  wave_sync();
  if (sp.stage == 0 && sp.obs_part)
    obs_partial(sp, s_rho, s_obs, proj_e(fex, fey, d0, d1), proj_e(fex, fey, v0, v1), k, b);
  if (!dyn) return;                              // final time of this instance: observables only
  if (LOWRANK && t < P) {
    const T re = kd_t.x * x_t.x - kd_t.y * x_t.y, im = kd_t.x * x_t.y + kd_t.y * x_t.x;
    s_y[2 * t] += (double)re;
    s_y[2 * t + 1] += (double)im;
  }
  wave_sync();

  // ---- H_k = eps_k + dSigma_k - E(t) e.d_k ----------------------------------
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
    const double2 de = proj_e(fex, fey, d0, d1);
    double2 h = make_double2(ds.x - ef * de.x, ds.y - ef * de.y);
    if (n == m) h.x += e_nn;
    s_h[t] = h;
  }
  wave_sync();

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
    double2 f = make_double2(c.y, -c.x);  // -i c
    const size_t g = kb + t;
    if (sp.links) {
      // intraband part of the field term: -E(t) e.(rho)_{;k}
      double2 dv = make_double2(0.0, 0.0);
      for (int a = 0; a < 2; ++a) {
        const double ea = a == 0 ? fex : fey;
        if (ea == 0.0) continue;
        const double2 *yf = s_cov + (4 * a) * nb2, *yr = yf + nb2, *lf = yr + nb2, *lr = lf + nb2;
        const double2 tt = tdg::covariant_axis_element(
            n, m, nb, sp.nv, [&](int r, int q) { return yf[r * nb + q]; }, [&](int r, int q) { return yr[r * nb + q]; },
            [&](int r, int q) { return lf[r * nb + q]; }, [&](int r, int q) { return lr[r * nb + q]; });
        const double cf = ea * (a == 0 ? sp.cov_c1 : sp.cov_c2);
        dv.x += cf * tt.x;
        dv.y += cf * tt.y;
      }
      f.x -= ef * dv.x;
      f.y -= ef * dv.y;
    }
    double2 next;
    if (sp.stage == 0) {
      sp.acc[g] = f;
      next = make_double2(r_n.x + 0.5 * sp.dt * f.x, r_n.y + 0.5 * sp.dt * f.y);
    } else if (sp.stage == 1) {
      sp.acc[g] = make_double2(r_acc.x + 2.0 * f.x, r_acc.y + 2.0 * f.y);
      next = make_double2(r_n.x + 0.5 * sp.dt * f.x, r_n.y + 0.5 * sp.dt * f.y);
    } else if (sp.stage == 2) {
      sp.acc[g] = make_double2(r_acc.x + 2.0 * f.x, r_acc.y + 2.0 * f.y);
      next = make_double2(r_n.x + sp.dt * f.x, r_n.y + sp.dt * f.y);
    } else {
      const double w = sp.dt / 6.0;
      next = make_double2(r_n.x + w * (r_acc.x + f.x), r_n.y + w * (r_acc.y + f.y));
      sp.rho_n[g] = next;
    }
    sp.rho_s_out[g] = next;
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
      reinterpret_cast<C*>(sp.xnext)[(size_t)b * sp.xstride + (CHANNEL ? (size_t)p * sp.nk + k : (size_t)k * P + p)] =
          xv;
    }
  }
}

// Low-rank projection z_j = sum_i W[j][i] x_i (W = V^H): block (g, q, b) takes
// rows ROWS*g .. ROWS*g + ROWS - 1 over the q-th of zsplit column slices and
// writes its partial to zpart[q][b][j]; the stage kernel sums the slices.
// Channel-wise (ch_ls > 0): W holds the V^H rows of every off-diagonal channel,
// P blocks of ch_ls rows (P - 1 channels of ch_rmax rows each).
template <typename T>
__global__ void __launch_bounds__(PROJ_THREADS) project_kernel(const void* __restrict__ W, int64_t n, int rank,
                                                     const void* __restrict__ x, int64_t xstride, void* zpart,
                                                     int64_t zstride, int64_t slice, int64_t split_stride,
                                                     int ch_ls, int ch_rmax) {
  using C = typename Cx<T>::type;
  const int q = blockIdx.y, b = blockIdx.z;
  if (ch_ls > 0) {
    // channel-wise: rows of the (p, q) block of V^H read x_q (channel-major,
    // n = nk columns per channel); a group of ROWS rows never spans two blocks
    const int pp = (int)(blockIdx.x * ROWS) / ch_ls, slot = ((int)(blockIdx.x * ROWS) % ch_ls) / ch_rmax;
    x = reinterpret_cast<const C*>(x) + (size_t)(slot < pp ? slot : slot + 1) * n;
  }
  __shared__ double s_red[PROJ_THREADS / 64 * 2 * ROWS];
  __shared__ double s_out[2 * ROWS];
  const int r0 = blockIdx.x * ROWS;
  const int nvalid = min(ROWS, rank - r0);
  const int64_t c0 = (int64_t)q * slice;
  const int ncols = (int)max<int64_t>(0, min<int64_t>(slice, n - c0));
  T ar[ROWS], ai[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) ar[r] = ai[r] = (T)0;
  rows_dot<PROJ_THREADS, 8>(reinterpret_cast<const C*>(W) + (int64_t)r0 * n + c0, n, nvalid, ncols,
                            reinterpret_cast<const C*>(x) + (size_t)b * xstride + c0, ar, ai);
  block_reduce<T, PROJ_THREADS>(ar, ai, s_red, s_out);
  if (threadIdx.x < nvalid) {
    C v;
    v.x = (T)s_out[2 * threadIdx.x];
    v.y = (T)s_out[2 * threadIdx.x + 1];
    reinterpret_cast<C*>(zpart)[(size_t)q * split_stride + (size_t)b * zstride + r0 + threadIdx.x] = v;
  }
}

// Working state from the caller's rho: rho_n <- rho_eq or rho[perm[b]],
// rho_s <- rho_n, x <- (rho_n - rho_eq)[pairs]; b is the sorted position.
// x_layout: 0 = [B][xstride] with pair index k P + p; 2 = [B][xstride]
// channel-major, p nk + k.  (The batched path has init_batched_kernel.)
template <typename T>
__global__ void init_kernel(const double2* __restrict__ rho_in, const int* __restrict__ perm, double2* rho_n,
                            double2* rho_s, void* x, int64_t xstride, int nk, int nb, int nv, int npair, int block,
                            int init_eq, int x_layout) {
  using C = typename Cx<T>::type;
  const int k = blockIdx.x, b = blockIdx.y, t = threadIdx.x, nb2 = nb * nb;
  if (t >= nb2) return;
  const int n = t / nb, m = t % nb;
  const size_t g = ((size_t)b * nk + k) * nb2 + t;
  const double occ = (n == m && n < nv) ? 1.0 : 0.0;
  const double2 r = init_eq ? make_double2(occ, 0.0) : rho_in[((size_t)perm[b] * nk + k) * nb2 + t];
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
    const size_t i = x_layout == 2 ? (size_t)p * nk + k : (size_t)k * npair + p;
    reinterpret_cast<C*>(x)[(size_t)b * xstride + i] = xv;
  }
}

// rho[perm[b]] <- rho_n[b]
__global__ void finish_kernel(const double2* __restrict__ rho_n, const int* __restrict__ perm, double2* rho_out,
                              int nk, int nb2) {
  const int k = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  if (t >= nb2) return;
  rho_out[((size_t)perm[b] * nk + k) * nb2 + t] = rho_n[((size_t)b * nk + k) * nb2 + t];
}

// Hermiticity residual of a caller's rho(0): thread i takes the (instance,
// k) block i of nb x nb elements; part[blockIdx.x] = the block's largest
// max_nm |rho_nm - conj rho_mn| (NaN counted as infinite).
__global__ void __launch_bounds__(256) herm_check_kernel(const double2* __restrict__ rho, int64_t nblk, int nb,
                                                         double* __restrict__ part) {
  __shared__ double s[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double h = 0.0;
  if (i < nblk) {
    const double2* r = rho + i * nb * nb;
    for (int n = 0; n < nb; ++n)
      for (int m = n; m < nb; ++m) {
        const double2 a = r[n * nb + m], c = r[m * nb + n];
        const double dx = a.x - c.x, dy = a.y + c.y;
        double v = sqrt(dx * dx + dy * dy);
        if (v != v) v = INFINITY;
        h = fmax(h, v);
      }
  }
  s[threadIdx.x] = h;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// out[0] = max of part[0 .. count)
__global__ void __launch_bounds__(256) max_reduce_kernel(const double* __restrict__ part, int64_t count, double* out) {
  __shared__ double s[256];
  double h = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) h = fmax(h, part[i]);
  s[threadIdx.x] = h;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// ---- batched path: per-k stage after the matrix-core contraction -----------
struct BatchParams {
  const float2* Y;    // contraction result, [slice][N][ldy] (instance fastest)
  int64_t ldy;
  int y_slices;
  int64_t y_slice_stride;
  const float2* kdiag;  // low rank: K_diag [N]; dense: NULL
  const float2* xcur;   // drho gather of this stage, [N][ldx] (read by the unpacked kernel)
  float2* xnext;        // not written by the packed kernel when it writes the split (xexp)
  int64_t ldx;
  double2* rho_n;
  double2* rho_s;
  double2* acc;
  const double* eps;
  const double2* dip;
  const double2* vel;
  const tdg_field* fields;
  double* obs_part;
  int obs_slot;
  int nk, nb, nv, npair, block, batch;
  int n_active;  // instances with blocks in this launch (stage 0: also those at their final time)
  int n_dyn;     // instances that integrate
  int step, stage;
  double dt;
  const int* step_dev;  // graph replays: the step is read here (obs slot = step % chunk); else NULL
  int chunk;
  const double2* intra;  // intraband term e.(rho_s)_{;k} of this stage, laid out as rho_s; NULL = none
  int tr_signed;         // per-k trace partial signed (summed over k) instead of |.| (maximised)
  const double* ftab;    // field at the stage times, [obs slot][B][4] (field_table_kernel)
  // the elements (n nb + m) the stage kernel updates: the upper triangle and
  // diagonal when the state is Hermitian-packed, else all nb^2; pair elements
  // (those that read the product) first.  Thread group g of a block takes
  // entries g, g + nb, g + 2 nb, ...
  int nelem;
  int elist[TDG_NB_MAX * TDG_NB_MAX];
  // the next gather also split for a BF16X2 product of tilings 1 to 4
  // (bf16x2.h layout, Kc = N); NULL = not written.  Used with 64
  // instances per block and a multiple of 4 pairs per k only.
  unsigned short* xexp;
  int64_t ldxb;
};

// The step counter of graph replays (vector stores: the address depends on the lane).
// A fixed non-zero operand for timing the products (the step-0 gather of
// rho_eq is all zeros): values in (-1e-3, 1e-3) from an integer hash of the
// element index, so the matrix cores see varied operands like the propagated ones.
__global__ void pattern_fill_kernel(float2* x, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ (uint32_t)(i >> 32);
    h ^= h >> 16; h *= 0x85EBCA6Bu; h ^= h >> 13; h *= 0xC2B2AE35u; h ^= h >> 16;
    const float re = ((float)(h & 0xFFFFu) - 32767.5f) * (1e-3f / 32768.f);
    const float im = ((float)(h >> 16) - 32767.5f) * (1e-3f / 32768.f);
    x[i] = make_float2(re, im);
  }
}

__global__ void set_step_kernel(int* c, int v) {
  const int t = threadIdx.x;
  if (t == 0) c[t] = v;
}
__global__ void advance_step_kernel(int* c) {
  const int t = threadIdx.x;
  if (t == 0) c[t] = c[t] + 1;
}

// Batched state layout: element e of instance b at k is [(k nb^2 + e) ldx + b]
// (instance fastest; ldx = the drho row stride), so a wave reads and writes
// consecutive instances of one element.  Per-k observable partials keep the
// [slot][B][nk][5] layout of obs_reduce_kernel.
__device__ inline size_t bidx(const BatchParams& bp, int k, int e, int b) {
  return ((size_t)k * bp.nb * bp.nb + e) * bp.ldx + b;
}

// Packed Hermitian state (batched path without the intraband term): rho(t_n),
// the stage state and the RK4 sum of stage derivatives are Hermitian, so only
// the nb (nb - 1) / 2 elements above the diagonal are kept, as double2
// [k][u][ldx] with u the row-major index of (n, m), n < m, followed (after nk
// U ldx double2) by the nb real diagonal elements as double [k][n][ldx]: half
// the bytes of the full matrices.
__device__ inline int upper_slot(int n, int m, int nb) { return n * nb - n * (n + 1) / 2 + (m - n - 1); }
__device__ inline double2 pk_get(const double2* A, int nk, int nb, int64_t ldx, int k, int n, int m, int b) {
  const int U = nb * (nb - 1) / 2;
  if (m == n)
    return make_double2(reinterpret_cast<const double*>(A + (size_t)nk * U * ldx)[((size_t)k * nb + n) * ldx + b], 0.0);
  return A[((size_t)k * U + upper_slot(n, m, nb)) * ldx + b];
}
// The stage kernel's form of pk_get: one aligned 16-byte load and no branch.
// Above the diagonal it is the element; on the diagonal it is the pair of
// instances (b & ~1, b | 1) holding b's real value (ldx is even, so the pair
// stays in its row), which pk_fix resolves at the first use.  A branch
// between an 8- and a 16-byte load made the compiler wait for every load in
// flight on the diagonal's path.
__device__ inline double2 pk_load(const double2* A, int nk, int nb, int64_t ldx, int k, int n, int m, int b) {
  const int U = nb * (nb - 1) / 2;
  const double* dg = reinterpret_cast<const double*>(A + (size_t)nk * U * ldx) + ((size_t)k * nb + n) * ldx + (b & ~1);
  const double2* p = m == n ? reinterpret_cast<const double2*>(dg) : A + ((size_t)k * U + upper_slot(n, m, nb)) * ldx + b;
  return *p;
}
__device__ inline double2 pk_fix(double2 v, bool diag, int b) {
  return diag ? make_double2((b & 1) ? v.y : v.x, 0.0) : v;
}
__device__ inline void pk_put(double2* A, int nk, int nb, int64_t ldx, int k, int n, int m, int b, double2 v) {
  const int U = nb * (nb - 1) / 2;
  if (m == n)
    reinterpret_cast<double*>(A + (size_t)nk * U * ldx)[((size_t)k * nb + n) * ldx + b] = v.x;
  else
    A[((size_t)k * U + upper_slot(n, m, nb)) * ldx + b] = v;
}

// One block per (k point, group of IB instances): thread t has lane i = t % IB
// (instance group * IB + i) and group n = t / IB, and owns elements n, n + nb,
// n + 2 nb, ... of bp.elist; the list puts the elements that read the product
// first, so each group has about the same loads.  For the observables, group
// n sums row n.  The instances' H and rho blocks are staged in LDS as
// [element][lane] (dynamic LDS: 2 nb^2 IB double2), followed by the k point's
// dipole and velocity planes and band energies (4 nb^2 double2 + nb double).
// NBT: a bound on nb (4 or TDG_NB_MAX); a thread holds NS element slots (3
// for a packed block at nb <= 4, else NBT), at least its group's entries.  The
// observable sums [5][nb][IB] share the H blocks' LDS when they fit (nb >= 3):
// they are consumed before H is built; otherwise they follow the H blocks.
// With bp.xexp, the next gather's P values per instance follow (P IB float2):
// the block then writes its k point's 16-byte chunks of the split operand,
// one per (plane, instance, 4 pairs).
// Blocks map to k XCD-aware (xcd_block): each XCD takes a contiguous range of
// k points.

// WG: IB is one wave (64), so a wave's threads share their group and every
// choice that depends on the group (which element, diagonal or not) is
// uniform across the wave; the element list is then read by scalar loads and
// no load waits at a divergent branch.  WIDE: every pair element is the first
// entry of its group (at most nb of them), and only that slot's product
// slices are loaded, SG0 at a time; without the other slots' slice registers
// the kernel fits 4 waves per SIMD.
template <int NBT, bool PACK, bool WG, bool WIDE = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NBT <= 4 ? 3 : 1, 8)))
batched_stage_kernel(BatchParams bp) {
  extern __shared__ double2 dyn_lds[];
  const int nb = bp.nb, nb2 = nb * nb, IB = WG ? 64 : blockDim.x / nb;
  double2* s_rho = dyn_lds;
  double2* s_h = dyn_lds + nb2 * IB;
  const bool o_shared = nb >= 3;
  double* s_o = reinterpret_cast<double*>(o_shared ? s_h : dyn_lds + 2 * nb2 * IB);  // [5][nb][IB]
  const int i = threadIdx.x % IB, n = WG ? __builtin_amdgcn_readfirstlane(threadIdx.x / 64) : threadIdx.x / IB;
  const int k = tdg::xcd_block(blockIdx.x, gridDim.x), b = blockIdx.y * IB + i;
  // WG: the wave takes the list entries of group (n + rot) % nb, rotating
  // with k, so the waves that own one more element (10 packed elements over
  // 4 groups) do not all sit on the same SIMDs of a CU
  const int rot = WG ? k % nb : 0;
  const bool act = b < bp.n_active, dyn = act && b < bp.n_dyn;
  const int step = bp.step_dev ? bp.step_dev[0] : bp.step;
  const int obs_slot = bp.step_dev ? step % bp.chunk : bp.obs_slot;
  const int P = bp.npair;
  const size_t plane = (size_t)bp.nk * nb2;
  // this k point's dipole planes, velocity planes (stage 0) and band energies,
  // shared by the block's instances: [dx][dy][vx][vy] blocks, then eps
  double2* s_d = dyn_lds + 2 * nb2 * IB + (o_shared ? 0 : (5 * nb * IB + 1) / 2);
  double* s_eps = reinterpret_cast<double*>(s_d + 4 * nb2);
  float2* s_x = reinterpret_cast<float2*>(s_eps + nb);  // [P][IB], with bp.xexp
  const bool want_obs = bp.stage == 0 && bp.obs_part;
  // this k point's dipole / velocity planes and band energies: with WG they
  // go to LDS just before the first barrier, so their loads are not waited
  // for ahead of the state loads (at most two entries per thread: 4 nb^2 <=
  // 2 blockDim for every nb and IB the host uses); otherwise they are stored
  // at once, which holds fewer registers
  double2 d_val[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  double e_val = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = threadIdx.x + h * blockDim.x;
    if (q < 4 * nb2) {
      const int pl = q / nb2, e = q - pl * nb2;
      if (pl < 2)
        d_val[h] = bp.dip[pl * plane + (size_t)k * nb2 + e];
      else if (want_obs)
        d_val[h] = bp.vel[(pl - 2) * plane + (size_t)k * nb2 + e];
      if (!WG) s_d[q] = d_val[h];
    }
  }
  if (threadIdx.x < nb) e_val = bp.eps[(size_t)k * nb + threadIdx.x];
  if (!WG && threadIdx.x < nb) s_eps[threadIdx.x] = e_val;

  tdg_field F = {};
  if (act) F = bp.fields[b];
  const double ef_stage = dyn ? bp.ftab[((size_t)obs_slot * bp.batch + b) * 4 + bp.stage] : 0.0;
  // Every global load of the thread's row is issued before its first use:
  // the state elements (and the intraband term), K_diag o x, then the
  // product's slices for the row's pair elements, SG slices at a time, or
  // SG0 when only the first slot holds pair elements (sums in slice order).
  // Packed, x of a pair element is formed from the element's own state (the
  // stage state less rho_eq, rounded to FP32 as the gather was), so the
  // gather is not read.
  // element slots per thread: a packed block at nb <= 4 has at most 3 per group
  constexpr int NS = (PACK && NBT <= 4) ? 3 : NBT;
  double2 rs[NS], r_n[NS], r_acc[NS], ds[NS], dv[NS];
  int ee[NS];           // element n nb + m of slot q; -1: none
  int prow[NS];         // product row (k P + p) of slot q, -1 = none
  bool partner[NS];     // element (v, c) of the conduction-valence block: conj of (c, v)
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    rs[q] = r_n[q] = r_acc[q] = ds[q] = dv[q] = make_double2(0.0, 0.0);
    prow[q] = -1;
    partner[q] = false;
    const int j = (WG ? (n + rot) % nb : n) + q * nb;
    ee[q] = j < bp.nelem ? bp.elist[j] : -1;
    if (WG) ee[q] = __builtin_amdgcn_readfirstlane(ee[q]);
    if (ee[q] < 0 || !act) continue;
    const int r = ee[q] / nb, c = ee[q] - r * nb;
    const size_t g = bidx(bp, k, ee[q], b);
    // packed: raw 16-byte loads, resolved by pk_fix at the first use
    rs[q] = PACK ? pk_load(bp.rho_s, bp.nk, nb, bp.ldx, k, r, c, b) : bp.rho_s[g];
    if (!dyn) continue;
    r_n[q] = PACK ? pk_load(bp.rho_n, bp.nk, nb, bp.ldx, k, r, c, b) : bp.rho_n[g];
    if (bp.stage != 0) r_acc[q] = PACK ? pk_load(bp.acc, bp.nk, nb, bp.ldx, k, r, c, b) : bp.acc[g];
    if (!PACK && bp.intra) dv[q] = bp.intra[g];
    int p = -1;
    if (bp.block == TDG_BLOCK_ALL) {
      p = r * nb + c;
    } else if (r >= bp.nv && c < bp.nv) {
      p = (r - bp.nv) * bp.nv + c;
    } else if (r < bp.nv && c >= bp.nv) {
      p = (c - bp.nv) * bp.nv + r;
      partner[q] = true;
    }
    if (p >= 0 && (!WIDE || q == 0)) prow[q] = k * P + p;
  }
  float2 kd[NS], xk[NS];
  float yr[NS], yi[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    yr[m] = yi[m] = 0.f;
    kd[m] = xk[m] = make_float2(0.f, 0.f);
    if (bp.kdiag && prow[m] >= 0) {
      kd[m] = bp.kdiag[prow[m]];
      if (!PACK) xk[m] = bp.xcur[(size_t)prow[m] * bp.ldx + b];
    }
  }
  if (WIDE) {
    // only slot 0 reads the product: up to SG0 of its slices in flight at once
    constexpr int SG0 = 16;
    for (int s0 = 0; s0 < bp.y_slices; s0 += SG0) {
      float2 yv[SG0];
#pragma unroll
      for (int q = 0; q < SG0; ++q)
        yv[q] = (prow[0] >= 0 && s0 + q < bp.y_slices)
                    ? bp.Y[(size_t)(s0 + q) * bp.y_slice_stride + (size_t)prow[0] * bp.ldy + b]
                    : make_float2(0.f, 0.f);
#pragma unroll
      for (int q = 0; q < SG0; ++q)
        if (prow[0] >= 0 && s0 + q < bp.y_slices) {
          yr[0] += yv[q].x;
          yi[0] += yv[q].y;
        }
    }
  }
  constexpr int SG = NBT <= 4 ? 4 : 2;  // slices per group
  for (int s0 = 0; s0 < (WIDE ? 0 : bp.y_slices); s0 += SG) {
    float2 yv[NS][SG];
#pragma unroll
    for (int m = 0; m < NS; ++m)
#pragma unroll
      for (int q = 0; q < SG; ++q)
        yv[m][q] = (prow[m] >= 0 && s0 + q < bp.y_slices)
                       ? bp.Y[(size_t)(s0 + q) * bp.y_slice_stride + (size_t)prow[m] * bp.ldy + b]
                       : make_float2(0.f, 0.f);
#pragma unroll
    for (int m = 0; m < NS; ++m)
#pragma unroll
      for (int q = 0; q < SG; ++q)
        if (prow[m] >= 0 && s0 + q < bp.y_slices) {
          yr[m] += yv[m][q].x;
          yi[m] += yv[m][q].y;
        }
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int r = ee[q] / nb, c = ee[q] - r * nb;
    if (PACK && ee[q] >= 0) rs[q] = pk_fix(rs[q], r == c, b);
    if (prow[q] >= 0) {
      float zr = yr[q], zi = yi[q];
      if (bp.kdiag) {
        float2 x = xk[q];
        if (PACK) {
          // pair p of this element, or of its mirror below the diagonal (partner)
          const float xi = (float)rs[q].y;
          x = make_float2((float)(rs[q].x - ((r == c && r < bp.nv) ? 1.0 : 0.0)), partner[q] ? -xi : xi);
        }
        zr += kd[q].x * x.x - kd[q].y * x.y;
        zi += kd[q].x * x.y + kd[q].y * x.x;
      }
      ds[q] = make_double2((double)zr, partner[q] ? -(double)zi : (double)zi);
    }
    if (ee[q] >= 0) {
      s_rho[ee[q] * IB + i] = rs[q];
      if (PACK && c > r) s_rho[(c * nb + r) * IB + i] = make_double2(rs[q].x, -rs[q].y);
    }
  }
  if (WG) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (threadIdx.x + h * blockDim.x < 4 * nb2) s_d[threadIdx.x + h * blockDim.x] = d_val[h];
    if (threadIdx.x < nb) s_eps[threadIdx.x] = e_val;
  }
  __syncthreads();

  // observables of rho(t_n), per (k, instance): row sums, then a fixed-order sum over rows
  if (want_obs) {
    double o[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (act) {
#pragma unroll
      for (int m = 0; m < NBT; ++m) {
        if (m >= nb) break;
        const int e = n * nb + m;
        const double2 de = proj_e(F, s_d[e], s_d[nb2 + e]);
        const double2 ve = proj_e(F, s_d[2 * nb2 + e], s_d[3 * nb2 + e]);
        const double2 rmn = s_rho[(m * nb + n) * IB + i], rnm = s_rho[e * IB + i];
        o[0] += de.x * rmn.x - de.y * rmn.y;
        o[1] += ve.x * rmn.x - ve.y * rmn.y;
        if (n == m && n == bp.nv) o[2] += rnm.x;
        if (n == m) o[3] += rnm.x;
        const double hx = rnm.x - rmn.x, hy = rnm.y + rmn.y, h = sqrt(hx * hx + hy * hy);
        if (h > o[4] || h != h) o[4] = h;
      }
    }
    for (int c = 0; c < 5; ++c) s_o[(c * nb + n) * IB + i] = o[c];
    __syncthreads();
    if (act && n < 5) {
      // row n of the block's threads writes observables n, n + nb, ... (< 5)
      for (int c = n; c < 5; c += nb) {
        double v = 0.0;
        for (int r = 0; r < nb; ++r) {
          const double q = s_o[(c * nb + r) * IB + i];
          if (c < 4)
            v += q;  // P, J, occupation and the trace are sums over rows
          else if (q > v || q != q)
            v = q;   // the Hermiticity residual is a maximum
        }
        if (c == 3) v = bp.tr_signed ? v - (double)bp.nv : fabs(v - (double)bp.nv);
        bp.obs_part[(((size_t)obs_slot * bp.batch + b) * bp.nk + k) * 5 + c] = v;
      }
    }
  }

  // the observable sums share LDS with the H blocks written next
  if (o_shared && want_obs) __syncthreads();

  // H = eps + dSigma - E(t) e.d
  const double ef = ef_stage;
  if (dyn) {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      if (ee[q] < 0) continue;
      const int e = ee[q], r = e / nb, c = e - r * nb;
      const double2 de = proj_e(F, s_d[e], s_d[nb2 + e]);
      double2 h = make_double2(ds[q].x - ef * de.x, ds[q].y - ef * de.y);
      if (r == c) h.x += s_eps[r];
      if (PACK && r == c) h.y = 0.0;  // Hermitian: a real diagonal
      s_h[e * IB + i] = h;
      if (PACK && c > r) s_h[(c * nb + r) * IB + i] = make_double2(h.x, -h.y);
    }
  }
  __syncthreads();

  // f = -i [H, rho], RK4 stage, next drho gather
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    if (!dyn || ee[q] < 0) continue;
    const int e = ee[q], n = e / nb, m = e - n * nb;
    if (PACK) {
      r_n[q] = pk_fix(r_n[q], n == m, b);
      r_acc[q] = pk_fix(r_acc[q], n == m, b);
    }
    double2 c = make_double2(0.0, 0.0);
    for (int l = 0; l < nb; ++l) {
      const double2 hr = cmul(s_h[(n * nb + l) * IB + i], s_rho[(l * nb + m) * IB + i]);
      const double2 rh = cmul(s_rho[(n * nb + l) * IB + i], s_h[(l * nb + m) * IB + i]);
      c.x += hr.x - rh.x;
      c.y += hr.y - rh.y;
    }
    double2 f = make_double2(c.y, -c.x);
    if (PACK && n == m) f.y = 0.0;  // the derivative of a Hermitian state is Hermitian
    const size_t g = bidx(bp, k, e, b);
    if (!PACK && bp.intra) {
      // intraband part of the field term: -E(t) e.(rho)_{;k}
      f.x -= ef * dv[q].x;
      f.y -= ef * dv[q].y;
    }
    double2 next, accv = f;
    if (bp.stage == 0) {
      next = make_double2(r_n[q].x + 0.5 * bp.dt * f.x, r_n[q].y + 0.5 * bp.dt * f.y);
    } else if (bp.stage == 1) {
      accv = make_double2(r_acc[q].x + 2.0 * f.x, r_acc[q].y + 2.0 * f.y);
      next = make_double2(r_n[q].x + 0.5 * bp.dt * f.x, r_n[q].y + 0.5 * bp.dt * f.y);
    } else if (bp.stage == 2) {
      accv = make_double2(r_acc[q].x + 2.0 * f.x, r_acc[q].y + 2.0 * f.y);
      next = make_double2(r_n[q].x + bp.dt * f.x, r_n[q].y + bp.dt * f.y);
    } else {
      const double w = bp.dt / 6.0;
      next = make_double2(r_n[q].x + w * (r_acc[q].x + f.x), r_n[q].y + w * (r_acc[q].y + f.y));
    }
    if (PACK) {
      if (bp.stage < 3) pk_put(bp.acc, bp.nk, nb, bp.ldx, k, n, m, b, accv);
      if (bp.stage == 3) pk_put(bp.rho_n, bp.nk, nb, bp.ldx, k, n, m, b, next);
      pk_put(bp.rho_s, bp.nk, nb, bp.ldx, k, n, m, b, next);
    } else {
      if (bp.stage < 3) bp.acc[g] = accv;
      if (bp.stage == 3) bp.rho_n[g] = next;
      bp.rho_s[g] = next;
    }
    const double dre = next.x - ((n == m && n < bp.nv) ? 1.0 : 0.0);
    // pair p of this element (and, packed, pair pm of its mirror) gets x
    int p = -1, pm = -1;
    float xi = (float)next.y;
    if (bp.block == TDG_BLOCK_ALL) {
      p = e;
      if (PACK && m > n) pm = m * nb + n;  // the pair below the diagonal: conj of this one
    } else if (!PACK && n >= bp.nv && m < bp.nv) {
      p = (n - bp.nv) * bp.nv + m;
    } else if (PACK && n < bp.nv && m >= bp.nv) {
      // conduction-valence pair (m, n) from its partner above the diagonal
      p = (m - bp.nv) * bp.nv + n;
      xi = -xi;
    }
    // packed with the split operand, nothing reads the FP32 gather: the
    // products read the split, and the next stage forms x from its state
    const bool x32 = !PACK || !bp.xexp;
    if (p >= 0) {
      if (x32) bp.xnext[((size_t)k * P + p) * bp.ldx + b] = make_float2((float)dre, xi);
      if (bp.xexp) s_x[p * IB + i] = make_float2((float)dre, xi);
    }
    if (pm >= 0) {
      if (x32) bp.xnext[((size_t)k * P + pm) * bp.ldx + b] = make_float2((float)dre, -xi);
      if (bp.xexp) s_x[pm * IB + i] = make_float2((float)dre, -xi);
    }
  }
  if (!bp.xexp) return;
  // the split operand of this k point: chunk g4 of instance c (pairs 4 g4 ..
  // 4 g4 + 3) in plane p is 16 bytes, and the 64 instances' chunks are
  // contiguous; rows of instances that no longer integrate are left as they
  // are (their product columns are unused)
  __syncthreads();
  const int nch = P / 4, ct = blockIdx.y;
  for (int q = threadIdx.x; q < 2 * nch * tdg::XB_TILE; q += blockDim.x) {
    const int c = q % tdg::XB_TILE, g4 = (q / tdg::XB_TILE) % nch, plane = q / (tdg::XB_TILE * nch);
    if (blockIdx.y * IB + c >= bp.n_dyn) continue;
    uint4 w;
    unsigned int* wp = reinterpret_cast<unsigned int*>(&w);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float2 v = s_x[(4 * g4 + u) * IB + c];
      wp[u] = tdg::xb_word(v.x, v.y, plane);
    }
    *reinterpret_cast<uint4*>(bp.xexp + tdg::xb_index(ct, plane, c, 2 * ((int64_t)k * P + 4 * g4), bp.ldxb)) = w;
  }
}

// Batched state from the caller's rho: element e of instance b (sorted
// position) at k to [(k nb^2 + e) ldx + b]; drho gather [N][ldx].  One block per k.
__global__ void init_batched_kernel(const double2* __restrict__ rho_in, const int* __restrict__ perm, double2* rho_n,
                                    double2* rho_s, float2* x, int64_t ldx, int nk, int nb, int nv, int npair,
                                    int block, int init_eq, int batch, int pack) {
  const int k = blockIdx.x, nb2 = nb * nb;
  for (int idx = threadIdx.x; idx < nb2 * batch; idx += blockDim.x) {
    const int e = idx / batch, b = idx % batch, n = e / nb, m = e % nb;
    const double occ = (n == m && n < nv) ? 1.0 : 0.0;
    double2 r = init_eq ? make_double2(occ, 0.0) : rho_in[((size_t)perm[b] * nk + k) * nb2 + e];
    if (pack) {
      // the Hermitian part: below the diagonal, the conjugate of the element above
      if (n > m && !init_eq) {
        const double2 u = rho_in[((size_t)perm[b] * nk + k) * nb2 + m * nb + n];
        r = make_double2(u.x, -u.y);
      }
      if (n == m) r.y = 0.0;
      if (m >= n) {
        pk_put(rho_n, nk, nb, ldx, k, n, m, b, r);
        pk_put(rho_s, nk, nb, ldx, k, n, m, b, r);
      }
    } else {
      const size_t g = ((size_t)k * nb2 + e) * ldx + b;
      rho_n[g] = r;
      rho_s[g] = r;
    }
    int p = -1;
    if (block == TDG_BLOCK_ALL)
      p = e;
    else if (n >= nv && m < nv)
      p = (n - nv) * nv + m;
    if (p >= 0) x[((size_t)k * npair + p) * ldx + b] = make_float2((float)(r.x - occ), (float)r.y);
  }
}

// rho[perm[b]] <- batched rho_n.  One block per k.
__global__ void finish_batched_kernel(const double2* __restrict__ rho_n, const int* __restrict__ perm,
                                      double2* rho_out, int64_t ldx, int nk, int nb, int batch, int pack) {
  const int k = blockIdx.x, nb2 = nb * nb;
  for (int idx = threadIdx.x; idx < nb2 * batch; idx += blockDim.x) {
    const int e = idx / batch, b = idx % batch, n = e / nb, m = e % nb;
    double2 v;
    if (pack) {
      v = pk_get(rho_n, nk, nb, ldx, k, min(n, m), max(n, m), b);
      if (n > m) v.y = -v.y;
    } else {
      v = rho_n[((size_t)k * nb2 + e) * ldx + b];
    }
    rho_out[((size_t)perm[b] * nk + k) * nb2 + e] = v;
  }
}

// Observables of an arbitrary state (tdg_observables), caller's order.
__global__ void obs_state_kernel(StageParams sp) {
  const int k = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  __shared__ double2 s_rho[NB2_MAX];
  __shared__ double s_obs[5][NB2_MAX];
  const int nb2 = sp.nb * sp.nb;
  const tdg_field F = sp.fields[b];
  double2 de = make_double2(0.0, 0.0), ve = de;
  if (t < nb2) {
    const size_t base = (size_t)k * nb2 + t, plane = (size_t)sp.nk * nb2;
    s_rho[t] = sp.rho_s[((size_t)b * sp.nk + k) * nb2 + t];
    de = proj_e(F, sp.dip[base], sp.dip[plane + base]);
    ve = proj_e(F, sp.vel[base], sp.vel[plane + base]);
  }
  __syncthreads();
  obs_partial(sp, s_rho, s_obs, de, ve, k, b);
}

// Fixed-order reduction of per-k observables: sums (P, J, occ) / nk and
// maxima (tr, herm), for steps step0 .. step0 + gridDim.x - 1 of the sorted
// instance b, written to row perm[b] (or to out5[b] for tdg_observables).
// tr_mean: the trace partials are signed and the result is |sum| / nk.
__global__ void __launch_bounds__(THREADS) obs_reduce_kernel(const double* __restrict__ part, int nk, int batch,
                                                             int step0, const tdg_field* fields,
                                                             const int* __restrict__ perm, tdg_obs obs,
                                                             double* out5, int tr_mean) {
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
    if (tr_mean) a[3] += q[3];
    for (int c = tr_mean ? 4 : 3; c < 5; ++c)
      if (q[c] > a[c] || q[c] != q[c]) a[c] = q[c];
  }
  for (int c = 0; c < 5; ++c) s[c][t] = a[c];
  __syncthreads();
  for (int w = THREADS / 2; w > 0; w >>= 1) {
    if (t < w) {
      for (int c = 0; c < 3; ++c) s[c][t] += s[c][t + w];
      if (tr_mean) s[3][t] += s[3][t + w];
      for (int c = tr_mean ? 4 : 3; c < 5; ++c) {
        const double o = s[c][t + w];
        if (o > s[c][t] || o != o) s[c][t] = o;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const double inv = 1.0 / (double)nk;
    if (tr_mean) s[3][0] = fabs(s[3][0]) * inv;
    if (out5) {
      double* o = out5 + (size_t)b * 5;
      o[0] = s[0][0] * inv;
      o[1] = s[1][0] * inv;
      o[2] = s[2][0] * inv;
      o[3] = s[3][0];
      o[4] = s[4][0];
    } else {
      const size_t i = (size_t)perm[b] * obs.stride + step;
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

namespace tdg {

int args_upload(tdg_ctx ctx, void* dev, const void* host, size_t bytes) {
  if ((bytes & 3) || ((uintptr_t)dev & 3)) return fail(ctx, TDG_E_INVAL, "args_upload: unaligned copy");
  const uint32_t* src = static_cast<const uint32_t*>(host);
  uint32_t* dst = static_cast<uint32_t*>(dev);
  const size_t words = bytes / 4;
  for (size_t w0 = 0; w0 < words; w0 += ARG_WORDS) {
    const int nw = (int)std::min<size_t>(ARG_WORDS, words - w0);
    ArgPayload pl;
    std::memcpy(pl.w, src + w0, (size_t)nw * 4);
    hipLaunchKernelGGL(arg_copy_kernel, dim3(1), dim3(256), 0, ctx->stream, pl, dst + w0, nw);
  }
  return launch_check(ctx, "argument upload");
}

}  // namespace tdg

// Device workspace of one propagation: the context's grow-only slots, or,
// when `arena` is set, consecutive 256-byte aligned pieces of a fixed device
// array of `cap` bytes (nothing is allocated then).
struct Workspace {
  tdg_ctx ctx;
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  int get(WsSlot slot, size_t bytes, void** out) {
    if (!arena) return ws_reserve(ctx, slot, bytes, out);
    const size_t want = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
    if (want > cap - used)
      return fail(ctx, TDG_E_INVAL, "workspace of %zu bytes exceeds the %zu-byte scratch array (slot %d)", used + want,
                  cap, (int)slot);
    *out = arena + used;
    used += want;
    return TDG_OK;
  }
  size_t left() const { return arena ? cap - used : SIZE_MAX; }
};

// ---- stage-kernel variants -------------------------------------------------
// Stage-kernel launch; with events (profiling) the dispatch itself is timed.
using StageLaunch = void (*)(dim3, size_t, hipStream_t, const StageParams&, hipEvent_t, hipEvent_t);

template <typename T, int MODE, int NT, int U, int WPE>
static void launch_stage(dim3 grid, size_t lds, hipStream_t stream, const StageParams& sp, hipEvent_t ea,
                         hipEvent_t eb) {
  if (ea)
    hipExtLaunchKernelGGL((stage_kernel<T, MODE, NT, U, WPE>), grid, dim3(NT), (uint32_t)lds, stream, ea, eb, 0u, sp);
  else
    hipLaunchKernelGGL((stage_kernel<T, MODE, NT, U, WPE>), grid, dim3(NT), lds, stream, sp);
}

struct Variant {
  const char* name;
  StageLaunch fn;
};

static const Variant kDenseF32[] = {
    {"dense_f32_nt256_u2_w6", launch_stage<float, 0, 256, 2, 6>},
    {"dense_f32_nt256_u4_w4", launch_stage<float, 0, 256, 4, 4>},
    {"dense_f32_nt256_u1_w8", launch_stage<float, 0, 256, 1, 8>},
    {"dense_f32_nt128_u4_w4", launch_stage<float, 0, 128, 4, 4>},
    {"dense_f32_nt512_u2_w4", launch_stage<float, 0, 512, 2, 4>},
};
static const Variant kDenseF64[] = {
    {"dense_f64_nt256_u2_w4", launch_stage<double, 0, 256, 2, 4>},
    {"dense_f64_nt256_u1_w6", launch_stage<double, 0, 256, 1, 6>},
    {"dense_f64_nt128_u2_w4", launch_stage<double, 0, 128, 2, 4>},
};
static const Variant kLowF32[] = {
    {"lowrank_f32_nt64", launch_stage<float, 1, 64, 1, 2>},
    {"lowrank_f32_nt128", launch_stage<float, 1, 128, 1, 2>},
    {"lowrank_f32_nt256", launch_stage<float, 1, 256, 1, 2>},
    {"lowrank_f32_nt128_c4", launch_stage<float, 1, 128, 2, 2>},
    {"lowrank_f32_nt64_c6", launch_stage<float, 1, 64, 3, 2>},
};
static const Variant kChanF32[] = {
    {"channel_f32_nt256_u2_w6", launch_stage<float, 2, 256, 2, 6>},
    {"channel_f32_nt256_u4_w4", launch_stage<float, 2, 256, 4, 4>},
    {"channel_f32_nt128_u4_w4", launch_stage<float, 2, 128, 4, 4>},
};
static const Variant kChanF64[] = {
    {"channel_f64_nt256_u2_w4", launch_stage<double, 2, 256, 2, 4>},
    {"channel_f64_nt128_u2_w4", launch_stage<double, 2, 128, 2, 4>},
};
static const Variant kLowF64[] = {
    {"lowrank_f64_nt64", launch_stage<double, 1, 64, 1, 2>},
    {"lowrank_f64_nt128", launch_stage<double, 1, 128, 1, 2>},
    {"lowrank_f64_nt256", launch_stage<double, 1, 256, 1, 2>},
};

// Timing events of a tuner, destroyed on every exit path.
struct TunerEvents {
  std::vector<hipEvent_t> ev;
  int create(tdg_ctx ctx, size_t count) {
    ev.assign(count, nullptr);
    for (auto& e : ev) TDG_TRY(hip_check(ctx, hipEventCreate(&e), "tuner event"));
    return TDG_OK;
  }
  ~TunerEvents() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

template <size_t N>
static void table(const Variant (&v)[N], const Variant*& out, int& count) {
  out = v;
  count = (int)N;
}

// Largest Hermiticity residual accepted in a caller's rho(0).
constexpr double RHO0_HERM_TOL = 1e-12;

// tdg_propagate on the workspace W.  With a fixed arena (W.arena) every
// instance takes the per-instance path and the stage-kernel choice comes from
// the context's tuner cache (or variant 0): no timing, nothing allocated.
static int propagate_impl(tdg_ctx ctx, const tdg_operator* op, const tdg_model* model, const tdg_field* fields,
                          int32_t batch, double dt, void* rho, int32_t init_eq, const tdg_obs* obs, Workspace& W) {
  const bool fixed = W.arena != nullptr;
  TDG_TRY(validate_model(ctx, model));
  if (!op) return fail(ctx, TDG_E_INVAL, "operator is NULL");
  if (op->dtype != TDG_C128 && op->dtype != TDG_C64 && op->dtype != TDG_BF16X2)
    return fail(ctx, TDG_E_INVAL, "operator dtype %d", op->dtype);
  const bool bf16 = op->dtype == TDG_BF16X2;
  if (fixed && bf16) return fail(ctx, TDG_E_UNSUPPORTED, "BF16X2 operators run on the batched path only");
  const int npair = pairs_per_k(model, op->block);
  if (npair <= 0) return fail(ctx, TDG_E_INVAL, "unknown block %d", op->block);
  const int nk = model->nk1 * model->nk2;
  const int64_t n = (int64_t)nk * npair;
  if (op->n != n) return fail(ctx, TDG_E_INVAL, "operator n = %lld, model gives N = %lld", (long long)op->n, (long long)n);
  if (n > ((int64_t)1 << 30)) return fail(ctx, TDG_E_UNSUPPORTED, "N = %lld too large", (long long)n);
  const size_t elt = op->dtype == TDG_C128 ? 16 : 8;  // x and z are complex64 for C64 and BF16X2
  const bool lowrank = op->kind == TDG_OP_LOWRANK;
  const bool channel = op->kind == TDG_OP_CHANNEL;
  const void* A = nullptr;
  int64_t lda = 0;
  int ncols = 0;
  int ch_ls = 0;
  if (channel) {
    // diagonal channels [P][nk][nk] in K, off-diagonal factors in us / w, rank = rmax
    if (!op->K || !op->us || !op->w) return fail(ctx, TDG_E_INVAL, "channel-wise operator with NULL array");
    if (bf16) return fail(ctx, TDG_E_UNSUPPORTED, "channel-wise operators are TDG_C128 or TDG_C64");
    if (op->rank < 4 || op->rank % 4 != 0 || op->rank > nk)
      return fail(ctx, TDG_E_INVAL, "channel rank capacity %lld must be a multiple of 4 in [4, nk]", (long long)op->rank);
    if (npair < 2) return fail(ctx, TDG_E_INVAL, "channel-wise operators need at least two pairs per k");
    A = op->K;
    lda = nk;
    ncols = nk;
    ch_ls = (int)((npair - 1) * op->rank);
  } else if (op->kind == TDG_OP_DENSE) {
    if (!op->K) return fail(ctx, TDG_E_INVAL, "dense operator without K");
    if (op->ld < n) return fail(ctx, TDG_E_INVAL, "K ld = %lld < N", (long long)op->ld);
    A = op->K;
    lda = op->ld;
    ncols = (int)n;
  } else if (lowrank) {
    if (!op->kdiag || !op->us || !op->w) return fail(ctx, TDG_E_INVAL, "low-rank operator with NULL factor");
    if (op->rank < 1 || op->rank > n) return fail(ctx, TDG_E_INVAL, "rank %lld outside [1, N]", (long long)op->rank);
    A = op->us;
    lda = op->rank;
    ncols = (int)op->rank;
  } else {
    return fail(ctx, TDG_E_INVAL, "operator kind %d", op->kind);
  }
  if (((uintptr_t)A | (uintptr_t)op->kdiag | (uintptr_t)op->w | (channel ? (uintptr_t)op->us : 0)) &
      (elt == 16 ? 15 : 7))
    return fail(ctx, TDG_E_INVAL, "operator arrays must be aligned to their complex element size");
  if (bf16 && ((((uintptr_t)A | (uintptr_t)op->w) & 15) || (op->kind == TDG_OP_DENSE && op->ld % 4 != 0) ||
               (lowrank && n % 4 != 0)))
    return fail(ctx, TDG_E_INVAL, "BF16X2 operators need 16-byte aligned planes and row strides that are multiples of 4");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, TDG_E_INVAL, "dt must be positive");
  if (!rho || ((uintptr_t)rho & 15)) return fail(ctx, TDG_E_INVAL, "rho NULL or not 16-byte aligned");
  int64_t max_steps = 0;
  TDG_TRY(validate_fields(ctx, fields, batch, &max_steps));
  if (!obs || !obs->P || !obs->J || !obs->occ) return fail(ctx, TDG_E_INVAL, "observable arrays are NULL");
  if (obs->stride < max_steps + 1)
    return fail(ctx, TDG_E_INVAL, "obs stride %lld < max nsteps + 1 = %lld", (long long)obs->stride,
                (long long)(max_steps + 1));
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));

  // instances by decreasing length: the running ones are always a prefix
  std::vector<int> perm(batch);
  for (int i = 0; i < batch; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return fields[x].nsteps > fields[y].nsteps; });
  std::vector<tdg_field> sorted(batch);
  std::vector<int64_t> len(batch);
  for (int i = 0; i < batch; ++i) {
    sorted[i] = fields[perm[i]];
    len[i] = (int64_t)sorted[i].nsteps;
  }

  const int nb2 = model->nb * model->nb;
  // matrix-core path: complex64 operator and enough instances
  const bool batched = !fixed && !channel && (bf16 || (op->dtype == TDG_C64 && batch >= ctx->batched_min));
  if (batched && n > 2147483647 / 2) return fail(ctx, TDG_E_UNSUPPORTED, "batched path: N < 2^30 required");
  // batched rows hold an even number of instances (two per 16-byte load)
  const int64_t xstride = batched ? (((int64_t)batch + 1) & ~int64_t(1)) : ((n + 1) & ~int64_t(1));
  // batched state is instance fastest with the drho row stride
  const size_t state_bytes = (size_t)(batched ? xstride : batch) * nk * nb2 * sizeof(double2);
  const int64_t zstride = channel ? (int64_t)npair * ch_ls : (op->rank + 1) & ~int64_t(1);
  void *rho_n, *rho_s, *acc, *x0, *x1, *z = nullptr, *part, *dperm, *dfields, *dintra = nullptr;
  // intraband term: e.(rho_s)_{;k} of each stage.  Batched path: computed by
  // its own launch before the stage kernel.  Per-instance path: formed in the
  // stage kernel's epilogue from the neighbours' states, read from one
  // stage-state buffer while the next stage state goes to the other.
  const bool intra = model->links != nullptr;
  if (intra && (int64_t)nk * nb2 * batch > ((int64_t)1 << 38))
    return fail(ctx, TDG_E_UNSUPPORTED, "intraband term: nk * nb^2 * batch too large for one launch");
  void* rho_s2 = nullptr;
  if (intra && batched) TDG_TRY(W.get(WS_INTRA, state_bytes, &dintra));
  if (intra && !batched) TDG_TRY(W.get(WS_RHO_S2, state_bytes, &rho_s2));
  TDG_TRY(W.get(WS_RHO_N, state_bytes, &rho_n));
  TDG_TRY(W.get(WS_RHO_S, state_bytes, &rho_s));
  TDG_TRY(W.get(WS_ACC, state_bytes, &acc));
  const size_t xbytes = batched ? (size_t)n * xstride * elt : (size_t)batch * xstride * elt;
  TDG_TRY(W.get(WS_X0, xbytes, &x0));
  TDG_TRY(W.get(WS_X1, xbytes, &x1));
  // low rank: the projection is split over zsplit column slices (at least
  // about 256 blocks per instance, at most ZSPLIT_MAX slices); the stage
  // kernel sums the slices it reads
  int zsplit = 1;
  int64_t zslice = n;
  if (channel) {
    zslice = nk;
    TDG_TRY(W.get(WS_Z, (size_t)batch * zstride * elt, &z));
  } else if (lowrank && !batched) {
    const int64_t groups = (op->rank + ROWS - 1) / ROWS;
    zsplit = (int)std::min<int64_t>(ZSPLIT_MAX, std::max<int64_t>(1, (256 + groups - 1) / groups));
    zslice = ((n + zsplit - 1) / zsplit + 1) & ~int64_t(1);
    zsplit = (int)((n + zslice - 1) / zslice);
    // room for the tuner's largest split
    TDG_TRY(W.get(WS_Z, (size_t)ZSPLIT_MAX * batch * zstride * elt, &z));
  }
  // a split of the projection's columns into `want` slices (at most ZSPLIT_MAX)
  auto set_split = [&](int want) {
    zslice = ((n + want - 1) / want + 1) & ~int64_t(1);
    zsplit = (int)((n + zslice - 1) / zslice);
  };
  // field records in sorted order, followed by the sorted position -> caller's
  // index map (one upload)
  const size_t fbytes = sizeof(tdg_field) * batch, pbytes = (sizeof(int) * batch + 3) & ~size_t(3);
  TDG_TRY(W.get(WS_FIELDS, fbytes + pbytes, &dfields));
  dperm = (char*)dfields + fbytes;
  void* dmisc = nullptr;
  TDG_TRY(W.get(WS_MISC, 256, &dmisc));
  // observable partials of `chunk` steps, and the field at their stage times
  // (refilled at each chunk start); a fixed arena bounds the chunk
  const size_t part_per_step = (size_t)batch * nk * 5 * sizeof(double);
  const size_t per_slot = part_per_step + (size_t)batch * 4 * sizeof(double);
  int chunk = (int)std::min<size_t>(256, std::max<size_t>(1, OBS_PART_BUDGET / part_per_step));
  if (fixed) chunk = (int)std::min<size_t>(chunk, W.left() >= 512 ? (W.left() - 512) / per_slot : 0);
  if (chunk < 1) return fail(ctx, TDG_E_INVAL, "the scratch array cannot hold one step of observable partials");
  TDG_TRY(W.get(WS_OBS_PART, part_per_step * chunk, &part));
  void* ftab = nullptr;
  TDG_TRY(W.get(WS_FTAB, (size_t)chunk * batch * 4 * sizeof(double), &ftab));
  auto field_table = [&](int64_t step0) {
    const int count = (int)std::min<int64_t>(chunk, max_steps - step0 + 1);
    const int total = count * batch * 4;
    hipLaunchKernelGGL(field_table_kernel, dim3((total + 255) / 256), dim3(256), 0, ctx->stream,
                       (const tdg_field*)dfields, batch, (int)step0, count, dt, (double*)ftab);
  };
  {
    std::vector<char> rec(fbytes + pbytes);
    std::memcpy(rec.data(), sorted.data(), fbytes);
    std::memcpy(rec.data() + fbytes, perm.data(), sizeof(int) * batch);
    TDG_TRY(args_upload(ctx, dfields, rec.data(), rec.size()));
  }
  if (!init_eq) {
    // rho(0) must be Hermitian; the check waits for its one-value result
    const int64_t nblk = (int64_t)batch * nk;
    const int64_t nparts = (nblk + 255) / 256;
    hipLaunchKernelGGL(herm_check_kernel, dim3((unsigned)nparts), dim3(256), 0, ctx->stream, (const double2*)rho, nblk,
                       model->nb, (double*)part);
    hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, ctx->stream, (const double*)part, nparts,
                       (double*)dmisc);
    TDG_TRY(launch_check(ctx, "rho(0) check launch"));
    double h = 0.0;
    TDG_TRY(hip_check(ctx, hipMemcpyAsync(&h, dmisc, sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
                      "rho(0) check copy"));
    TDG_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "rho(0) check sync"));
    if (!(h <= RHO0_HERM_TOL))
      return fail(ctx, TDG_E_INVAL, "rho(0) is not Hermitian: max |rho_nm - conj rho_mn| = %.3g > %g", h,
                  RHO0_HERM_TOL);
  }

  const int init_threads = ((nb2 + 63) / 64) * 64;
  auto init = [&]() {
    if (batched) {
      hipLaunchKernelGGL(init_batched_kernel, dim3(nk), dim3(256), 0, ctx->stream, (const double2*)rho,
                         (const int*)dperm, (double2*)rho_n, (double2*)rho_s, (float2*)x0, xstride, nk, model->nb,
                         model->nv, npair, op->block, init_eq, batch, (int)!intra);
      return launch_check(ctx, "init launch");
    }
    if (op->dtype == TDG_C128)
      hipLaunchKernelGGL(init_kernel<double>, dim3(nk, batch), dim3(init_threads), 0, ctx->stream,
                         (const double2*)rho, (const int*)dperm, (double2*)rho_n, (double2*)rho_s, x0, xstride, nk,
                         model->nb, model->nv, npair, op->block, init_eq, channel ? 2 : 0);
    else
      hipLaunchKernelGGL(init_kernel<float>, dim3(nk, batch), dim3(init_threads), 0, ctx->stream,
                         (const double2*)rho, (const int*)dperm, (double2*)rho_n, (double2*)rho_s, x0, xstride, nk,
                         model->nb, model->nv, npair, op->block, init_eq, channel ? 2 : 0);
    return launch_check(ctx, "init launch");
  };
  TDG_TRY(init());

  StageParams sp = {};
  sp.A = A;
  sp.lda = lda;
  sp.ncols = ncols;
  sp.kdiag = lowrank ? op->kdiag : nullptr;
  sp.chS = channel ? op->us : nullptr;
  sp.chLS = ch_ls;
  sp.xstride = xstride;
  sp.rho_n = (double2*)rho_n;
  sp.rho_s = (double2*)rho_s;
  sp.acc = (double2*)acc;
  sp.eps = model->eps;
  sp.dip = (const double2*)model->dip;
  sp.vel = (const double2*)model->vel;
  sp.fields = (const tdg_field*)dfields;
  sp.obs_part = (double*)part;
  sp.nk = nk;
  sp.nb = model->nb;
  sp.nv = model->nv;
  sp.npair = npair;
  sp.block = op->block;
  sp.batch = batch;
  sp.dt = dt;
  sp.tr_signed = intra;
  sp.ftab = (const double*)ftab;
  sp.rho_s_out = intra && !batched ? (double2*)rho_s2 : (double2*)rho_s;
  if (intra && !batched) {
    sp.links = (const double2*)model->links;
    sp.nk1 = model->nk1;
    sp.nk2 = model->nk2;
    sp.cov_c1 = model->nk1 * model->a_bohr / (4.0 * M_PI);  // 1 / (2 |b_1|)
    sp.cov_c2 = model->nk2 * model->a_bohr / (4.0 * M_PI);
  }
  const int64_t split_stride = (int64_t)batch * zstride;
  sp.zsplit_stride = split_stride;
  // projection rows: the rank (low rank) or every off-diagonal channel's rows (channel-wise)
  const int prows = channel ? npair * ch_ls : (int)op->rank;
  const int64_t pcols = channel ? nk : n;
  const unsigned groups = (unsigned)((prows + ROWS - 1) / ROWS);

  auto project = [&](const void* xin, int active, hipEvent_t ea = nullptr, hipEvent_t eb = nullptr) {
    sp.zsplit = zsplit;
    const dim3 g(groups, zsplit, active);
    const int chr = (int)(channel ? op->rank : 0);
    if (op->dtype == TDG_C128)
      hipExtLaunchKernelGGL(project_kernel<double>, g, dim3(PROJ_THREADS), 0u, ctx->stream, ea, eb, 0u, op->w, pcols,
                            prows, xin, xstride, z, zstride, zslice, split_stride, ch_ls, chr);
    else
      hipExtLaunchKernelGGL(project_kernel<float>, g, dim3(PROJ_THREADS), 0u, ctx->stream, ea, eb, 0u, op->w, pcols,
                            prows, xin, xstride, z, zstride, zslice, split_stride, ch_ls, chr);
  };
  const bool projects = lowrank || channel;
  // instances with len > step integrate; those with len == step only record
  auto count_gt = [&](int64_t step) {
    int c = 0;
    while (c < batch && len[c] > step) ++c;
    return c;
  };
  auto count_ge = [&](int64_t step) {
    int c = 0;
    while (c < batch && len[c] >= step) ++c;
    return c;
  };

  if (batched) {
    // split-K so that each product launches about 1024 blocks of 64 rows;
    // the default slices are multiples of 32 complex columns (whole LDS
    // stages of every tiling: 16 columns, or 32 for BF16X2 tiling 3)
    const int tile = 64;
    auto kslice_for = [&](int64_t M, int64_t Kc) {
      const int64_t tiles = ((M + tile - 1) / tile) * ((batch + 63) / 64);
      int64_t splits = std::max<int64_t>(1, std::min<int64_t>(64, (1024 + tiles - 1) / tiles));
      int64_t ks = (Kc + splits - 1) / splits;
      ks = std::max<int64_t>(32, (ks + 31) / 32 * 32);
      return ks;
    };
    const int64_t ldy = xstride;
    int64_t ks_main, ks_proj = 0;
    int y_slices, z_slices = 0;
    void* Ybuf = nullptr;
    void* Zbuf = nullptr;
    void* Zsum = nullptr;
    // the buffers hold up to twice the default number of slices (tuner range)
    if (!lowrank) {
      ks_main = kslice_for(n, n);
      y_slices = (int)((n + ks_main - 1) / ks_main);
      TDG_TRY(ws_reserve(ctx, WS_Y, (size_t)2 * y_slices * n * ldy * 8, &Ybuf));
    } else {
      ks_proj = kslice_for(op->rank, n);
      z_slices = (int)((n + ks_proj - 1) / ks_proj);
      TDG_TRY(ws_reserve(ctx, WS_Z, (size_t)2 * z_slices * op->rank * ldy * 8, &Zbuf));
      // the expansion has few K columns (the rank): split it too, at most 8
      // ways, and let the stage kernel sum the slices it reads
      ks_main = std::max<int64_t>(kslice_for(n, op->rank), (op->rank + 7) / 8);
      ks_main = (ks_main + 31) / 32 * 32;
      y_slices = (int)((op->rank + ks_main - 1) / ks_main);
      TDG_TRY(ws_reserve(ctx, WS_Y, (size_t)2 * y_slices * n * ldy * 8, &Ybuf));
      TDG_TRY(ws_reserve(ctx, WS_ZSUM, (size_t)op->rank * ldy * 8, &Zsum));
    }
    BatchParams bp = {};
    bp.Y = (const float2*)Ybuf;
    bp.ldy = ldy;
    bp.y_slices = y_slices;
    bp.y_slice_stride = n * ldy;
    bp.kdiag = lowrank ? (const float2*)op->kdiag : nullptr;
    bp.ldx = xstride;
    bp.rho_n = (double2*)rho_n;
    bp.rho_s = (double2*)rho_s;
    bp.acc = (double2*)acc;
    bp.eps = model->eps;
    bp.dip = (const double2*)model->dip;
    bp.vel = (const double2*)model->vel;
    bp.fields = (const tdg_field*)dfields;
    bp.obs_part = (double*)part;
    bp.nk = nk;
    bp.nb = model->nb;
    bp.nv = model->nv;
    bp.npair = npair;
    bp.block = op->block;
    bp.batch = batch;
    bp.dt = dt;
    bp.tr_signed = intra;
    bp.ftab = (const double*)ftab;
    // the elements the stage kernel updates (Hermitian-packed unless the
    // intraband term is on), the ones that read the product first
    bp.nelem = 0;
    int npe = 0;  // pair elements
    for (int pass = 0; pass < 2; ++pass)
      for (int r = 0; r < model->nb; ++r)
        for (int c = 0; c < model->nb; ++c) {
          if (!intra && c < r) continue;
          const bool pair = op->block == TDG_BLOCK_ALL || (r >= model->nv) != (c >= model->nv);
          if (pair == (pass == 0)) bp.elist[bp.nelem++] = r * model->nb + c;
          if (pair && pass == 0) ++npe;
        }
    const bool pair_slot0 = npe <= model->nb;
    // stage kernel blocks: IB instances x nb rows, LDS for their H and rho blocks and row sums
    int IB = 16;  // instances per block: up to 64 for nb <= 4, matched to the batch
    while (model->nb <= 4 && IB < 64 && IB < batch) IB *= 2;
    // H and rho blocks; the observable sums share the H blocks' space when they fit (nb >= 3)
    const size_t stage_lds = (size_t)2 * nb2 * IB * sizeof(double2) +
                             (model->nb >= 3 ? 0 : (size_t)(5 * model->nb * IB + 1) / 2 * sizeof(double2)) +
                             (size_t)4 * nb2 * sizeof(double2) + (size_t)model->nb * sizeof(double);

    // tiling and split-K of each product (pick below): the tuner runs the
    // products on the step-0 operands; they only write Y / Z, which the loop
    // below recomputes
    int gv_main = 0, gv_proj = 0;
    const int n_dyn0 = count_gt(0);
    // BF16X2: tilings 1 to 4 need X split once into a bf16 work array
    void* xbw = nullptr;
    if (bf16) TDG_TRY(ws_reserve(ctx, WS_XB, cgemm_bf16x2_work_bytes((int)n, batch), &xbw));
    // With those tilings the stage kernel can write the next gather split as
    // well, which saves the product's own split of X (64 instances per stage
    // block and whole 16-byte chunks of 4 pairs).  The array is cleared once:
    // its padding past 2N stays zero.
    void* xe = nullptr;
    const bool fuse_ok = bf16 && IB == tdg::XB_TILE && npair % 4 == 0;
    if (fuse_ok) {
      const size_t xe_bytes = cgemm_bf16x2_work_bytes((int)n, batch);
      TDG_TRY(ws_reserve(ctx, WS_XE, xe_bytes, &xe));
      TDG_TRY(hip_check(ctx, hipMemsetAsync(xe, 0, xe_bytes, ctx->stream), "split gather clear"));
    }
    // FP32: 64-row, prefetching 64-row, 128-row; BF16X2: 64-row, 128-row,
    // 256-row, 128-row with 64 real K per stage, 128-row direct-to-LDS
    const int ntilings = bf16 ? 5 : 3;
    if (n_dyn0 > 0) {
      // Split-K candidates: the default (about 1024 blocks), no split, twice
      // the default, and slice counts that put about 256 j blocks (j = 1..4)
      // on the 256 CUs; at most twice the default (the buffers' size).
      // Slice widths are multiples of 16 complex columns (one LDS stage of
      // every tiling); the counts aim at about 256 j blocks for 64-row tiles
      // (j = 1..4) and for the 128- and 256-row tiles (j = 1, 2).
      auto split_options = [&](int64_t M, int64_t Kc, int64_t ks_def) {
        const int64_t ctiles = (n_dyn0 + 63) / 64;
        const int64_t s_def = (Kc + ks_def - 1) / ks_def;
        std::vector<int64_t> out{ks_def};
        std::vector<int64_t> counts{1, 2 * s_def};
        for (int j = 1; j <= 4; ++j) counts.push_back((256 * j) / (((M + tile - 1) / tile) * ctiles));
        for (int64_t rows : {128, 256})
          for (int j = 1; j <= 2; ++j) counts.push_back((256 * j) / (((M + rows - 1) / rows) * ctiles));
        for (int64_t sc : counts) {
          if (sc < 1 || sc > 2 * s_def) continue;
          const int64_t ks = std::max<int64_t>(16, ((Kc + sc - 1) / sc + 15) / 16 * 16);
          if (std::find(out.begin(), out.end(), ks) == out.end()) out.push_back(ks);
        }
        return out;
      };
      // tiling v and slice width ks of one product: forced tiling (default or
      // forced split), cached for its shape, or timed now (the projection's
      // timing includes the sum of its slices)
      auto pick = [&](const char* what, int64_t M, int64_t Kc, int64_t ks_def,
                      const std::function<void(int, int64_t)>& run, int* out_v, int64_t* out_ks) -> int {
        // forced slice count (TDG_OPT_GEMM_SLICES), at most twice the default (the buffers' size)
        int64_t ks_forced = 0;
        if (ctx->gemm_slices > 0) {
          const int64_t s_def = (Kc + ks_def - 1) / ks_def;
          const int64_t sc = std::max<int64_t>(1, std::min<int64_t>(ctx->gemm_slices, 2 * s_def));
          ks_forced = std::max<int64_t>(32, ((Kc + sc - 1) / sc + 31) / 32 * 32);
        }
        *out_ks = ks_forced > 0 ? ks_forced : ks_def;
        if (ctx->gemm_variant >= 0) {
          *out_v = std::min(ctx->gemm_variant, ntilings - 1);
          return TDG_OK;
        }
        char key[160];
        snprintf(key, sizeof(key), "gemm/%s/%s/%lld/%lld/%d/%lld/%lld", bf16 ? "bf16x2" : "f32", what, (long long)M,
                 (long long)Kc, n_dyn0, (long long)ks_def, (long long)ks_forced);
        for (auto& kv : ctx->tuned)
          if (kv.first == key) {
            *out_v = kv.second % 8;
            *out_ks = kv.second / 8;
            return TDG_OK;
          }
        const std::vector<int64_t> opts =
            ks_forced > 0 ? std::vector<int64_t>{ks_forced} : split_options(M, Kc, ks_def);
        const size_t ncand = opts.size() * ntilings;
        TunerEvents te;
        TDG_TRY(te.create(ctx, 2 * ncand));
        const std::vector<hipEvent_t>& ev = te.ev;
        // one untimed round, then each candidate timed once per round, right
        // after another candidate's run (back-to-back repeats of one product
        // slow down and would penalise the wider splits)
        std::vector<float> tmin(ncand, 1e30f);
        for (int round = 0; round < 6; ++round) {
          for (size_t c = 0; c < ncand; ++c) {
            (void)hipEventRecord(ev[2 * c], ctx->stream);
            run((int)(c % ntilings), opts[c / ntilings]);
            (void)hipEventRecord(ev[2 * c + 1], ctx->stream);
          }
          TDG_TRY(hip_check(ctx, hipEventSynchronize(ev[2 * ncand - 1]), "GEMM tuning"));
          for (size_t c = 0; c < ncand && round > 0; ++c) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1]) != hipSuccess) ms = 1e30f;
            tmin[c] = std::min(tmin[c], ms);
          }
        }
        // the earliest (split, tiling) within 2 % of the fastest (the default split first)
        const float fastest = *std::min_element(tmin.begin(), tmin.end());
        int bestv = 0;
        int64_t bestks = ks_def;
        bool found = false;
        for (size_t oi = 0; oi < opts.size() && !found; ++oi)
          for (int v = 0; v < ntilings; ++v)
            if (tmin[oi * ntilings + v] <= 1.02f * fastest) {
              bestv = v;
              bestks = opts[oi];
              found = true;
              break;
            }
        TDG_TRY(launch_check(ctx, "GEMM tuning"));
        ctx->tuned.emplace_back(key, (int)(bestks * 8 + bestv));
        *out_v = bestv;
        *out_ks = bestks;
        return TDG_OK;
      };
      // The stage kernel reads every slice of the dense or expansion product:
      // their timing includes one fixed-order pass over the slices as a proxy.
      void* slice_out = nullptr;
      TDG_TRY(ws_reserve(ctx, WS_TMP2, (size_t)n * ldy * 8, &slice_out));
      auto slice_read = [&](int slices) {
        sum_slices_c64(ctx->stream, Ybuf, slices, n * ldy, n * ldy, slice_out);
      };
      // timing operand: a non-zero pattern in the second gather buffer, which
      // stage 0 of step 0 overwrites
      void* xt = x1;
      hipLaunchKernelGGL(pattern_fill_kernel, dim3(1024), dim3(256), 0, ctx->stream, (float2*)xt,
                         (int64_t)n * xstride);
      // tilings 1 to 4 then read X split by the stage kernel: timed without their own split
      if (fuse_ok) expand_bf16x2(ctx->stream, xt, xstride, (int)n, n_dyn0, xe);
      auto gemm_x = [&](hipStream_t st, const void* A, int64_t lda, int M, const void* X, void* Y, int64_t ystride,
                        int ks, int v) {
        if (fuse_ok && v > 0)
          cgemm_bf16x2(st, A, lda, M, (int)n, nullptr, xstride, Y, ldy, ystride, n_dyn0, ks, v, xe, true);
        else
          cgemm_bf16x2(st, A, lda, M, (int)n, X, xstride, Y, ldy, ystride, n_dyn0, ks, v, xbw);
      };
      const int64_t ld_us0 = bf16 ? (op->rank + 3) / 4 * 4 : op->rank;
      if (!lowrank) {
        TDG_TRY(pick("dense", n, n, ks_main, [&](int v, int64_t ks) {
          if (bf16)
            gemm_x(ctx->stream, op->K, op->ld, (int)n, xt, Ybuf, n * ldy, (int)ks, v);
          else
            cgemm_f32(ctx->stream, op->K, op->ld, (int)n, (int)n, xt, xstride, Ybuf, ldy, n * ldy, n_dyn0,
                      (int)ks, v);
          slice_read((int)((n + ks - 1) / ks));
        }, &gv_main, &ks_main));
        y_slices = (int)((n + ks_main - 1) / ks_main);
      } else {
        TDG_TRY(pick("project", op->rank, n, ks_proj, [&](int v, int64_t ks) {
          if (bf16)
            gemm_x(ctx->stream, op->w, n, (int)op->rank, xt, Zbuf, op->rank * ldy, (int)ks, v);
          else
            cgemm_f32(ctx->stream, op->w, n, (int)op->rank, (int)n, xt, xstride, Zbuf, ldy, op->rank * ldy,
                      n_dyn0, (int)ks, v);
          sum_slices_c64(ctx->stream, Zbuf, (int)((n + ks - 1) / ks), op->rank * ldy, op->rank * ldy, Zsum);
        }, &gv_proj, &ks_proj));
        z_slices = (int)((n + ks_proj - 1) / ks_proj);
        // Zsum now holds the step-0 projection (the expansion's timing input)
        // BF16X2 tilings 1 to 4 take the split projection straight from its
        // slices (one kernel instead of the slice sum and the split); tiling
        // 0 reads the summed projection, so its timing includes the sum
        TDG_TRY(pick("expand", n, op->rank, ks_main, [&](int v, int64_t ks) {
          if (bf16 && v > 0) {
            sum_expand_bf16x2(ctx->stream, Zbuf, z_slices, op->rank * ldy, (int)op->rank, ldy, n_dyn0, xbw);
            cgemm_bf16x2(ctx->stream, op->us, ld_us0, (int)n, (int)op->rank, nullptr, ldy, Ybuf, ldy, n * ldy,
                         n_dyn0, (int)ks, v, xbw, true);
          } else if (bf16) {
            sum_slices_c64(ctx->stream, Zbuf, z_slices, op->rank * ldy, op->rank * ldy, Zsum);
            cgemm_bf16x2(ctx->stream, op->us, ld_us0, (int)n, (int)op->rank, Zsum, ldy, Ybuf, ldy, n * ldy, n_dyn0,
                         (int)ks, v, xbw);
          } else
            cgemm_f32(ctx->stream, op->us, op->rank, (int)n, (int)op->rank, Zsum, ldy, Ybuf, ldy, n * ldy,
                      n_dyn0, (int)ks, v);
          slice_read((int)((op->rank + ks - 1) / ks));
        }, &gv_main, &ks_main));
        y_slices = (int)((op->rank + ks_main - 1) / ks_main);
      }
      bp.y_slices = y_slices;
    }
    // the stage kernel writes the next gather split when the product that
    // reads the gather (the projection, or the dense product) uses tiling 1
    // or 2; the first stage's gather is split here
    const bool fuse_x = fuse_ok && (lowrank ? gv_proj : gv_main) > 0;
    bp.xexp = fuse_x ? (unsigned short*)xe : nullptr;
    bp.ldxb = 2 * ((n + 31) / 32 * 32);
    if (fuse_x) expand_bf16x2(ctx->stream, x0, xstride, (int)n, n_dyn0, xe);
    const size_t stage_lds_run = stage_lds + (fuse_x ? (size_t)npair * IB * sizeof(float2) : 0);
    ctx->last_variant = std::string(lowrank ? "batched_mfma_lowrank_" : "batched_mfma_dense_") +
                        (bf16 ? "bf16x2" : "f32");
    ctx->last_variant += lowrank ? " (tilings " + std::to_string(gv_proj) + "/" + std::to_string(gv_main) +
                                       ", slices " + std::to_string(z_slices) + "/" + std::to_string(y_slices) + ")"
                                 : " (tiling " + std::to_string(gv_main) + ", slices " + std::to_string(y_slices) + ")";
    if (ctx->graphs && !ctx->prof) ctx->last_variant += " graphs";
    tdg_obs ob = *obs;
    void* dstep = nullptr;
    TDG_TRY(ws_reserve(ctx, WS_STEP, 256, &dstep));
    bp.chunk = chunk;

    // One RK4 step's launches on stream st.  dev_step: the stage kernels read
    // the step from the device counter (the form captured into graphs); every
    // step ends by advancing that counter.
    auto issue_step = [&](hipStream_t st, int64_t step, int slot_, int n_obs, int n_dyn, bool dev_step, bool prof) {
      bp.n_dyn = n_dyn;
      bp.step_dev = dev_step ? (const int*)dstep : nullptr;
      void* xc = x0;
      void* xn = x1;
      for (int s = 0; s < 4; ++s) {
        const int active = s == 0 ? n_obs : n_dyn;
        if (active == 0) break;
        if (n_dyn > 0) {
          if (prof) prof_begin(ctx, TDG_KCLASS_GEMM);
          const int64_t ld_us = bf16 ? (op->rank + 3) / 4 * 4 : op->rank;
          if (!lowrank) {
            if (fuse_x)
              cgemm_bf16x2(st, op->K, op->ld, (int)n, (int)n, nullptr, xstride, Ybuf, ldy, n * ldy, n_dyn,
                           (int)ks_main, gv_main, xe, true);
            else if (bf16)
              cgemm_bf16x2(st, op->K, op->ld, (int)n, (int)n, xc, xstride, Ybuf, ldy, n * ldy, n_dyn, (int)ks_main,
                           gv_main, xbw);
            else
              cgemm_f32(st, op->K, op->ld, (int)n, (int)n, xc, xstride, Ybuf, ldy, n * ldy, n_dyn,
                        (int)ks_main, gv_main);
          } else {
            // projection split over K, summed once in fixed order, then expansion
            if (fuse_x)
              cgemm_bf16x2(st, op->w, n, (int)op->rank, (int)n, nullptr, xstride, Zbuf, ldy, op->rank * ldy, n_dyn,
                           (int)ks_proj, gv_proj, xe, true);
            else if (bf16)
              cgemm_bf16x2(st, op->w, n, (int)op->rank, (int)n, xc, xstride, Zbuf, ldy, op->rank * ldy, n_dyn,
                           (int)ks_proj, gv_proj, xbw);
            else
              cgemm_f32(st, op->w, n, (int)op->rank, (int)n, xc, xstride, Zbuf, ldy, op->rank * ldy, n_dyn,
                        (int)ks_proj, gv_proj);
            if (bf16 && gv_main > 0) {
              sum_expand_bf16x2(st, Zbuf, z_slices, op->rank * ldy, (int)op->rank, ldy, n_dyn, xbw);
              cgemm_bf16x2(st, op->us, ld_us, (int)n, (int)op->rank, nullptr, ldy, Ybuf, ldy, n * ldy, n_dyn,
                           (int)ks_main, gv_main, xbw, true);
            } else {
              sum_slices_c64(st, Zbuf, z_slices, op->rank * ldy, op->rank * ldy, Zsum);
              if (bf16)
                cgemm_bf16x2(st, op->us, ld_us, (int)n, (int)op->rank, Zsum, ldy, Ybuf, ldy, n * ldy, n_dyn,
                             (int)ks_main, gv_main, xbw);
              else
                cgemm_f32(st, op->us, op->rank, (int)n, (int)op->rank, Zsum, ldy, Ybuf, ldy, n * ldy, n_dyn,
                          (int)ks_main, gv_main);
            }
          }
          if (prof) prof_end(ctx, TDG_KCLASS_GEMM);
        }
        bp.xcur = (const float2*)xc;
        bp.xnext = (float2*)xn;
        bp.step = (int)step;
        bp.stage = s;
        bp.obs_slot = slot_;
        bp.n_active = active;
        bp.intra = (intra && n_dyn > 0) ? (const double2*)dintra : nullptr;
        if (bp.intra)
          covariant_derivative(st, model, rho_s, 1, (int64_t)nb2 * xstride, xstride, (const tdg_field*)dfields, n_dyn,
                               dintra);
        if (prof) prof_begin(ctx, TDG_KCLASS_STAGE);
        // Hermitian-packed state unless the intraband term (which reads the
        // full stage state) is on
        const dim3 sg(nk, (active + IB - 1) / IB), sb(IB * model->nb);
        if (model->nb <= 4 && !intra && IB == 64 && pair_slot0)
          hipLaunchKernelGGL((batched_stage_kernel<4, true, true, true>), sg, sb, stage_lds_run, st, bp);
        else if (model->nb <= 4 && !intra && IB == 64)
          hipLaunchKernelGGL((batched_stage_kernel<4, true, true>), sg, sb, stage_lds_run, st, bp);
        else if (model->nb <= 4 && IB == 64)
          hipLaunchKernelGGL((batched_stage_kernel<4, false, true>), sg, sb, stage_lds_run, st, bp);
        else if (model->nb <= 4 && !intra)
          hipLaunchKernelGGL((batched_stage_kernel<4, true, false>), sg, sb, stage_lds_run, st, bp);
        else if (model->nb <= 4)
          hipLaunchKernelGGL((batched_stage_kernel<4, false, false>), sg, sb, stage_lds_run, st, bp);
        else if (!intra)
          hipLaunchKernelGGL((batched_stage_kernel<TDG_NB_MAX, true, false>), sg, sb, stage_lds_run, st, bp);
        else
          hipLaunchKernelGGL((batched_stage_kernel<TDG_NB_MAX, false, false>), sg, sb, stage_lds_run, st, bp);
        if (prof) prof_end(ctx, TDG_KCLASS_STAGE);
        std::swap(xc, xn);
      }
      hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, st, (int*)dstep);
    };

    // Graph replays (TDG_OPT_GRAPHS): a step in which no instance reaches its
    // final time is the same launch sequence for a given running count; it is
    // captured once per count on a private stream and replayed on the
    // context stream.  Steps where instances finish, the observable
    // reductions and profiled runs stay direct launches.
    const bool use_graphs = ctx->graphs && !ctx->prof;
    std::vector<std::pair<int, hipGraphExec_t>> execs;
    hipStream_t cap = nullptr;
    auto release = [&]() {
      for (auto& e : execs) (void)hipGraphExecDestroy(e.second);
      execs.clear();
      if (cap) (void)hipStreamDestroy(cap);
      cap = nullptr;
    };
    if (use_graphs && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
      return fail(ctx, TDG_E_HIP, "capture stream");
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, ctx->stream, (int*)dstep, 0);
    int slot = 0;
    int64_t chunk_start = 0;
    int rc = TDG_OK;
    for (int64_t step = 0; step <= max_steps && rc == TDG_OK; ++step) {
      const int n_obs = count_ge(step), n_dyn = count_gt(step);
      if (slot == 0) field_table(step);
      if (use_graphs && n_dyn > 0 && n_obs == n_dyn) {
        hipGraphExec_t ex = nullptr;
        for (auto& e : execs)
          if (e.first == n_dyn) ex = e.second;
        if (!ex) {
          hipGraph_t g = nullptr;
          if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(ctx, TDG_E_HIP, "graph capture begin");
            break;
          }
          issue_step(cap, step, 0, n_obs, n_dyn, true, false);
          const hipError_t e1 = hipStreamEndCapture(cap, &g);
          const hipError_t e2 = e1 == hipSuccess ? hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) : e1;
          if (g) (void)hipGraphDestroy(g);
          if (e2 != hipSuccess) {
            rc = fail(ctx, TDG_E_HIP, "graph capture: %s", hipGetErrorString(e2));
            break;
          }
          execs.emplace_back(n_dyn, ex);
        }
        if (hipGraphLaunch(ex, ctx->stream) != hipSuccess) {
          rc = fail(ctx, TDG_E_HIP, "graph launch");
          break;
        }
      } else {
        issue_step(ctx->stream, step, slot, n_obs, n_dyn, false, ctx->prof);
      }
      ++slot;
      if (slot == chunk || step == max_steps) {
        hipLaunchKernelGGL(obs_reduce_kernel, dim3(slot, batch), dim3(THREADS), 0, ctx->stream, (const double*)part,
                           nk, batch, (int)chunk_start, (const tdg_field*)dfields, (const int*)dperm, ob,
                           (double*)nullptr, (int)intra);
        chunk_start += slot;
        slot = 0;
      }
      if ((step & 63) == 0) rc = launch_check(ctx, "batched propagation launch");
    }
    // the graph executables are destroyed only after their replays finished
    if (use_graphs) {
      const hipError_t es = hipStreamSynchronize(ctx->stream);
      if (es != hipSuccess && rc == TDG_OK) rc = fail(ctx, TDG_E_HIP, "graph replay: %s", hipGetErrorString(es));
    }
    release();
    TDG_TRY(rc);
    hipLaunchKernelGGL(finish_batched_kernel, dim3(nk), dim3(256), 0, ctx->stream, (const double2*)rho_n,
                       (const int*)dperm, (double2*)rho, xstride, nk, model->nb, batch, (int)!intra);
    return launch_check(ctx, "batched propagation launch");
  }

  // ---- variant choice ------------------------------------------------------
  const Variant* vt = nullptr;
  int nvar = 0;
  if (op->dtype == TDG_C128)
    channel ? table(kChanF64, vt, nvar) : (lowrank ? table(kLowF64, vt, nvar) : table(kDenseF64, vt, nvar));
  else
    channel ? table(kChanF32, vt, nvar) : (lowrank ? table(kLowF32, vt, nvar) : table(kDenseF32, vt, nvar));
  int var = 0;
  sp.zsplit = zsplit;
  // low rank: the tuner also picks the projection's column split
  const bool tune_split = lowrank && !batched;
  const int splits[3] = {1, 2, ZSPLIT_MAX};

  if (ctx->forced_variant >= 0) {
    if (ctx->forced_variant >= nvar)
      return fail(ctx, TDG_E_INVAL, "variant %d of %d for this operator", ctx->forced_variant, nvar);
    var = ctx->forced_variant;
  } else if (ctx->autotune && max_steps > 0) {
    char key[160];
    snprintf(key, sizeof(key), "%d/%d/%lld/%d/%d/%lld/%d", op->kind, op->dtype, (long long)n, nk, batch,
             (long long)op->rank, op->block);
    int found = -1;
    for (auto& kv : ctx->tuned)
      if (kv.first == key) found = kv.second;
    if (found >= 0) {
      var = found % 100;
      if (tune_split) set_split(splits[found / 100]);
    } else if (!fixed) {
      // time each variant on stage 0 of step 0: it reads rho and writes only
      // the stage state, accumulator and next gather, which init restores
      TunerEvents te;
      TDG_TRY(te.create(ctx, 2));
      const hipEvent_t ea = te.ev[0], eb = te.ev[1];
      const int dyn0 = count_gt(0);
      field_table(0);
      sp.step = 0;
      sp.stage = 0;
      sp.obs_slot = 0;
      sp.n_dyn = dyn0;
      sp.xcur = x0;
      sp.xnext = x1;
      sp.vec = projects ? z : x0;
      sp.vstride = projects ? zstride : xstride;
      const dim3 g(nk, dyn0);
      // three interleaved rounds of 8 repetitions per (split, variant); the
      // fastest round counts (single short timings vary by tens of per cent)
      float tmin[3][8];
      for (auto& row : tmin)
        for (float& x : row) x = 1e30f;
      const int nsplit = tune_split ? 3 : 1;
      for (int round = 0; round < 3; ++round) {
        for (int si = 0; si < nsplit; ++si) {
          if (tune_split) set_split(splits[si]);
          // with the split tuned, each timed repetition includes the projection
          auto run = [&](int v) {
            if (projects && (tune_split || si == 0)) project(x0, dyn0);
            vt[v].fn(g, 0, ctx->stream, sp, nullptr, nullptr);
          };
          if (projects && !tune_split) project(x0, dyn0);
          for (int v = 0; v < nvar; ++v) {
            run(v);  // warm-up
            (void)hipEventRecord(ea, ctx->stream);
            for (int rep = 0; rep < 8; ++rep) {
              if (tune_split) {
                run(v);
              } else {
                vt[v].fn(g, 0, ctx->stream, sp, nullptr, nullptr);
              }
            }
            (void)hipEventRecord(eb, ctx->stream);
            TDG_TRY(launch_check(ctx, "tuner launch"));
            TDG_TRY(hip_check(ctx, hipEventSynchronize(eb), "tuner sync"));
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ea, eb) != hipSuccess) ms = 1e30f;
            tmin[si][v] = std::min(tmin[si][v], ms);
          }
        }
      }
      // the earliest (split, variant) within 2 % of the fastest: near-equal
      // candidates would otherwise alternate between runs with timing noise
      float fastest = 1e30f;
      for (int si = 0; si < nsplit; ++si)
        for (int v = 0; v < nvar; ++v) fastest = std::min(fastest, tmin[si][v]);
      int best_split = -1;
      for (int si = 0; si < nsplit && best_split < 0; ++si)
        for (int v = 0; v < nvar; ++v)
          if (tmin[si][v] <= 1.02f * fastest) {
            var = v;
            best_split = si;
            break;
          }
      if (tune_split) set_split(splits[best_split]);
      ctx->tuned.emplace_back(key, var + 100 * best_split);
      TDG_TRY(init());  // the caller's rho was only read
    }
  }
  ctx->last_variant = vt[var].name;
  if (tune_split) ctx->last_variant += "_z" + std::to_string(zsplit);
  sp.zsplit = zsplit;
  const StageLaunch stage_fn = vt[var].fn;

  tdg_obs ob = *obs;
  void* xc = x0;
  void* xn = x1;
  // one observable chunk: the field table, steps c0 .. c1 - 1, the reduction
  auto issue_chunk = [&](int64_t c0, int64_t c1) {
    field_table(c0);
    for (int64_t step = c0; step < c1; ++step) {
      const int n_obs = count_ge(step), n_dyn = count_gt(step);
      sp.n_dyn = n_dyn;
      for (int s = 0; s < 4; ++s) {
        const int active = s == 0 ? n_obs : n_dyn;
        if (active == 0) break;
        if (projects && n_dyn > 0) {
          hipEvent_t pa = nullptr, pb = nullptr;
          if (!fixed) prof_pair(ctx, TDG_KCLASS_PROJECT, &pa, &pb);
          project(xc, n_dyn, pa, pb);
        }
        sp.vec = projects ? z : xc;
        sp.vstride = projects ? zstride : xstride;
        sp.xcur = xc;
        sp.xnext = xn;
        sp.step = (int)step;
        sp.stage = s;
        sp.obs_slot = (int)(step - c0);
        hipEvent_t sa = nullptr, sb = nullptr;
        if (!fixed) prof_pair(ctx, TDG_KCLASS_STAGE, &sa, &sb);
        stage_fn(dim3(nk, active), 0, ctx->stream, sp, sa, sb);
        std::swap(xc, xn);
        // with links the next stage reads the buffer this one wrote (four
        // stages per step: every step starts from the first buffer)
        if (sp.links) std::swap(sp.rho_s, sp.rho_s_out);
      }
    }
    hipLaunchKernelGGL(obs_reduce_kernel, dim3((unsigned)(c1 - c0), batch), dim3(THREADS), 0, ctx->stream,
                       (const double*)part, nk, batch, (int)c0, (const tdg_field*)dfields, (const int*)dperm, ob,
                       (double*)nullptr, (int)intra);
  };
  // Graph replays (TDG_OPT_GRAPHS): a full chunk in which every running
  // instance runs through is captured on a private stream (its launches
  // read ctx->stream) and replayed once on the context stream; the host
  // captures the next chunk while the GPU runs this one.  Profiled and
  // allocation-free runs launch directly.
  const bool use_graphs = ctx->graphs && !ctx->prof && !fixed;
  std::vector<hipGraphExec_t> execs;
  hipStream_t cap = nullptr;
  if (use_graphs && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
    return fail(ctx, TDG_E_HIP, "capture stream");
  int rc = TDG_OK;
  for (int64_t c0 = 0; c0 <= max_steps && rc == TDG_OK; c0 += chunk) {
    const int64_t c1 = std::min<int64_t>(c0 + chunk, max_steps + 1);
    const bool uniform = c1 - c0 == chunk && c1 - 1 < max_steps && count_gt(c1 - 1) == count_ge(c0);
    if (use_graphs && uniform) {
      hipStream_t own = ctx->stream;
      if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = fail(ctx, TDG_E_HIP, "graph capture begin");
        break;
      }
      ctx->stream = cap;
      issue_chunk(c0, c1);
      ctx->stream = own;
      hipGraph_t g = nullptr;
      hipGraphExec_t ex = nullptr;
      const hipError_t e1 = hipStreamEndCapture(cap, &g);
      const hipError_t e2 = e1 == hipSuccess ? hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) : e1;
      if (g) (void)hipGraphDestroy(g);
      if (e2 != hipSuccess) {
        rc = fail(ctx, TDG_E_HIP, "graph capture: %s", hipGetErrorString(e2));
        break;
      }
      execs.push_back(ex);
      if (hipGraphLaunch(ex, ctx->stream) != hipSuccess) rc = fail(ctx, TDG_E_HIP, "graph launch");
    } else {
      issue_chunk(c0, c1);
      rc = launch_check(ctx, "propagation launch");
    }
  }
  // the graph executables are destroyed only after their replays finished
  if (use_graphs) {
    const hipError_t es = hipStreamSynchronize(ctx->stream);
    if (es != hipSuccess && rc == TDG_OK) rc = fail(ctx, TDG_E_HIP, "graph replay: %s", hipGetErrorString(es));
    for (hipGraphExec_t e : execs) (void)hipGraphExecDestroy(e);
    (void)hipStreamDestroy(cap);
    if (!execs.empty()) ctx->last_variant += " graphs";
  }
  TDG_TRY(rc);
  hipLaunchKernelGGL(finish_kernel, dim3(nk, batch), dim3(init_threads), 0, ctx->stream, (const double2*)rho_n,
                     (const int*)dperm, (double2*)rho, nk, nb2);
  return launch_check(ctx, "propagation launch");
}

extern "C" int tdg_propagate(tdg_ctx ctx, const tdg_operator* op, const tdg_model* model, const tdg_field* fields,
                             int32_t batch, double dt, void* rho, int32_t init_eq, const tdg_obs* obs) {
  if (!ctx) return TDG_E_INVAL;
  Workspace W{ctx};
  return propagate_impl(ctx, op, model, fields, batch, dt, rho, init_eq, obs, W);
}

// ---- allocation-free propagation ---------------------------------------------
// The workspace of tdg_propagate_noalloc.  Each device holds its own copy from
// the load of the library's code object until the process ends.  Host code
// never uses this name for the memory (on the host it is only a stand-in):
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[TDG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_DEVICES] = {};
}  // namespace

namespace tdg {

int scratch_init(int device) {
  if (device < 0 || device >= SCRATCH_DEVICES)
    return fail(nullptr, TDG_E_UNSUPPORTED, "device %d: at most %d devices", device, SCRATCH_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return TDG_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(nullptr, TDG_E_HIP, "device %d: address of the scratch array: %s", device, hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return TDG_OK;
}

}  // namespace tdg

extern "C" int tdg_propagate_noalloc(tdg_ctx ctx, const tdg_operator* op, const tdg_model* model,
                                     const tdg_field* fields, int32_t batch, double dt, void* rho, int32_t init_eq,
                                     const tdg_obs* obs) {
  if (!ctx) return TDG_E_INVAL;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < SCRATCH_DEVICES) base = g_scratch_ptr[ctx->device];
  }
  if (!base) return fail(ctx, TDG_E_HIP, "no scratch array address for device %d", ctx->device);
  Workspace W{ctx, (char*)base, (size_t)TDG_NOALLOC_SCRATCH_BYTES};
  return propagate_impl(ctx, op, model, fields, batch, dt, rho, init_eq, obs, W);
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
  void *part = nullptr, *dfields = nullptr;
  TDG_TRY(ws_reserve(ctx, WS_OBS_PART, (size_t)batch * nk * 5 * sizeof(double), &part));
  TDG_TRY(ws_reserve(ctx, WS_FIELDS, sizeof(tdg_field) * batch, &dfields));
  TDG_TRY(args_upload(ctx, dfields, fields, sizeof(tdg_field) * batch));
  StageParams sp = {};
  sp.rho_s = (double2*)rho;
  sp.dip = (const double2*)model->dip;
  sp.vel = (const double2*)model->vel;
  sp.fields = (const tdg_field*)dfields;
  sp.obs_part = (double*)part;
  sp.obs_slot = 0;
  sp.nk = nk;
  sp.nb = model->nb;
  sp.nv = model->nv;
  sp.batch = batch;
  sp.tr_signed = model->links != nullptr;
  hipLaunchKernelGGL(obs_state_kernel, dim3(nk, batch), dim3(64), 0, ctx->stream, sp);
  TDG_TRY(launch_check(ctx, "observables launch"));
  tdg_obs none = {};
  hipLaunchKernelGGL(obs_reduce_kernel, dim3(1, batch), dim3(THREADS), 0, ctx->stream, (const double*)part, nk, batch,
                     0, (const tdg_field*)dfields, (const int*)nullptr, none, out, sp.tr_signed);
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
