// Reverse-mode derivative of the RK4 propagation: the exact gradient of the
// discrete scheme integrated by tdg_propagate (classical RK4, the field at
// t_n, t_n + dt/2 twice and t_n + dt), for a real loss L given through its
// cotangents on the observable series P, J, occupation.  The paper integrates
// forward only; this is the standard adjoint of an explicit Runge-Kutta step.
//
// For f(t, y) = -i [H(t, y), y], H = diag(eps) + dSigma(x) - E(t) e.d with
// x = gather(y - rho_eq) and dSigma = K x (or K_diag o x + S (V^H x)), a
// cotangent g of f pulls back to
//   ybar   = i [H^H, g] + scatter(K^H sbar),
//   Sigbar = -i [y^H, g],  sbar = gather(Sigbar) (e-h block: Sigbar_cv + conj(Sigbar_vc)),
//   dL/dE  = Re sum conj(g) i [e.d, y],
//   dL/dS += sbar (V^H x)^H,  dL/dV^H += (S^H sbar) x^H.
// With the intraband term (model links) f gains -E(t) D(y), D = e.(.)_{;k} the
// covariant central difference; D is anti-self-adjoint for Re sum conj(a) b
// (transport to k + b and to k - b are each other's adjoints), so
//   ybar += E(t) D(g),  dL/dE += -Re sum conj(g) D(y),
// with D(g) = coef D(abar) + cnext D(ybar_next) from the linearity of D.
// Complex gradients are dL/dRe + i dL/dIm.  The step is pulled back from its
// fourth stage to its first: with a = dL/drho_{n+1},
//   g_4 = dt/6 a, g_3 = dt/3 a + dt ybar_4, g_2 = dt/3 a + dt/2 ybar_3,
//   g_1 = dt/6 a + dt/2 ybar_2,  dL/drho_n = a + sum_s ybar_s + (observable cotangent at t_n).
//
// Memory: rho is stored every M steps on the forward sweep; the backward
// sweep recomputes a segment's states from its checkpoint, then each step's
// four stages (states, dSigma pairs, x, z) before pulling the step back.
// Products with K, S and V (and their transposes, from copies transposed once
// per call) run as fixed-order FP64 row products, one block per row or four;
// the per-k commutator pullbacks run in the kernels below.  The factor
// gradients are accumulated once per segment as sums of outer products over
// its stage columns, in column order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace {

constexpr int AT = 64;  // threads per block of the per-k kernels (a block holds 64 / nb^2 k points)
// Threads per block of the per-k kernels that also form their rows of a
// low-rank factor product: all of them share the product, the first AT do
// the k-local work and the rest stay idle there.
constexpr int ATW = 4 * AT;
// Largest per-segment stage stash (bytes) kept instead of rerunning each
// forward step in the backward sweep.
constexpr double ADJ_STASH_BYTES = 8.0 * (1 << 30);

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ inline double field_value(const tdg_field& f, double t) {
  const double d = t - f.t0;
  return f.e0 * exp(-d * d / (2.0 * f.tau * f.tau)) * cos(f.omega * t);
}

struct AdjArgs {
  int nk, nb, nv, npair, block, batch, nsteps;
  int64_t n;  // nk * npair
  double dt;
  const double* eps;
  const double2* dip;
  const double2* vel;
  const tdg_field* fields;  // device [B]
  const double2* kdiag;     // low rank: K_diag [n]; dense: NULL
};

__device__ inline double stage_offset(int s) { return s == 0 ? 0.0 : (s == 3 ? 1.0 : 0.5); }

// Thread t of a block: local k point t / nb^2, matrix element t % nb^2.
struct Slot {
  int lk, e, k, b, nn, m;
  bool active;
  size_t g;
};

__device__ inline Slot slot_of(const AdjArgs& a) {
  Slot s;
  const int nb2 = a.nb * a.nb, kpb = AT / nb2;
  s.lk = threadIdx.x / nb2;
  s.e = threadIdx.x % nb2;
  s.k = blockIdx.x * kpb + s.lk;
  s.b = blockIdx.y;
  s.active = s.lk < kpb && s.k < a.nk;
  s.nn = s.e / a.nb;
  s.m = s.e % a.nb;
  s.g = ((size_t)s.b * a.nk + s.k) * nb2 + s.e;
  return s;
}

// Pair index of element (n, m) in the gathered vector, or -1.
__device__ inline int pair_of(const AdjArgs& a, int nn, int m) {
  if (a.block == TDG_BLOCK_ALL) return nn * a.nb + m;
  if (nn >= a.nv && m < a.nv) return (nn - a.nv) * a.nv + m;
  return -1;
}

__device__ inline double2 proj_e(const tdg_field& F, const AdjArgs& a, const double2* arr, int k, int e) {
  const size_t base = (size_t)k * a.nb * a.nb + e, plane = (size_t)a.nk * a.nb * a.nb;
  const double2 u = arr[base], v = arr[plane + base];
  return make_double2(F.ex * u.x + F.ey * v.x, F.ex * u.y + F.ey * v.y);
}

// dSigma pair value: S (from the products) plus K_diag o x for the low-rank
// form; S is [B][n].
__device__ inline double2 sigma_pair(const AdjArgs& a, const double2* S, const double2* X, int b, int k, int p) {
  const size_t i = (size_t)b * a.n + (size_t)k * a.npair + p;
  double2 v = S[i];
  if (a.kdiag) v = cadd(v, cmul(a.kdiag[(size_t)k * a.npair + p], X[i]));
  return v;
}

// Element (n, m) of H_k = diag(eps) + dSigma - E e.d (e-h block: dSigma_vc = conj(dSigma_cv)).
__device__ inline double2 ham_element(const AdjArgs& a, const double2* S, const double2* X, const Slot& s, double ef,
                                      double2 de) {
  double2 ds = make_double2(0.0, 0.0);
  const int p = pair_of(a, s.nn, s.m);
  if (p >= 0) {
    ds = sigma_pair(a, S, X, s.b, s.k, p);
  } else if (a.block == TDG_BLOCK_EH && s.nn < a.nv && s.m >= a.nv) {
    ds = cconj(sigma_pair(a, S, X, s.b, s.k, (s.m - a.nv) * a.nv + s.nn));
  }
  double2 h = make_double2(ds.x - ef * de.x, ds.y - ef * de.y);
  if (s.nn == s.m) h.x += a.eps[(size_t)s.k * a.nb + s.nn];
  return h;
}

// Cotangent of rho(t_n) from the observable weights: (gP D^H + gJ V^H) / nk,
// plus gocc / nk on the first conduction band's occupation.
__device__ inline double2 obs_cotangent(const AdjArgs& a, const Slot& s, const tdg_field& F, const double* gP,
                                        const double* gJ, const double* gocc, int64_t gstride, int step) {
  const size_t w = (size_t)s.b * gstride + step;
  const double wp = gP ? gP[w] : 0.0, wj = gJ ? gJ[w] : 0.0, wo = gocc ? gocc[w] : 0.0;
  const int et = s.m * a.nb + s.nn;  // transposed element
  double2 c = make_double2(0.0, 0.0);
  if (wp != 0.0) {
    const double2 d = proj_e(F, a, a.dip, s.k, et);
    c.x += wp * d.x;
    c.y -= wp * d.y;
  }
  if (wj != 0.0) {
    const double2 v = proj_e(F, a, a.vel, s.k, et);
    c.x += wj * v.x;
    c.y -= wj * v.y;
  }
  if (s.nn == s.m && s.nn == a.nv) c.x += wo;
  return make_double2(c.x / a.nk, c.y / a.nk);
}

__global__ void __launch_bounds__(AT) adj_init_kernel(AdjArgs a, const double2* rho_in, double2* rho, double2* abar,
                                                      const double* gP, const double* gJ, const double* gocc,
                                                      int64_t gstride) {
  const Slot s = slot_of(a);
  if (!s.active) return;
  const double occ = (s.nn == s.m && s.nn < a.nv) ? 1.0 : 0.0;
  rho[s.g] = rho_in ? rho_in[s.g] : make_double2(occ, 0.0);
  abar[s.g] = obs_cotangent(a, s, a.fields[s.b], gP, gJ, gocc, gstride, a.nsteps);
}

// x[b][k P + p] = (y - rho_eq)[pair p of k], column-major [n] x [B].
__global__ void __launch_bounds__(AT) adj_gather_kernel(AdjArgs a, const double2* __restrict__ y, double2* x) {
  const Slot s = slot_of(a);
  if (!s.active) return;
  const int p = pair_of(a, s.nn, s.m);
  if (p < 0) return;
  const double2 v = y[s.g];
  x[(size_t)s.b * a.n + (size_t)s.k * a.npair + p] =
      make_double2(v.x - ((s.nn == s.m && s.nn < a.nv) ? 1.0 : 0.0), v.y);
}

// The block's rows of a factor product, low rank: out[lk P + p] = sum_j
// M[(k P + p) ldm + j] vec[b r + j] for the block's k points k = k0 + lk and
// pairs p (kpb P <= AT rows), over all the block's threads.  tpr consecutive
// lanes (a power of two, within one wave) share a row, each summing every
// tpr-th column in order, eight columns' loads issued together; the lanes'
// sums are then combined by a butterfly, whose partners add the same two
// values, so every lane of the row holds the same sum.
__device__ inline void block_rows_dot(const AdjArgs& a, const double2* __restrict__ M, int64_t ldm,
                                      const double2* __restrict__ vec, int r, double2* out) {
  const int kpb = AT / (a.nb * a.nb), P = a.npair, rows = kpb * P, nt = blockDim.x;
  int tpr = 1;
  while (2 * tpr * rows <= nt && 2 * tpr <= 64) tpr *= 2;
  const int t = threadIdx.x, row = t / tpr, part = t % tpr;
  const int k = blockIdx.x * kpb + row / P;
  double sr = 0.0, si = 0.0;
  if (row < rows && k < a.nk) {
    const double2* mr = M + ((size_t)k * P + row % P) * ldm;
    const double2* v = vec + (size_t)blockIdx.y * r;
    constexpr int U = 8;
    for (int j0 = part; j0 < r; j0 += U * tpr) {
      double2 m[U], x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // past the last column: load column j0 (in range) and use zero
        const int j = j0 + u * tpr, jc = j < r ? j : j0;
        m[u] = mr[jc];
        x[u] = v[jc];
        if (j >= r) m[u] = make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        sr += m[u].x * x[u].x - m[u].y * x[u].y;
        si += m[u].x * x[u].y + m[u].y * x[u].x;
      }
    }
  }
  for (int off = 1; off < tpr; off <<= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  if (part == 0 && row < rows) out[row] = make_double2(sr, si);
}

// Forward stage s of step `step` at the state y: f = -i [H, y]; RK4
// accumulation; the next stage's state (or rho_{n+1} after the fourth stage)
// into y_next and its gather into x_next (if not NULL).  Dense: S is K x.
// Low rank (M not NULL): the block forms its rows of S = M vec itself (M = S~,
// vec = z = V^H x) and stores them into S for the backward sweep.
__global__ void __launch_bounds__(ATW) adj_fwd_stage_kernel(AdjArgs a, int step, int st, const double2* rho_n,
                                                           const double2* y, double2* S, const double2* X,
                                                           const double2* M, int64_t ldm, const double2* vec, int r,
                                                           const double2* dy, double2* acc, double2* y_next,
                                                           double2* x_next) {
  __shared__ double2 sh_y[AT], sh_h[AT], sh_s[AT];
  const Slot s = slot_of(a);
  const int t = threadIdx.x, nb = a.nb, o = s.lk * nb * nb;
  // the slot's own inputs, read before the product so that their latency
  // overlaps it: the state, and H but for the product's own term (dense: all
  // of H; low rank: its pair, K_diag o x, the field term and the band energy,
  // added to the product's row below in the order of ham_element)
  const double2 zero = make_double2(0.0, 0.0);
  double2 yv = zero, rn = zero, ac = zero, dv = zero, hv = zero, kx = zero, de = zero;
  double ef = 0.0, eps = 0.0;
  int hp = -1;
  bool hcj = false;
  if (s.active) {
    yv = y[s.g];
    rn = rho_n[s.g];
    if (st > 0) ac = acc[s.g];
    if (dy) dv = dy[s.g];
    const tdg_field F = a.fields[s.b];
    ef = field_value(F, ((double)step + stage_offset(st)) * a.dt);
    de = proj_e(F, a, a.dip, s.k, s.e);
    if (!M) {
      hv = ham_element(a, S, X, s, ef, de);
    } else {
      hp = pair_of(a, s.nn, s.m);
      if (hp < 0 && a.block == TDG_BLOCK_EH && s.nn < a.nv && s.m >= a.nv) {
        hp = (s.m - a.nv) * a.nv + s.nn;
        hcj = true;
      }
      if (hp >= 0 && a.kdiag)
        kx = cmul(a.kdiag[(size_t)s.k * a.npair + hp], X[(size_t)s.b * a.n + (size_t)s.k * a.npair + hp]);
      if (s.nn == s.m) eps = a.eps[(size_t)s.k * a.nb + s.nn];
    }
  }
  if (M) {
    block_rows_dot(a, M, ldm, vec, r, sh_s);
    __syncthreads();
    const int kpb = AT / (nb * nb), P = a.npair, k = blockIdx.x * kpb + t / P;
    if (t < kpb * P && k < a.nk) S[(size_t)blockIdx.y * a.n + (size_t)k * P + t % P] = sh_s[t];
  }
  if (s.active) {
    sh_y[t] = yv;
    if (M) {
      double2 ds = zero;
      if (hp >= 0) {
        double2 v = sh_s[s.lk * a.npair + hp];
        if (a.kdiag) v = cadd(v, kx);
        ds = hcj ? cconj(v) : v;
      }
      hv = make_double2(ds.x - ef * de.x, ds.y - ef * de.y);
      if (s.nn == s.m) hv.x += eps;
    }
    sh_h[t] = hv;
  }
  __syncthreads();
  if (!s.active) return;
  double2 c = make_double2(0.0, 0.0);
  for (int l = 0; l < nb; ++l) {
    const double2 hr = cmul(sh_h[o + s.nn * nb + l], sh_y[o + l * nb + s.m]);
    const double2 rh = cmul(sh_y[o + s.nn * nb + l], sh_h[o + l * nb + s.m]);
    c.x += hr.x - rh.x;
    c.y += hr.y - rh.y;
  }
  double2 f = make_double2(c.y, -c.x);  // -i c
  if (dy) {
    // intraband term -E(t) D(y)
    f.x -= ef * dv.x;
    f.y -= ef * dv.y;
  }
  const double dt = a.dt;
  double2 next;
  if (st == 0) {
    acc[s.g] = f;
    next = make_double2(rn.x + 0.5 * dt * f.x, rn.y + 0.5 * dt * f.y);
  } else if (st == 1) {
    acc[s.g] = make_double2(ac.x + 2.0 * f.x, ac.y + 2.0 * f.y);
    next = make_double2(rn.x + 0.5 * dt * f.x, rn.y + 0.5 * dt * f.y);
  } else if (st == 2) {
    acc[s.g] = make_double2(ac.x + 2.0 * f.x, ac.y + 2.0 * f.y);
    next = make_double2(rn.x + dt * f.x, rn.y + dt * f.y);
  } else {
    const double w = dt / 6.0;
    next = make_double2(rn.x + w * (ac.x + f.x), rn.y + w * (ac.y + f.y));
  }
  y_next[s.g] = next;
  const int p = pair_of(a, s.nn, s.m);
  if (x_next && p >= 0)
    x_next[(size_t)s.b * a.n + (size_t)s.k * a.npair + p] =
        make_double2(next.x - ((s.nn == s.m && s.nn < a.nv) ? 1.0 : 0.0), next.y);
}

// Pullback, first half, for stage s: g = coef * abar + cnext * ybar_next;
// ydirect = i [H^H, g]; sbc = conj(gather(Sigbar)) with Sigbar = -i [y^H, g];
// part[s][b][k] = Re sum conj(g) i [e.d, y] over the k point's elements.
// Intraband term (dy = D(y) not NULL; da = D(abar), dyb = D(ybar_next)):
// ydirect += E D(g), part -= Re sum conj(g) D(y).
// The first half's inputs that nothing in the backward sweep writes while it
// runs (stage state, H, the field term): read ahead of any other work of the
// launch, so that their latency overlaps it.
struct BwdAIn {
  double ef;
  double2 de, yv, hv;
};
__device__ inline BwdAIn adj_bwd_a_inputs(const AdjArgs& a, int step, int st, const double2* y, const double2* S,
                                          const double2* X) {
  BwdAIn in;
  in.ef = 0.0;
  in.de = in.yv = in.hv = make_double2(0.0, 0.0);
  const Slot s = slot_of(a);
  if (s.active) {
    const tdg_field F = a.fields[s.b];
    in.ef = field_value(F, ((double)step + stage_offset(st)) * a.dt);
    in.de = proj_e(F, a, a.dip, s.k, s.e);
    in.yv = y[s.g];
    in.hv = ham_element(a, S, X, s, in.ef, in.de);
  }
  return in;
}

__device__ inline void adj_bwd_a(const AdjArgs& a, int st, const BwdAIn& in, const double2* abar,
                                  double coef, const double2* ybar_next, double cnext, const double2* dy,
                                  const double2* da, const double2* dyb, double2* ydirect, double2* sbc,
                                  double* part) {
  __shared__ double2 sh_y[AT], sh_h[AT], sh_g[AT], sh_d[AT], sh_sig[AT];
  __shared__ double sh_de[AT];
  const Slot s = slot_of(a);
  const int t = threadIdx.x, nb = a.nb, nb2 = nb * nb, o = s.lk * nb2;
  const double ef = in.ef;
  if (s.active) {
    const double2 de = in.de;
    const double2 ab = abar[s.g];
    double2 g = make_double2(coef * ab.x, coef * ab.y);
    if (ybar_next) {
      const double2 yb = ybar_next[s.g];
      g.x += cnext * yb.x;
      g.y += cnext * yb.y;
    }
    sh_y[t] = in.yv;
    sh_h[t] = in.hv;
    sh_g[t] = g;
    sh_d[t] = de;
  }
  __syncthreads();
  if (s.active) {
    double2 c1 = make_double2(0.0, 0.0), c2 = c1, c3 = c1;
    for (int l = 0; l < nb; ++l) {
      // (H^H)[n][l] g[l][m] - g[n][l] (H^H)[l][m],  (H^H)[i][j] = conj(H[j][i])
      const double2 a1 = cmul(cconj(sh_h[o + l * nb + s.nn]), sh_g[o + l * nb + s.m]);
      const double2 b1 = cmul(sh_g[o + s.nn * nb + l], cconj(sh_h[o + s.m * nb + l]));
      c1.x += a1.x - b1.x;
      c1.y += a1.y - b1.y;
      const double2 a2 = cmul(cconj(sh_y[o + l * nb + s.nn]), sh_g[o + l * nb + s.m]);
      const double2 b2 = cmul(sh_g[o + s.nn * nb + l], cconj(sh_y[o + s.m * nb + l]));
      c2.x += a2.x - b2.x;
      c2.y += a2.y - b2.y;
      const double2 a3 = cmul(sh_d[o + s.nn * nb + l], sh_y[o + l * nb + s.m]);
      const double2 b3 = cmul(sh_y[o + s.nn * nb + l], sh_d[o + l * nb + s.m]);
      c3.x += a3.x - b3.x;
      c3.y += a3.y - b3.y;
    }
    double2 yd = make_double2(-c1.y, c1.x);  // i c1
    sh_sig[t] = make_double2(c2.y, -c2.x);   // -i c2
    // Re(conj(g) * i c3) = g.x (-c3.y) + g.y c3.x
    const double2 g = sh_g[t];
    double dl = -g.x * c3.y + g.y * c3.x;
    if (dy) {
      const double2 d_a = da[s.g];
      double2 dg = make_double2(coef * d_a.x, coef * d_a.y);
      if (ybar_next) {
        const double2 d_y = dyb[s.g];
        dg.x += cnext * d_y.x;
        dg.y += cnext * d_y.y;
      }
      yd.x += ef * dg.x;
      yd.y += ef * dg.y;
      const double2 d = dy[s.g];
      dl -= g.x * d.x + g.y * d.y;
    }
    ydirect[s.g] = yd;
    sh_de[t] = dl;
  }
  __syncthreads();
  if (!s.active) return;
  const int p = pair_of(a, s.nn, s.m);
  if (p >= 0) {
    double2 sb = sh_sig[t];
    if (a.block == TDG_BLOCK_EH) {
      const double2 tr = sh_sig[o + s.m * nb + s.nn];
      sb = make_double2(sb.x + tr.x, sb.y - tr.y);
    }
    sbc[(size_t)s.b * a.n + (size_t)s.k * a.npair + p] = cconj(sb);
  }
  if (s.e == 0) {
    double v = 0.0;
    for (int i = 0; i < nb2; ++i) v += sh_de[o + i];
    part[((size_t)st * a.batch + s.b) * a.nk + s.k] = v;
  }
}

// Pullback, second half, for stage s: ybar = ydirect + scatter(conj(T + K_diag o sbc));
// acca accumulates dL/drho_n; after the first stage abar <- acca + ybar + observable cotangent.
// Dense: T = K^T conj(sbar) is given.  Low rank (M not NULL): the block forms
// its rows of T = M vec itself (M = V^H transposed, vec = S~^T conj(sbar)).
__device__ inline void adj_bwd_b(const AdjArgs& a, int step, int st, const double2* ydirect, const double2* T,
                                  const double2* M, int64_t ldm, const double2* vec, int r, const double2* sbc,
                                  double2* ybar, double2* acca, double2* abar, const double* gP, const double* gJ,
                                  const double* gocc, int64_t gstride) {
  __shared__ double2 sh_t[AT];
  if (M) {
    block_rows_dot(a, M, ldm, vec, r, sh_t);
    __syncthreads();
  }
  const Slot s = slot_of(a);
  if (!s.active) return;
  double2 yb = ydirect[s.g];
  const int p = pair_of(a, s.nn, s.m);
  if (p >= 0) {
    const size_t i = (size_t)s.b * a.n + (size_t)s.k * a.npair + p;
    double2 v = M ? sh_t[s.lk * a.npair + p] : T[i];
    if (a.kdiag) v = cadd(v, cmul(a.kdiag[(size_t)s.k * a.npair + p], sbc[i]));
    yb.x += v.x;
    yb.y -= v.y;
  }
  ybar[s.g] = yb;
  if (st == 3) {
    const double2 ab = abar[s.g];
    acca[s.g] = make_double2(ab.x + yb.x, ab.y + yb.y);
  } else if (st > 0) {
    const double2 ac = acca[s.g];
    acca[s.g] = make_double2(ac.x + yb.x, ac.y + yb.y);
  } else {
    const double2 ac = acca[s.g];
    const double2 oc = obs_cotangent(a, s, a.fields[s.b], gP, gJ, gocc, gstride, step);
    abar[s.g] = make_double2(ac.x + yb.x + oc.x, ac.y + yb.y + oc.y);
  }
}

__global__ void __launch_bounds__(AT) adj_bwd_a_kernel(AdjArgs a, int step, int st, const double2* y, const double2* S,
                                                       const double2* X, const double2* abar, double coef,
                                                       const double2* ybar_next, double cnext, const double2* dy,
                                                       const double2* da, const double2* dyb, double2* ydirect,
                                                       double2* sbc, double* part) {
  const BwdAIn in = adj_bwd_a_inputs(a, step, st, y, S, X);
  adj_bwd_a(a, st, in, abar, coef, ybar_next, cnext, dy, da, dyb, ydirect, sbc, part);
}

__global__ void __launch_bounds__(ATW) adj_bwd_b_kernel(AdjArgs a, int step, int st, const double2* ydirect,
                                                       const double2* T, const double2* M, int64_t ldm,
                                                       const double2* vec, int r, const double2* sbc, double2* ybar,
                                                       double2* acca, double2* abar, const double* gP,
                                                       const double* gJ, const double* gocc, int64_t gstride) {
  adj_bwd_b(a, step, st, ydirect, T, M, ldm, vec, r, sbc, ybar, acca, abar, gP, gJ, gocc, gstride);
}

// The second half of stage st's pullback, then the first half of the stage
// before it (no intraband term): stage st - 1 of the same step, or, after
// stage 0, stage 3 of step - 1 (its stage data stashed).  Both halves are
// local to a k point, and the first reads only the thread's own elements of
// ybar and abar, which the second has just written, so one launch does both.
// step_a, st_a, ybar_next, part: the first half's step, stage, ybar of the
// stage after it (NULL for stage 3) and dE partials.
__global__ void __launch_bounds__(ATW) adj_bwd_ba_kernel(AdjArgs a, int step, int st, const double2* M, int64_t ldm,
                                                        const double2* vec, int r, const double2* T,
                                                        const double2* sbc_in, double2* ybar, double2* acca,
                                                        double2* abar, const double* gP, const double* gJ,
                                                        const double* gocc, int64_t gstride, int step_a, int st_a,
                                                        const double2* y, const double2* S, const double2* X,
                                                        double coef, const double2* ybar_next, double cnext,
                                                        double2* ydirect, double2* sbc_out, double* part) {
  const BwdAIn in = adj_bwd_a_inputs(a, step_a, st_a, y, S, X);
  adj_bwd_b(a, step, st, ydirect, T, M, ldm, vec, r, sbc_in, ybar, acca, abar, gP, gJ, gocc, gstride);
  adj_bwd_a(a, st_a, in, abar, coef, ybar_next, cnext, nullptr, nullptr, nullptr, ydirect, sbc_out, part);
}

// dL/dE at the four stage times of each of a segment's steps start + i (sum
// over k in fixed order), and each stage's contribution to dL/d(e0, omega,
// tau, t0) into terms[i][b][stage][4].  Block (i, b), one wave per stage:
// each lane sums every 64th k in order (sixteen loads issued together), a
// butterfly combines the lanes.  part[i] holds step start + i's partials.
__global__ void __launch_bounds__(256) adj_de_kernel(AdjArgs a, int start, const double* part, double* dE,
                                                     double* terms) {
  const int i = blockIdx.x, b = blockIdx.y, t = threadIdx.x, st = t >> 6, lane = t & 63;
  const int step = start + i;
  const tdg_field F = a.fields[b];
  const double* ps = part + (((size_t)i * 4 + st) * a.batch + b) * a.nk;
  constexpr int U = 16;
  double v = 0.0;
  for (int k0 = lane; k0 < a.nk; k0 += 64 * U) {
    double q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // past the last k: load k0 (in range) and use zero
      const int k = k0 + 64 * u;
      q[u] = ps[k < a.nk ? k : k0];
      if (k >= a.nk) q[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v += q[u];
  }
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) {
    const double d = v;
    if (dE) dE[((size_t)b * a.nsteps + step) * 4 + st] = d;
    const double tt = ((double)step + stage_offset(st)) * a.dt;
    const double dd = tt - F.t0, g = exp(-dd * dd / (2.0 * F.tau * F.tau));
    const double c = cos(F.omega * tt), sn = sin(F.omega * tt);
    double* tm = terms + (((size_t)i * a.batch + b) * 4 + st) * 4;
    tm[0] = d * (g * c);
    tm[1] = d * (-F.e0 * g * tt * sn);
    tm[2] = d * (F.e0 * g * c * dd * dd / (F.tau * F.tau * F.tau));
    tm[3] = d * (F.e0 * g * c * dd / (F.tau * F.tau));
  }
}

// dfield[b] += the terms of a segment's count steps, the last step first and
// the stages in order within a step (the order of the backward sweep).  One
// thread per (instance, parameter).
__global__ void adj_dfield_kernel(AdjArgs a, int count, const double* terms, double* dfield) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)a.batch * 4) return;
  const int b = (int)(idx / 4), c = (int)(idx % 4);
  double acc = dfield[idx];
  for (int i = count - 1; i >= 0; --i)
    for (int st = 0; st < 4; ++st) acc += terms[(((size_t)i * a.batch + b) * 4 + st) * 4 + c];
  dfield[idx] = acc;
}

__global__ void fill_zero_kernel(double* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// out[j][i] = in[i][j] for in [rows][cols] row-major with row stride ld
// (32 x 32 tiles through LDS); out is [cols][rows].
__global__ void __launch_bounds__(256) transpose_kernel(const double2* __restrict__ in, int64_t rows, int64_t cols,
                                                        int64_t ld, double2* __restrict__ out) {
  __shared__ double2 tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int q = ty; q < 32; q += 8) {
    const int64_t r = r0 + q, c = c0 + tx;
    if (r < rows && c < cols) tile[q][tx] = in[r * ld + c];
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int64_t c = c0 + q, r = r0 + tx;
    if (r < rows && c < cols) out[c * rows + r] = tile[tx][q];
  }
}

// C[b][i] = sum_j A[i][j] B[b][j], i < m, for every instance b: A row-major
// [m][lda] complex128, B[b] at B + b k, C[b] at C + b m.  Block (g, b): R
// consecutive rows, the NT threads striding over the k columns, U columns'
// loads issued together (the products are latency bound: a few thousand
// columns); each row's sum is reduced in a fixed order (wave sums, then the
// waves in order).
template <int R, int NT>
__global__ void __launch_bounds__(NT) rowdot_kernel(const double2* __restrict__ A, int64_t lda, int64_t m, int64_t k,
                                                    const double2* __restrict__ B, double2* __restrict__ C) {
  constexpr int NW = NT / 64;
  const int64_t i0 = (int64_t)blockIdx.x * R;
  const int b = blockIdx.y, t = threadIdx.x;
  const double2* x = B + (size_t)b * k;
  double ar[R], ai[R];
#pragma unroll
  for (int r = 0; r < R; ++r) ar[r] = ai[r] = 0.0;
  constexpr int U = R == 1 ? 8 : 2;
  const double2 zero = make_double2(0.0, 0.0);
  for (int64_t j0 = t; j0 < k; j0 += NT * U) {
    double2 xv[U], av[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // past the last column or row: load an in-range element and use zero
      const int64_t j = j0 + (int64_t)u * NT, jc = j < k ? j : j0;
      xv[u] = x[jc];
      if (j >= k) xv[u] = zero;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t i = i0 + r < m ? i0 + r : i0;
        av[u][r] = A[i * lda + jc];
        if (i0 + r >= m) av[u][r] = zero;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        ar[r] += av[u][r].x * xv[u].x - av[u][r].y * xv[u].y;
        ai[r] += av[u][r].x * xv[u].y + av[u][r].y * xv[u].x;
      }
    }
  }
  __shared__ double red[NW][2 * R];
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    for (int off = 32; off > 0; off >>= 1) {
      ar[r] += __shfl_down(ar[r], off, 64);
      ai[r] += __shfl_down(ai[r], off, 64);
    }
    if (lane == 0) {
      red[wave][2 * r] = ar[r];
      red[wave][2 * r + 1] = ai[r];
    }
  }
  __syncthreads();
  if (t < R && i0 + t < m) {
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < NW; ++w) {
      sr += red[w][2 * t];
      si += red[w][2 * t + 1];
    }
    C[(size_t)b * m + i0 + t] = make_double2(sr, si);
  }
}

// out[i][j] += sum_{c < cols} a[c sa + i] b[c sb + j], i < mi, j < mj (complex
// products, not conjugated; out row-major with row stride ldo).  A block owns a
// 64 x 64 tile of out and the columns [z cs, (z + 1) cs) of split z =
// blockIdx.z; each thread owns 4 x 4 elements of the tile, with 16 of the c
// at a time in LDS, and sums each element over its columns in order.  One
// split adds into out; with several, split z stores its partial tile into
// part[z] and outer_sum_kernel adds the splits to out in order.
__global__ void __launch_bounds__(256) outer_acc_kernel(const double2* __restrict__ a, int64_t sa, int64_t mi,
                                                        const double2* __restrict__ b, int64_t sb, int64_t mj,
                                                        int64_t cols, int64_t cs, double2* __restrict__ out,
                                                        int64_t ldo, double2* __restrict__ part) {
  __shared__ double2 as[16][64], bs[16][64];
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  const int64_t c_begin = (int64_t)blockIdx.z * cs, c_end = min(cols, c_begin + cs);
  const int t = threadIdx.x, ti = t >> 4, tj = t & 15;
  const double2 zero = make_double2(0.0, 0.0);
  double2 acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = zero;
  for (int64_t c0 = c_begin; c0 < c_end; c0 += 16) {
    for (int q = t; q < 16 * 64; q += 256) {
      const int cc = q >> 6, e = q & 63;
      const int64_t c = c0 + cc;
      as[cc][e] = (c < c_end && i0 + e < mi) ? a[c * sa + i0 + e] : zero;
      bs[cc][e] = (c < c_end && j0 + e < mj) ? b[c * sb + j0 + e] : zero;
    }
    __syncthreads();
    for (int cc = 0; cc < 16; ++cc) {
      double2 x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = as[cc][ti + 16 * u];
        y[u] = bs[cc][tj + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc[u][v].x += x[u].x * y[v].x - x[u].y * y[v].y;
          acc[u][v].y += x[u].x * y[v].y + x[u].y * y[v].x;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + ti + 16 * u, j = j0 + tj + 16 * v;
      if (i < mi && j < mj) {
        if (gridDim.z == 1) {
          double2& o = out[i * ldo + j];
          o.x += acc[u][v].x;
          o.y += acc[u][v].y;
        } else {
          part[((size_t)blockIdx.z * mi + i) * mj + j] = acc[u][v];
        }
      }
    }
}

// out[i][j] += sum over splits z in order of part[z][i][j] (outer_acc_kernel's
// partial tiles), one thread per element.
__global__ void outer_sum_kernel(const double2* __restrict__ part, int splits, int64_t mi, int64_t mj, double2* out,
                                 int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mi * mj) return;
  const int64_t i = idx / mj, j = idx % mj;
  double2 o = out[i * ldo + j];
  for (int z = 0; z < splits; ++z) {
    const double2 v = part[(size_t)z * mi * mj + idx];
    o.x += v.x;
    o.y += v.y;
  }
  out[i * ldo + j] = o;
}

__global__ void conj_kernel(double2* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i].y = -p[i].y;
}

// Column splits of a factor-gradient product out[mi][mj] over cols columns:
// about 512 blocks of 64 x 64 tiles, each split at least 16 columns, at most
// 64 splits; 1 when the tiles alone fill the device.
int64_t outer_splits(int64_t mi, int64_t mj, int64_t cols) {
  const int64_t tiles = ((mi + 63) / 64) * ((mj + 63) / 64);
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>(64, 512 / tiles));
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, cols / 16));
  const int64_t cs = (cols + splits - 1) / splits;
  return (cols + cs - 1) / cs;
}

// Carves 256-byte-aligned pieces out of one workspace block.
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  }
};

}  // namespace

using namespace tdg;

extern "C" int tdg_propagate_adjoint(tdg_ctx ctx, const tdg_operator* op, const tdg_model* model,
                                     const tdg_field* fields, int32_t batch, double dt, const void* rho0,
                                     int32_t checkpoint_every, const tdg_obs_grad* gobs, tdg_grads* out) {
  if (!ctx) return TDG_E_INVAL;
  if (!op || !model || !fields || !gobs || !out) return fail(ctx, TDG_E_INVAL, "NULL argument");
  TDG_TRY(validate_model(ctx, model));
  if (op->dtype != TDG_C128) return fail(ctx, TDG_E_UNSUPPORTED, "the adjoint runs on TDG_C128 operators only");
  if (op->kind != TDG_OP_DENSE && op->kind != TDG_OP_LOWRANK) return fail(ctx, TDG_E_INVAL, "operator kind %d", op->kind);
  const bool lowrank = op->kind == TDG_OP_LOWRANK;
  const int npair = pairs_per_k(model, op->block);
  if (npair <= 0) return fail(ctx, TDG_E_INVAL, "unknown block %d", op->block);
  const int nk = model->nk1 * model->nk2, nb = model->nb, nb2 = nb * nb;
  const int64_t n = (int64_t)nk * npair;
  if (op->n != n) return fail(ctx, TDG_E_INVAL, "operator n = %lld, model needs %lld", (long long)op->n, (long long)n);
  if (batch < 1 || batch > 65535) return fail(ctx, TDG_E_INVAL, "batch = %d", batch);
  if (!(dt > 0.0)) return fail(ctx, TDG_E_INVAL, "dt must be positive");
  const int64_t rank = lowrank ? op->rank : 0;
  if (lowrank) {
    if (!op->kdiag || !op->us || !op->w || rank < 1 || rank > n) return fail(ctx, TDG_E_INVAL, "low-rank operator");
  } else {
    if (!op->K || op->ld < n) return fail(ctx, TDG_E_INVAL, "dense operator");
    if (out->dus || out->dw) return fail(ctx, TDG_E_INVAL, "factor gradients need a low-rank operator");
  }
  const double ns = fields[0].nsteps;
  for (int b = 0; b < batch; ++b) {
    const tdg_field& f = fields[b];
    if (!(f.tau > 0.0) || !std::isfinite(f.e0) || !std::isfinite(f.omega) || !std::isfinite(f.t0))
      return fail(ctx, TDG_E_INVAL, "field %d parameters", b);
    if (f.nsteps != ns) return fail(ctx, TDG_E_UNSUPPORTED, "the adjoint needs equal nsteps for every instance");
  }
  if (!(ns >= 1.0) || ns > 1e8 || ns != std::floor(ns)) return fail(ctx, TDG_E_INVAL, "nsteps");
  const int nsteps = (int)ns;
  if ((gobs->gP || gobs->gJ || gobs->gocc) && gobs->stride < nsteps + 1)
    return fail(ctx, TDG_E_INVAL, "observable cotangent stride < nsteps + 1");
  if (checkpoint_every < 1) return fail(ctx, TDG_E_INVAL, "checkpoint_every must be >= 1");
  if (model->links && (int64_t)nk * nb2 * batch > ((int64_t)1 << 38))
    return fail(ctx, TDG_E_UNSUPPORTED, "intraband term: nk * nb^2 * batch too large for one launch");
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));

  // ---- workspace ---------------------------------------------------------
  const size_t st_el = (size_t)batch * nk * nb2;
  const size_t st_b = st_el * sizeof(double2);
  const size_t xn_b = (size_t)n * batch * sizeof(double2);
  const size_t zr_b = (size_t)std::max<int64_t>(rank, 1) * batch * sizeof(double2);
  // Whole run (stash mode 2): when every step's segment data (segment state,
  // stage states, products, gathers, their cotangents and the factor-space
  // columns) fits in ADJ_STASH_BYTES, one segment spans the run, so the
  // checkpoint sweep, one of the two forward passes, is skipped.  If the
  // device cannot hold that workspace, the run falls back to checkpoint_every
  // segments.
  const int M0 = std::min(checkpoint_every, nsteps);
  const bool whole = ctx->adj_stash == 2 && M0 < nsteps &&
                     (double)nsteps * (4.0 * st_b + 12.0 * xn_b + (lowrank ? 8.0 * zr_b : 0.0) +
                                       32.0 * batch * nk + 128.0 * batch) <= ADJ_STASH_BYTES;
  const bool intra = model->links != nullptr;
  // workspace layout for segments of Ms steps
  struct Layout {
    int M, nck, per_step, cblocks;
    bool stash;
    size_t o_ck, o_seg, o_ys, o_out, o_acc, o_abar, o_ybar, o_yd, o_acca, o_s, o_x, o_sbc, o_t, o_z, o_uc, o_part,
        o_terms, o_df, o_f, o_ust, o_wt, o_kt, o_dy, o_da, o_dyb, o_fg, total;
  };
  auto layout = [&](int Ms) {
    Layout L;
    L.M = Ms;
    L.nck = (nsteps + Ms - 1) / Ms;
    // Stage stash: when a segment's stage states, products and gathers fit in
    // ADJ_STASH_BYTES, the segment's recompute keeps them for every step and
    // the backward steps read them; otherwise each backward step reruns its
    // forward step (one more forward pass).
    L.stash = ctx->adj_stash && (double)Ms * (3.0 * st_b + 8.0 * xn_b) <= ADJ_STASH_BYTES;
    L.per_step = L.stash ? Ms : 1;
    L.cblocks = (lowrank || L.stash ? Ms : 1) * 4;
    Carver cv;
    L.o_ck = cv.take(st_b * L.nck);
    L.o_seg = cv.take(st_b * Ms);
    L.o_ys = cv.take(st_b * 3 * L.per_step);
    L.o_out = cv.take(st_b);
    L.o_acc = cv.take(st_b);
    L.o_abar = cv.take(st_b);
    L.o_ybar = cv.take(st_b);
    L.o_yd = cv.take(st_b);
    L.o_acca = cv.take(st_b);
    L.o_s = cv.take(xn_b * 4 * L.per_step);
    L.o_x = cv.take(xn_b * L.cblocks);
    L.o_sbc = cv.take(xn_b * L.cblocks);
    L.o_t = cv.take(lowrank ? 0 : xn_b);
    L.o_z = cv.take(lowrank ? zr_b * L.cblocks : 0);
    L.o_uc = cv.take(lowrank ? zr_b * L.cblocks : 0);
    // dE partials of every step of a segment, and each step's dfield terms
    L.o_part = cv.take((size_t)Ms * 4 * batch * nk * sizeof(double));
    L.o_terms = cv.take((size_t)Ms * batch * 16 * sizeof(double));
    L.o_df = cv.take((size_t)batch * 4 * sizeof(double));
    L.o_f = cv.take((size_t)batch * sizeof(tdg_field));
    // transposed copies, so that every product is a row-major row product:
    // S^T ([rank][n]) and V^H transposed ([n][rank]) for low rank, K^T for dense
    L.o_ust = cv.take(lowrank ? (size_t)n * rank * sizeof(double2) : 0);
    L.o_wt = cv.take(lowrank ? (size_t)n * rank * sizeof(double2) : 0);
    L.o_kt = cv.take(lowrank ? 0 : (size_t)n * n * sizeof(double2));
    // intraband term: D of a stage state, of abar and of ybar
    L.o_dy = cv.take(intra ? st_b : 0);
    L.o_da = cv.take(intra ? st_b : 0);
    L.o_dyb = cv.take(intra ? st_b : 0);
    // partial tiles of the factor gradients when their columns are split
    int64_t fg = 0;
    if (lowrank && (out->dus || out->dw)) {
      const int64_t cols = (int64_t)Ms * 4 * batch;
      fg = std::max(outer_splits(n, rank, cols), outer_splits(rank, n, cols)) * n * rank;
    }
    L.o_fg = cv.take((fg > n * rank ? fg : 0) * sizeof(double2));
    L.total = cv.off;
    return L;
  };
  Layout L = layout(whole ? nsteps : M0);
  void* base = nullptr;
  int rc_ws = ws_reserve(ctx, WS_ADJ, L.total, &base);
  if (rc_ws == TDG_E_NOMEM && whole) {
    (void)hipGetLastError();  // the failed allocation's error is not this call's
    L = layout(M0);
    rc_ws = ws_reserve(ctx, WS_ADJ, L.total, &base);
  }
  if (rc_ws != TDG_OK) return rc_ws;
  const int M = L.M, nck = L.nck;
  const bool stash = L.stash;
  ctx->last_variant = std::string("adjoint: ") +
                      (nck == 1 ? std::string("one segment")
                                : std::to_string(nck) + " segments of " + std::to_string(M) + " steps") +
                      (stash ? ", stage data stashed" : ", forward steps recomputed");
  char* wb = (char*)base;
  auto P2 = [&](size_t o) { return (double2*)(wb + o); };
  double2 *CK = P2(L.o_ck), *SEG = P2(L.o_seg), *YS = P2(L.o_ys), *OUT = P2(L.o_out), *ACC = P2(L.o_acc),
          *ABAR = P2(L.o_abar), *YBAR = P2(L.o_ybar), *YD = P2(L.o_yd), *ACCA = P2(L.o_acca), *SS = P2(L.o_s),
          *XS = P2(L.o_x), *SBC = P2(L.o_sbc), *TT = lowrank ? nullptr : P2(L.o_t), *ZS = P2(L.o_z), *UC = P2(L.o_uc);
  double2 *DY = intra ? P2(L.o_dy) : nullptr, *DA = intra ? P2(L.o_da) : nullptr,
          *DYB = intra ? P2(L.o_dyb) : nullptr;
  double2* UST = lowrank ? P2(L.o_ust) : nullptr;
  double2* WT = lowrank ? P2(L.o_wt) : nullptr;
  double2* KT = lowrank ? nullptr : P2(L.o_kt);
  // dE partials of a segment's steps (reduced once per segment) and their
  // dfield terms; the step's index within its segment is set per segment
  double* part_base = (double*)(wb + L.o_part);
  double* terms = (double*)(wb + L.o_terms);
  int seg_start = 0;
  auto partof = [&](int step) { return part_base + (size_t)(step - seg_start) * 4 * batch * nk; };
  double* dfacc = (double*)(wb + L.o_df);
  tdg_field* dfields = (tdg_field*)(wb + L.o_f);
  TDG_TRY(args_upload(ctx, dfields, fields, sizeof(tdg_field) * batch));

  AdjArgs a;
  a.nk = nk;
  a.nb = nb;
  a.nv = model->nv;
  a.npair = npair;
  a.block = op->block;
  a.batch = batch;
  a.nsteps = nsteps;
  a.n = n;
  a.dt = dt;
  a.eps = model->eps;
  a.dip = (const double2*)model->dip;
  a.vel = (const double2*)model->vel;
  a.fields = dfields;
  a.kdiag = lowrank ? (const double2*)op->kdiag : nullptr;

  // C[b] = A B[b] for every instance (A row-major [m_][lda], B[b] of k_
  // values, C[b] of m_): one fixed-order row product per row (four rows per
  // block when there are many rows; one row over 512 threads otherwise, so
  // that a row of a few thousand columns takes one batch of loads)
  auto prod = [&](const double2* A, int64_t lda, int64_t m_, int64_t k_, const double2* B, double2* C) -> int {
    if (m_ >= 1024)
      hipLaunchKernelGGL((rowdot_kernel<4, 256>), dim3((unsigned)((m_ + 3) / 4), (unsigned)batch), dim3(256), 0,
                         ctx->stream, A, lda, m_, k_, B, C);
    else
      hipLaunchKernelGGL((rowdot_kernel<1, 512>), dim3((unsigned)m_, (unsigned)batch), dim3(512), 0, ctx->stream, A,
                         lda, m_, k_, B, C);
    return launch_check(ctx, "adjoint product");
  };
  const double2* Kd = (const double2*)op->K;
  const double2* USd = (const double2*)op->us;
  const double2* Wd = (const double2*)op->w;
  // S = K X (dense) or Z = W X (low rank: the forward stage kernel forms
  // S = US Z itself); K, W, US row-major
  auto apply_k = [&](const double2* X, double2* S, double2* Z) -> int {
    if (!lowrank) return prod(Kd, op->ld, n, n, X, S);
    return prod(Wd, n, rank, n, X, Z);
  };
  // T with K^H sbar = conj(T) (+ K_diag term in the kernel): T = K^T conj(sbar),
  // or Uc = US^T conj(sbar) = conj(US^H sbar) (low rank: the backward kernel
  // forms T = W^T Uc itself)
  auto apply_kh = [&](const double2* Sbc, double2* Uc) -> int {
    if (!lowrank) return prod(KT, n, n, n, Sbc, TT);
    return prod(UST, n, rank, n, Sbc, Uc);
  };
  auto transpose = [&](const double2* in, int64_t rows, int64_t cols, int64_t ld, double2* o) {
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)), dim3(256), 0,
                       ctx->stream, in, rows, cols, ld, o);
  };
  if (lowrank) {
    transpose(USd, n, rank, rank, UST);
    transpose(Wd, rank, n, n, WT);
  } else {
    transpose(Kd, n, n, op->ld, KT);
  }
  TDG_TRY(launch_check(ctx, "transpose launch"));

  const int kpb = AT / nb2;
  const dim3 grid((unsigned)((nk + kpb - 1) / kpb), (unsigned)batch);
  // threads of the kernels that form their rows of a factor product
  const int pt = lowrank ? ATW : AT;
  auto xblk = [&](int cb) { return XS + (size_t)cb * n * batch; };
  auto sbcblk = [&](int cb) { return SBC + (size_t)cb * n * batch; };
  auto zblk = [&](int cb) { return ZS + (size_t)cb * rank * batch; };
  auto ucblk = [&](int cb) { return UC + (size_t)cb * rank * batch; };
  // stage s of stash slot j (slot 0 without the stash)
  auto sst = [&](int s, int j) { return SS + ((size_t)j * 4 + s) * n * batch; };
  auto ys = [&](int s, int j) { return YS + ((size_t)j * 3 + s - 1) * st_el; };  // s = 1, 2, 3

  // D(v) of a state-shaped array (caller's instance order) into out
  auto covd = [&](const double2* v, double2* o) {
    covariant_derivative(ctx->stream, model, v, (int64_t)nk * nb2, nb2, 1, dfields, batch, o);
  };
  // One forward step from rho_in to rho_out, keeping X_s, Z_s of its stages
  // in the column block group j and y_s, S_s in stash slot js.  gathered:
  // X_0 of rho_in is already in block group j (the previous step's last stage
  // wrote it); x_out (or NULL): where the last stage gathers rho_out.
  auto run_step = [&](int step, const double2* rho_in, double2* rho_out, int j, int js, bool gathered,
                      double2* x_out) -> int {
    if (!gathered) hipLaunchKernelGGL(adj_gather_kernel, grid, dim3(AT), 0, ctx->stream, a, rho_in, xblk(j * 4));
    for (int s = 0; s < 4; ++s) {
      const double2* y = s == 0 ? rho_in : ys(s, js);
      TDG_TRY(apply_k(xblk(j * 4 + s), sst(s, js), lowrank ? zblk(j * 4 + s) : nullptr));
      if (intra) covd(y, DY);
      hipLaunchKernelGGL(adj_fwd_stage_kernel, grid, dim3(pt), 0, ctx->stream, a, step, s, rho_in, y, sst(s, js),
                         xblk(j * 4 + s), lowrank ? USd : nullptr, (int64_t)rank,
                         lowrank ? (const double2*)zblk(j * 4 + s) : nullptr, (int)rank, (const double2*)DY, ACC,
                         s < 3 ? ys(s + 1, js) : rho_out, s < 3 ? xblk(j * 4 + s + 1) : x_out);
    }
    return launch_check(ctx, "adjoint forward step");
  };

  // ---- forward sweep with checkpoints -------------------------------------
  hipLaunchKernelGGL(adj_init_kernel, grid, dim3(AT), 0, ctx->stream, a, (const double2*)rho0, CK, ABAR, gobs->gP,
                     gobs->gJ, gobs->gocc, gobs->stride);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(256), 0, ctx->stream, dfacc, (int64_t)batch * 4);
  if (lowrank && out->dus)
    hipLaunchKernelGGL(fill_zero_kernel, dim3(256), dim3(256), 0, ctx->stream, (double*)out->dus, n * rank * 2);
  if (lowrank && out->dw)
    hipLaunchKernelGGL(fill_zero_kernel, dim3(256), dim3(256), 0, ctx->stream, (double*)out->dw, n * rank * 2);
  TDG_TRY(launch_check(ctx, "adjoint init"));
  for (int c = 0; c + 1 < nck; ++c) {
    // steps c M .. (c + 1) M - 1, the last landing on checkpoint c + 1; the
    // states between alternate over SEG's first slot and OUT (both idle here);
    // each step gathers the next one's X_0 into block group 0
    const double2* rin = CK + (size_t)c * st_el;
    for (int i = 0; i < M; ++i) {
      double2* rout = (i == M - 1) ? CK + (size_t)(c + 1) * st_el : ((i & 1) ? OUT : SEG);
      const bool last = c + 2 == nck && i == M - 1;
      TDG_TRY(run_step(c * M + i, rin, rout, 0, 0, c > 0 || i > 0, last ? nullptr : xblk(0)));
      rin = rout;
    }
  }

  // ---- backward sweep ------------------------------------------------------
  for (int c = nck - 1; c >= 0; --c) {
    const int start = c * M, end = std::min(nsteps, start + M);
    // states rho_start .. rho_{end-1}: slot 0 is the checkpoint itself
    auto seg = [&](int i) { return i == 0 ? CK + (size_t)c * st_el : SEG + (size_t)i * st_el; };
    if (stash) {
      // every step of the segment once, each keeping its stages in slot i
      for (int i = 0; i < end - start; ++i) {
        const bool more = i + 1 < end - start;
        TDG_TRY(run_step(start + i, seg(i), more ? seg(i + 1) : OUT, i, i, i > 0, more ? xblk((i + 1) * 4) : nullptr));
      }
    } else {
      for (int i = 0; i + 1 < end - start; ++i)
        TDG_TRY(run_step(start + i, seg(i), seg(i + 1), 0, 0, false, nullptr));
    }
    // a3_done: stage 3's first half of `step` ran in the previous step's last launch
    bool a3_done = false;
    seg_start = start;
    for (int step = end - 1; step >= start; --step) {
      const int j = lowrank || stash ? step - start : 0;
      const int js = stash ? step - start : 0;
      if (!stash) TDG_TRY(run_step(step, seg(step - start), OUT, j, 0, false, nullptr));
      double* part = partof(step);
      // stage 0's second half also does step - 1's stage 3 first half when
      // that step's stage data is stashed
      const bool a3_next = stash && !intra && step > start;
      static const double coef[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
      static const double cnext[4] = {0.5, 0.5, 1.0, 0.0};
      if (intra) covd(ABAR, DA);
      for (int s = 3; s >= 0; --s) {
        const double2* y = s == 0 ? seg(step - start) : ys(s, js);
        const int cb = j * 4 + s;
        // without the intraband term, stage s's first half ran in stage
        // s + 1's last launch
        if ((s == 3 && !a3_done) || intra) {
          if (intra) {
            covd(y, DY);
            if (s < 3) covd(YBAR, DYB);
          }
          hipLaunchKernelGGL(adj_bwd_a_kernel, grid, dim3(AT), 0, ctx->stream, a, step, s, y, sst(s, js), xblk(cb),
                             ABAR, coef[s] * dt, s == 3 ? (const double2*)nullptr : YBAR, cnext[s] * dt,
                             (const double2*)DY, (const double2*)DA, (const double2*)DYB, YD, sbcblk(cb), part);
        }
        TDG_TRY(apply_kh(sbcblk(cb), lowrank ? ucblk(cb) : nullptr));
        const double2* Mt = lowrank ? (const double2*)WT : nullptr;
        const double2* vt = lowrank ? (const double2*)ucblk(cb) : nullptr;
        if (s > 0 && !intra)
          hipLaunchKernelGGL(adj_bwd_ba_kernel, grid, dim3(pt), 0, ctx->stream, a, step, s, Mt, (int64_t)rank, vt,
                             (int)rank, (const double2*)TT, (const double2*)sbcblk(cb), YBAR, ACCA, ABAR,
                             (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, (int64_t)0, step,
                             s - 1, s - 1 == 0 ? seg(step - start) : ys(s - 1, js), (const double2*)sst(s - 1, js),
                             (const double2*)xblk(cb - 1), coef[s - 1] * dt, (const double2*)YBAR, cnext[s - 1] * dt,
                             YD, sbcblk(cb - 1), part);
        else if (s == 0 && a3_next)
          hipLaunchKernelGGL(adj_bwd_ba_kernel, grid, dim3(pt), 0, ctx->stream, a, step, 0, Mt, (int64_t)rank, vt,
                             (int)rank, (const double2*)TT, (const double2*)sbcblk(cb), YBAR, ACCA, ABAR, gobs->gP,
                             gobs->gJ, gobs->gocc, gobs->stride, step - 1, 3, (const double2*)ys(3, js - 1),
                             (const double2*)sst(3, js - 1), (const double2*)xblk((j - 1) * 4 + 3), coef[3] * dt,
                             (const double2*)nullptr, cnext[3] * dt, YD, sbcblk((j - 1) * 4 + 3), partof(step - 1));
        else
          hipLaunchKernelGGL(adj_bwd_b_kernel, grid, dim3(pt), 0, ctx->stream, a, step, s, YD, TT, Mt, (int64_t)rank,
                             vt, (int)rank, sbcblk(cb), YBAR, ACCA, ABAR, gobs->gP, gobs->gJ, gobs->gocc,
                             gobs->stride);
      }
      TDG_TRY(launch_check(ctx, "adjoint backward step"));
      a3_done = a3_next;
    }
    // dE of the segment's steps and their dfield terms, added in sweep order
    hipLaunchKernelGGL(adj_de_kernel, dim3((unsigned)(end - start), (unsigned)batch), dim3(256), 0, ctx->stream, a,
                       start, (const double*)part_base, out->dE, terms);
    hipLaunchKernelGGL(adj_dfield_kernel, dim3((unsigned)((batch * 4 + 255) / 256)), dim3(256), 0, ctx->stream, a,
                       end - start, (const double*)terms, dfacc);
    TDG_TRY(launch_check(ctx, "adjoint dE launch"));
    if (lowrank && (out->dus || out->dw)) {
      // conj(dL/dS)[i][j] += sum_c Sbc_c[i] Z_c[j] and conj(dL/dV^H)[j][i] += sum_c Uc_c[j] X_c[i]
      // over the segment's stage columns c
      const int64_t cols = (int64_t)(end - start) * 4 * batch;
      double2* fgp = (double2*)(wb + L.o_fg);
      // out[mi][mj] += sum_c a[c][i] b[c][j], its columns split over blocks when
      // the tiles alone would leave the device idle
      auto outer = [&](const double2* av, int64_t mi, const double2* bv, int64_t mj, double2* o) {
        const int64_t splits = outer_splits(mi, mj, cols);
        const int64_t cs = (cols + splits - 1) / splits;
        hipLaunchKernelGGL(outer_acc_kernel, dim3((unsigned)((mj + 63) / 64), (unsigned)((mi + 63) / 64), (unsigned)splits),
                           dim3(256), 0, ctx->stream, av, mi, mi, bv, mj, mj, cols, cs, o, mj, fgp);
        if (splits > 1)
          hipLaunchKernelGGL(outer_sum_kernel, dim3((unsigned)((mi * mj + 255) / 256)), dim3(256), 0, ctx->stream,
                             (const double2*)fgp, (int)splits, mi, mj, o, mj);
      };
      if (out->dus) outer((const double2*)SBC, n, (const double2*)ZS, rank, (double2*)out->dus);
      if (out->dw) outer((const double2*)UC, rank, (const double2*)XS, n, (double2*)out->dw);
      TDG_TRY(launch_check(ctx, "factor gradient launch"));
    }
  }

  if (lowrank && out->dus)
    hipLaunchKernelGGL(conj_kernel, dim3(256), dim3(256), 0, ctx->stream, (double2*)out->dus, n * rank);
  if (lowrank && out->dw)
    hipLaunchKernelGGL(conj_kernel, dim3(256), dim3(256), 0, ctx->stream, (double2*)out->dw, n * rank);
  if (out->drho0)
    TDG_TRY(hip_check(ctx, hipMemcpyAsync(out->drho0, ABAR, st_b, hipMemcpyDeviceToDevice, ctx->stream), "drho0 copy"));
  if (out->dfield)
    TDG_TRY(hip_check(ctx, hipMemcpyAsync(out->dfield, dfacc, (size_t)batch * 4 * sizeof(double),
                                          hipMemcpyDeviceToDevice, ctx->stream),
                      "dfield copy"));
  TDG_TRY(launch_check(ctx, "adjoint finish"));
  return hip_check(ctx, hipStreamSynchronize(ctx->stream), "adjoint sync");
}
