// One element of the covariant central difference of the intraband field term
// (paper Eq. tdagw with r in the smooth gauge of Appendix A.1), shared by the
// standalone kernel and the per-k stage kernels' epilogue:
//
//   T_a(k)_{nm} = [ L_a(k) y(k + b_a) L_a(k)^H - L_a(k - b_a)^H y(k - b_a) L_a(k - b_a) ]_{nm}
//
// for one axis a.  The links are block diagonal (valence and conduction
// subspaces), so the sums run over the blocks of row band n and column band m
// only.  yf(i, j) = y(k + b_a)[i][j], yb(i, j) = y(k - b_a)[i][j],
// lf(i, j) = L_a(k)[i][j], lb(i, j) = L_a(k - b_a)[i][j].
#pragma once

#include <hip/hip_runtime.h>

namespace tdg {

__device__ inline double2 cov_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ inline double2 cov_mulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

template <class YF, class YB, class LF, class LB>
__device__ inline double2 covariant_axis_element(int n, int m, int nb, int nv, YF yf, YB yb, LF lf, LB lb) {
  const int on = n < nv ? 0 : nv, sn = n < nv ? nv : nb - nv;
  const int om = m < nv ? 0 : nv, sm = m < nv ? nv : nb - nv;
  double2 t = make_double2(0.0, 0.0);
  for (int i = on; i < on + sn; ++i) {
    // forward: L[n][i] sum_j y_f[i][j] conj(L[m][j]);  backward: conj(Lb[i][n]) sum_j y_b[i][j] Lb[j][m]
    double2 sf = make_double2(0.0, 0.0), sbk = make_double2(0.0, 0.0);
    for (int jj = om; jj < om + sm; ++jj) {
      const double2 pf = cov_mulc(lf(m, jj), yf(i, jj));
      const double2 pb = cov_mul(yb(i, jj), lb(jj, m));
      sf.x += pf.x;
      sf.y += pf.y;
      sbk.x += pb.x;
      sbk.y += pb.y;
    }
    const double2 f = cov_mul(lf(n, i), sf);
    const double2 g = cov_mulc(lb(i, n), sbk);
    t.x += f.x - g.x;
    t.y += f.y - g.y;
  }
  return t;
}

// Grid neighbours of k = i1 nk2 + i2 along axis a (periodic): k + b_a, k - b_a.
__device__ inline void covariant_neighbours(int k, int a, int nk1, int nk2, int& kf, int& kb) {
  const int i1 = k / nk2, i2 = k - i1 * nk2;
  kf = a == 0 ? ((i1 + 1) % nk1) * nk2 + i2 : i1 * nk2 + (i2 + 1) % nk2;
  kb = a == 0 ? ((i1 + nk1 - 1) % nk1) * nk2 + i2 : i1 * nk2 + (i2 + nk2 - 1) % nk2;
}

}  // namespace tdg
