// Complex FP32 GEMM on the matrix cores for the batched contraction
// (many field instances at once turn dSigma = K drho, paper Eq. sigma-from-k,
// and the two products of Eq. svd_acc into matrix products).
//
//   Y[s][i][b] = sum_{c in slice s} A[i][c] * X[c][b]      (complex)
//
// A is row-major complex [M][lda]; X is complex [Kc][ldx], optionally the sum
// of several slices (the split-K partials of a previous product); b runs over
// the first ncols instances.  The complex product is done as one real product
// on v_mfma_f32_32x32x2f32: A viewed as real [M][2Kc] (re, im interleaved)
// times the real expansion
//     Xr[2c][b] = Re x,  Xr[2c+1][b] = -Im x,  Xr[2c][64+b] = Im x,  Xr[2c+1][64+b] = Re x
// so output columns 0..63 are Re y and 64..127 are Im y of 64 instances; the
// expansion is formed while X is staged into LDS, never stored.
//
// Tiles: a block of 256 threads (4 waves) owns 64 rows x 64 instances and
// walks its K slice 16 complex columns at a time through LDS; wave w computes
// rows 32*(w/2) .. +31 and real columns 64*(w%2) .. +63 as two 32x32 MFMA
// accumulators.  MFMA operand layout (checked on the device): lane l holds
// A[l%32][l/32] and B[l/32][l%32]; accumulator register r of lane l holds
// D[8*(r/4) + 4*(l/32) + r%4][l%32].
#include <algorithm>

#include "internal.h"

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 64;    // rows per block
constexpr int BKC = 16;   // complex K columns per LDS stage
constexpr int BNI = 64;   // instances per block
constexpr int APAD = 1;   // LDS padding (conflict-free column reads of A)

struct GemmArgs {
  const float2* A;
  int64_t lda;
  int M, Kc;
  const float2* X;
  int64_t ldx;
  int x_slices;
  int64_t x_slice_stride;
  float2* Y;
  int64_t ldy;
  int64_t y_slice_stride;
  int ncols;
  int kslice;
};

__global__ void __launch_bounds__(256) cgemm_f32_mfma(GemmArgs g) {
  __shared__ float As[BM][2 * BKC + APAD];
  __shared__ float Bs[2 * BKC][2 * BNI];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.x * BM, b0 = blockIdx.y * BNI, s = blockIdx.z;
  const int kc_begin = s * g.kslice;
  const int kc_end = min(g.Kc, kc_begin + g.kslice);
  const int wr = (w >> 1) * 32, wc = (w & 1) * 64;
  floatx16 acc0, acc1;
  for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0.f;

  // A loader: row t/4, complex columns 4*(t%4) .. +3;  X loader: complex row
  // t/16, instances 4*(t%16) .. +3
  const int arow = t >> 2, acol = (t & 3) * 4;
  const int xrow = t >> 4, xcol = (t & 15) * 4;
  const int gi = m0 + arow;
  for (int kc0 = kc_begin; kc0 < kc_end; kc0 += BKC) {
    float2 av[4], xv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kc = kc0 + acol + q;
      av[q] = (gi < g.M && kc < kc_end) ? g.A[(int64_t)gi * g.lda + kc] : make_float2(0.f, 0.f);
    }
    const int kx = kc0 + xrow;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + xcol + q;
      float2 v = make_float2(0.f, 0.f);
      if (kx < kc_end && b < g.ncols)
        for (int sl = 0; sl < g.x_slices; ++sl) {
          const float2 u = g.X[sl * g.x_slice_stride + (int64_t)kx * g.ldx + b];
          v.x += u.x;
          v.y += u.y;
        }
      xv[q] = v;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[arow][2 * (acol + q)] = av[q].x;
      As[arow][2 * (acol + q) + 1] = av[q].y;
      Bs[2 * xrow][xcol + q] = xv[q].x;
      Bs[2 * xrow + 1][xcol + q] = -xv[q].y;
      Bs[2 * xrow][BNI + xcol + q] = xv[q].y;
      Bs[2 * xrow + 1][BNI + xcol + q] = xv[q].x;
    }
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < 2 * BKC; k2 += 2) {
      const float a = As[wr + (lane & 31)][k2 + (lane >> 5)];
      const float x0 = Bs[k2 + (lane >> 5)][wc + (lane & 31)];
      const float x1 = Bs[k2 + (lane >> 5)][wc + 32 + (lane & 31)];
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, x0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, x1, acc1, 0, 0, 0);
    }
    __syncthreads();
  }

  // real column c = wc + 32*tile + (lane%32): instance c % 64, part c / 64
  float* Yf = reinterpret_cast<float*>(g.Y + s * g.y_slice_stride);
  const int part = wc >> 6;  // 0: real parts, 1: imaginary parts
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int row = m0 + wr + i;
    if (row >= g.M) continue;
    const int b_0 = b0 + (lane & 31), b_1 = b0 + 32 + (lane & 31);
    if (b_0 < g.ncols) Yf[2 * ((int64_t)row * g.ldy + b_0) + part] = acc0[r];
    if (b_1 < g.ncols) Yf[2 * ((int64_t)row * g.ldy + b_1) + part] = acc1[r];
  }
}

// out[i] = sum_s in[s * stride + i] for i < count (complex), fixed order.
__global__ void __launch_bounds__(256) sum_slices_kernel(const float2* __restrict__ in, int slices, int64_t stride,
                                                        int64_t count, float2* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    float2 v = make_float2(0.f, 0.f);
    for (int sl = 0; sl < slices; ++sl) {
      const float2 u = in[sl * stride + i];
      v.x += u.x;
      v.y += u.y;
    }
    out[i] = v;
  }
}

}  // namespace

namespace tdg {

void sum_slices_c64(hipStream_t stream, const void* in, int slices, int64_t stride, int64_t count, void* out) {
  const int64_t blocks = std::min<int64_t>(4096, (count + 255) / 256);
  hipLaunchKernelGGL(sum_slices_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, stream,
                     (const float2*)in, slices, stride, count, (float2*)out);
}

int cgemm_f32_kslices(int kc) { return (kc + BKC - 1) / BKC; }

// Launch Y[s] = A * sum(X slices) over split-K slices of `kslice` complex
// columns (a multiple of 16; the number of slices is ceil(Kc / kslice)).
void cgemm_f32(hipStream_t stream, const void* A, int64_t lda, int M, int Kc, const void* X, int64_t ldx,
               int x_slices, int64_t x_slice_stride, void* Y, int64_t ldy, int64_t y_slice_stride, int ncols,
               int kslice) {
  GemmArgs g;
  g.A = (const float2*)A;
  g.lda = lda;
  g.M = M;
  g.Kc = Kc;
  g.X = (const float2*)X;
  g.ldx = ldx;
  g.x_slices = x_slices;
  g.x_slice_stride = x_slice_stride;
  g.Y = (float2*)Y;
  g.ldy = ldy;
  g.y_slice_stride = y_slice_stride;
  g.ncols = ncols;
  g.kslice = kslice;
  const int splits = (Kc + kslice - 1) / kslice;
  const dim3 grid((M + BM - 1) / BM, (ncols + BNI - 1) / BNI, splits);
  hipLaunchKernelGGL(cgemm_f32_mfma, grid, dim3(256), 0, stream, g);
}

}  // namespace tdg
