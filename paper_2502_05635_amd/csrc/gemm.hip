// Complex FP32 GEMM on the matrix cores for the batched contraction
// (many field instances at once turn dSigma = K drho, paper Eq. sigma-from-k,
// and the two products of Eq. svd_acc into matrix products).
//
//   Y[s][i][b] = sum_{c in slice s} A[i][c] * X[c][b]      (complex)
//
// A is row-major complex [M][lda]; X is complex [Kc][ldx]; b runs over the
// first ncols instances.  The complex product is done as one real product
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

#include "bf16x2.h"
#include "internal.h"
#include "xcd.h"

namespace {

using tdg::bf2f;
using tdg::f2bf;
using tdg::xb_imag;
using tdg::xb_index;
using tdg::xb_word;

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
  float2* Y;
  int64_t ldy;
  int64_t y_slice_stride;
  int ncols;
  int kslice;
};

// Tile loads only issue loads into zero-initialised registers; masking and
// recombination happen when the tile is written to LDS.  A prefetched tile's
// loads are then not waited for before the current tile's products (a value
// combined right after its load forces the wait there).

// Instances b .. b + 3 of complex row kx of X (raw; zero where out of range).
__device__ inline void x_load(const GemmArgs& g, int kx, int kc_end, int b, float4& x01, float4& x23) {
  x01 = make_float4(0.f, 0.f, 0.f, 0.f);
  x23 = x01;
  if (kx < kc_end && b < g.ncols) {
    const float2* src = g.X + (int64_t)kx * g.ldx + b;
    x01 = *reinterpret_cast<const float4*>(src);
    if (b + 2 < g.ncols) x23 = *reinterpret_cast<const float4*>(src + 2);
  }
}
// The four instances of a raw X load, those at or beyond ncols zeroed.
__device__ inline void x_mask(const GemmArgs& g, int b, float4 x01, float4 x23, float2 (&xv)[4]) {
  xv[0] = make_float2(x01.x, x01.y);
  xv[1] = (b + 1 < g.ncols) ? make_float2(x01.z, x01.w) : make_float2(0.f, 0.f);
  xv[2] = (b + 2 < g.ncols) ? make_float2(x23.x, x23.y) : make_float2(0.f, 0.f);
  xv[3] = (b + 3 < g.ncols) ? make_float2(x23.z, x23.w) : make_float2(0.f, 0.f);
}
// Complex columns kc, kc + 1 of row gi of A as one 16-byte load, or the last
// column alone when kc + 1 is past the slice (raw; zero out of range).
__device__ inline void a_load2(const GemmArgs& g, int gi, int kc, int kc_end, float4& v, float2& tail) {
  // two independent predicated loads (nested branches made the compiler wait
  // for one load before issuing the next)
  v = make_float4(0.f, 0.f, 0.f, 0.f);
  tail = make_float2(0.f, 0.f);
  const float2* src = g.A + (int64_t)gi * g.lda + kc;
  if (gi < g.M && kc + 1 < kc_end) v = *reinterpret_cast<const float4*>(src);
  if (gi < g.M && kc + 1 == kc_end) tail = *src;
}
__device__ inline void a_pair(int kc, int kc_end, float4 v, float2 tail, float2& lo, float2& hi) {
  if (kc + 1 < kc_end) {
    lo = make_float2(v.x, v.y);
    hi = make_float2(v.z, v.w);
  } else {
    lo = tail;
    hi = make_float2(0.f, 0.f);
  }
}

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
    float4 x01, x23;
    x_load(g, kc0 + xrow, kc_end, b0 + xcol, x01, x23);
    x_mask(g, b0 + xcol, x01, x23, xv);
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
    // the stage's fragments first, then its products: LDS latency overlaps the MFMAs
    float fa[BKC], fx0[BKC], fx1[BKC];
#pragma unroll
    for (int q = 0; q < BKC; ++q) {
      fa[q] = As[wr + (lane & 31)][2 * q + (lane >> 5)];
      fx0[q] = Bs[2 * q + (lane >> 5)][wc + (lane & 31)];
      fx1[q] = Bs[2 * q + (lane >> 5)][wc + 32 + (lane & 31)];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the products
#pragma unroll
    for (int q = 0; q < BKC; ++q) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[q], fx0[q], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[q], fx1[q], acc1, 0, 0, 0);
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

// FP32 tiling 2: 128 rows x 64 instances per block; wave w owns rows
// 64*(w/2) .. +63 and real columns 64*(w%2) .. +63 as 2 x 2 MFMA accumulators,
// so each fragment read from LDS feeds two products.  The next K tile is
// loaded into registers while the current one is multiplied (one LDS buffer,
// two barriers per tile).  AVEC: A rows are 16-byte aligned (lda even), so A
// is read two complex numbers per load; X rows are always read that way (the
// host keeps ldx even).
constexpr int BM2 = 128;

template <bool AVEC>
__global__ void __launch_bounds__(256) cgemm_f32_mfma_128(GemmArgs g) {
  __shared__ float As[BM2][2 * BKC + APAD];
  __shared__ float Bs[2 * BKC][2 * BNI];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.x * BM2, b0 = blockIdx.y * BNI, s = blockIdx.z;
  const int kc_begin = s * g.kslice;
  const int kc_end = min(g.Kc, kc_begin + g.kslice);
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  floatx16 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // A loader: rows t/2 and t/2 + 128/2 ... : thread t covers row t/2, complex
  // columns 8*(t%2) .. +7 (4 pairs);  X loader: row t/16, instances 4*(t%16) .. +3
  const int arow = t >> 1, acol = (t & 1) * 8;
  const int xrow = t >> 4, xcol = (t & 15) * 4;
  const int gi = m0 + arow;
  // raw loads of the tile in flight (see a_load2 / x_load) and its first column
  float4 ar[4], xr01, xr23;
  float2 at[4], av[8], xv[4];
  int kc_tile = kc_begin;

  auto load_tile = [&](int kc0) {
    kc_tile = kc0;
    if (AVEC) {
#pragma unroll
      for (int q = 0; q < 4; ++q) a_load2(g, gi, kc0 + acol + 2 * q, kc_end, ar[q], at[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kc = kc0 + acol + q;
        av[q] = (gi < g.M && kc < kc_end) ? g.A[(int64_t)gi * g.lda + kc] : make_float2(0.f, 0.f);
      }
    }
    x_load(g, kc0 + xrow, kc_end, b0 + xcol, xr01, xr23);
  };
  auto store_tile = [&]() {
    if (AVEC) {
#pragma unroll
      for (int q = 0; q < 4; ++q) a_pair(kc_tile + acol + 2 * q, kc_end, ar[q], at[q], av[2 * q], av[2 * q + 1]);
    }
    x_mask(g, b0 + xcol, xr01, xr23, xv);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      As[arow][2 * (acol + q)] = av[q].x;
      As[arow][2 * (acol + q) + 1] = av[q].y;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Bs[2 * xrow][xcol + q] = xv[q].x;
      Bs[2 * xrow + 1][xcol + q] = -xv[q].y;
      Bs[2 * xrow][BNI + xcol + q] = xv[q].y;
      Bs[2 * xrow + 1][BNI + xcol + q] = xv[q].x;
    }
  };

  if (kc_begin < kc_end) {
    load_tile(kc_begin);
    store_tile();
  }
  __syncthreads();
  for (int kc0 = kc_begin; kc0 < kc_end; kc0 += BKC) {
    const bool more = kc0 + BKC < kc_end;
    if (more) load_tile(kc0 + BKC);
    // fragments of half a stage first, then its products (LDS latency overlaps the MFMAs)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      constexpr int HQ = BKC / 2;
      float fa0[HQ], fa1[HQ], fx0[HQ], fx1[HQ];
#pragma unroll
      for (int q = 0; q < HQ; ++q) {
        const int k2 = 2 * (h * HQ + q);
        fa0[q] = As[wr + (lane & 31)][k2 + (lane >> 5)];
        fa1[q] = As[wr + 32 + (lane & 31)][k2 + (lane >> 5)];
        fx0[q] = Bs[k2 + (lane >> 5)][wc + (lane & 31)];
        fx1[q] = Bs[k2 + (lane >> 5)][wc + 32 + (lane & 31)];
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the products
#pragma unroll
      for (int q = 0; q < HQ; ++q) {
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa0[q], fx0[q], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa0[q], fx1[q], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa1[q], fx0[q], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa1[q], fx1[q], acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
    if (more) store_tile();
    __syncthreads();
  }

  float* Yf = reinterpret_cast<float*>(g.Y + s * g.y_slice_stride);
  const int part = wc >> 6;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int row = m0 + wr + 32 * ti + i;
      if (row >= g.M) continue;
      const int b_0 = b0 + (lane & 31), b_1 = b0 + 32 + (lane & 31);
      if (b_0 < g.ncols) Yf[2 * ((int64_t)row * g.ldy + b_0) + part] = acc[ti][0][r];
      if (b_1 < g.ncols) Yf[2 * ((int64_t)row * g.ldy + b_1) + part] = acc[ti][1][r];
    }
}

// FP32 tiling 1: tiling 0's 64 rows x 64 instances and wave layout, with
// the next K tile loaded into registers while the current one is multiplied
// and two LDS buffers, so one barrier per tile separates the writers of one
// buffer from the readers of the other.  AVEC as above.
template <bool AVEC>
__global__ void __launch_bounds__(256) cgemm_f32_mfma_pf(GemmArgs g) {
  __shared__ float As[2][BM][2 * BKC + APAD];
  __shared__ float Bs[2][2 * BKC][2 * BNI];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.x * BM, b0 = blockIdx.y * BNI, s = blockIdx.z;
  const int kc_begin = s * g.kslice;
  const int kc_end = min(g.Kc, kc_begin + g.kslice);
  const int wr = (w >> 1) * 32, wc = (w & 1) * 64;
  floatx16 acc0, acc1;
  for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0.f;

  const int arow = t >> 2, acol = (t & 3) * 4;
  const int xrow = t >> 4, xcol = (t & 15) * 4;
  const int gi = m0 + arow;
  // raw loads of the tile in flight (see a_load2 / x_load) and its first column
  float4 ar[2], xr01, xr23;
  float2 at[2], av[4], xv[4];
  int kc_tile = kc_begin;

  auto load_tile = [&](int kc0) {
    kc_tile = kc0;
    if (AVEC) {
#pragma unroll
      for (int q = 0; q < 2; ++q) a_load2(g, gi, kc0 + acol + 2 * q, kc_end, ar[q], at[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kc = kc0 + acol + q;
        av[q] = (gi < g.M && kc < kc_end) ? g.A[(int64_t)gi * g.lda + kc] : make_float2(0.f, 0.f);
      }
    }
    x_load(g, kc0 + xrow, kc_end, b0 + xcol, xr01, xr23);
  };
  auto store_tile = [&](int buf) {
    if (AVEC) {
#pragma unroll
      for (int q = 0; q < 2; ++q) a_pair(kc_tile + acol + 2 * q, kc_end, ar[q], at[q], av[2 * q], av[2 * q + 1]);
    }
    x_mask(g, b0 + xcol, xr01, xr23, xv);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[buf][arow][2 * (acol + q)] = av[q].x;
      As[buf][arow][2 * (acol + q) + 1] = av[q].y;
      Bs[buf][2 * xrow][xcol + q] = xv[q].x;
      Bs[buf][2 * xrow + 1][xcol + q] = -xv[q].y;
      Bs[buf][2 * xrow][BNI + xcol + q] = xv[q].y;
      Bs[buf][2 * xrow + 1][BNI + xcol + q] = xv[q].x;
    }
  };

  if (kc_begin < kc_end) {
    load_tile(kc_begin);
    store_tile(0);
  }
  __syncthreads();
  int buf = 0;
  for (int kc0 = kc_begin; kc0 < kc_end; kc0 += BKC) {
    const bool more = kc0 + BKC < kc_end;
    if (more) load_tile(kc0 + BKC);
    // the stage's fragments first, then its products (LDS latency overlaps the MFMAs)
    float fa[BKC], fx0[BKC], fx1[BKC];
#pragma unroll
    for (int q = 0; q < BKC; ++q) {
      fa[q] = As[buf][wr + (lane & 31)][2 * q + (lane >> 5)];
      fx0[q] = Bs[buf][2 * q + (lane >> 5)][wc + (lane & 31)];
      fx1[q] = Bs[buf][2 * q + (lane >> 5)][wc + 32 + (lane & 31)];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the products
#pragma unroll
    for (int q = 0; q < BKC; ++q) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[q], fx0[q], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[q], fx1[q], acc1, 0, 0, 0);
    }
    if (more) store_tile(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  float* Yf = reinterpret_cast<float*>(g.Y + s * g.y_slice_stride);
  const int part = wc >> 6;
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

// Thread group g of a slice sum adds slices g, g + 4, g + 8, ... of element
// pair i in that order; the loads of up to SUM_PASS slices are issued before
// the first add (the sums run to 80 slices and more).
constexpr int SUM_PASS = 16;
__device__ inline float4 group_slice_sum(const float4* __restrict__ in, int slices, int64_t stride2, int64_t i,
                                         int g) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int s0 = g; s0 < slices; s0 += 4 * SUM_PASS) {
    float4 a[SUM_PASS];
#pragma unroll
    for (int q = 0; q < SUM_PASS; ++q) {
      a[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (s0 + 4 * q < slices) a[q] = in[(int64_t)(s0 + 4 * q) * stride2 + i];
    }
#pragma unroll
    for (int q = 0; q < SUM_PASS; ++q)
      if (s0 + 4 * q < slices) {
        v.x += a[q].x; v.y += a[q].y; v.z += a[q].z; v.w += a[q].w;
      }
  }
  return v;
}

// out[i] = sum_s in[s * stride + i] for i < count (complex), fixed order.
// Blocks of 64 outputs x 4 slice groups: thread (o, g) sums slices g, g + 4,
// ... of its output pair (16-byte loads), then the four group sums are added
// in order.  count and stride are even (pairs of complex).
__global__ void __launch_bounds__(256) sum_slices_kernel(const float4* __restrict__ in, int slices, int64_t stride2,
                                                        int64_t count2, float4* __restrict__ out) {
  __shared__ float4 red[4][64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + o;
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (i < count2) v = group_slice_sum(in, slices, stride2, i, g);
  red[g][o] = v;
  __syncthreads();
  if (g == 0 && i < count2) {
    float4 r = red[0][o];
    for (int q = 1; q < 4; ++q) {
      const float4 a = red[q][o];
      r.x += a.x; r.y += a.y; r.z += a.z; r.w += a.w;
    }
    out[i] = r;
  }
}

}  // namespace

namespace tdg {

void sum_slices_c64(hipStream_t stream, const void* in, int slices, int64_t stride, int64_t count, void* out) {
  // pairs of complex values: count and stride are even (the batched row stride is)
  const int64_t count2 = count / 2, blocks = (count2 + 63) / 64;
  hipLaunchKernelGGL(sum_slices_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, stream,
                     (const float4*)in, slices, stride / 2, count2, (float4*)out);
}

int cgemm_f32_kslices(int kc) { return (kc + BKC - 1) / BKC; }

// Launch Y[s] = A * X over split-K slices of `kslice` complex columns (a
// multiple of 16; the number of slices is ceil(Kc / kslice)) with tiling
// `variant`: 0 = 64 rows, 1 = 64 rows with the next tile prefetched and two
// LDS buffers, 2 = 128 rows.  ldx must be even (two instances per 16-byte load).
void cgemm_f32(hipStream_t stream, const void* A, int64_t lda, int M, int Kc, const void* X, int64_t ldx, void* Y,
               int64_t ldy, int64_t y_slice_stride, int ncols, int kslice, int variant) {
  GemmArgs g;
  g.A = (const float2*)A;
  g.lda = lda;
  g.M = M;
  g.Kc = Kc;
  g.X = (const float2*)X;
  g.ldx = ldx;
  g.Y = (float2*)Y;
  g.ldy = ldy;
  g.y_slice_stride = y_slice_stride;
  g.ncols = ncols;
  g.kslice = kslice;
  const int splits = (Kc + kslice - 1) / kslice;
  const bool avec = ((lda & 1) == 0) && (((uintptr_t)A & 15) == 0);
  if (variant == 0) {
    const dim3 grid((M + BM - 1) / BM, (ncols + BNI - 1) / BNI, splits);
    hipLaunchKernelGGL(cgemm_f32_mfma, grid, dim3(256), 0, stream, g);
    return;
  }
  if (variant == 1) {
    const dim3 grid((M + BM - 1) / BM, (ncols + BNI - 1) / BNI, splits);
    if (avec)
      hipLaunchKernelGGL(cgemm_f32_mfma_pf<true>, grid, dim3(256), 0, stream, g);
    else
      hipLaunchKernelGGL(cgemm_f32_mfma_pf<false>, grid, dim3(256), 0, stream, g);
    return;
  }
  const dim3 grid((M + BM2 - 1) / BM2, (ncols + BNI - 1) / BNI, splits);
  if (avec)
    hipLaunchKernelGGL(cgemm_f32_mfma_128<true>, grid, dim3(256), 0, stream, g);
  else
    hipLaunchKernelGGL(cgemm_f32_mfma_128<false>, grid, dim3(256), 0, stream, g);
}

}  // namespace tdg

// ---- BF16 split-precision product ------------------------------------------
// A in TDG_BF16X2 storage: a high plane of bf16 (re, im) pairs, row-major
// [M][lda] complex, followed by a low plane of the same shape; the element is
// hi + lo (about 16 significant bits).  X (complex64) is split the same way
// while it is staged into LDS.  Y = A_hi X_hi + A_hi X_lo + A_lo X_hi with
// FP32 accumulation (the dropped A_lo X_lo term is ~2^-16 relative) on
// v_mfma_f32_32x32x16_bf16, whose operand layout (checked on the device) is:
// lane l holds A[l%32][8*(l/32) + j] and B[8*(l/32) + j][l%32], j = 0..7.
// Tiles: 64 rows x 64 instances per block, 32 complex K columns per LDS stage,
// wave w owns rows 32*(w/2) .. +31 and real columns 64*(w%2) .. +63.  The
// expanded X tile is kept transposed in LDS (column-major) so each lane's 8
// consecutive K values are one 16-byte read.  Requires lda % 4 == 0.
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int BKC2 = 32;                 // complex K columns per stage
constexpr int KR = 2 * BKC2;             // real K per stage
constexpr int LPAD = 8;                  // bf16 padding per LDS row


struct GemmBf16Args {
  const unsigned short* Ahi;  // bf16 bits, [M][2*lda]
  const unsigned short* Alo;
  int64_t lda;                // complex elements per row
  int M, Kc;
  const float2* X;
  int64_t ldx;
  float2* Y;
  int64_t ldy;
  int64_t y_slice_stride;
  int ncols;
  int kslice;
};

__global__ void __launch_bounds__(256) cgemm_bf16x2_mfma(GemmBf16Args g) {
  __shared__ __align__(16) unsigned short Ah[BM][KR + LPAD];
  __shared__ __align__(16) unsigned short Al[BM][KR + LPAD];
  __shared__ __align__(16) unsigned short Xh[2 * BNI][KR + LPAD];
  __shared__ __align__(16) unsigned short Xl[2 * BNI][KR + LPAD];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.x * BM, b0 = blockIdx.y * BNI, s = blockIdx.z;
  const int kc_begin = s * g.kslice;
  const int kc_end = min(g.Kc, kc_begin + g.kslice);
  const int wr = (w >> 1) * 32, wc = (w & 1) * 64;
  floatx16 acc0, acc1;
  for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0.f;

  // A loader: row t/4, real K 16*(t%4) .. +15 of both planes (2 x 16 B each)
  const int arow = t >> 2, akr = (t & 3) * 16;
  const int gi = m0 + arow;
  // X loader: complex row t/8, instances 8*(t%8) .. +7
  const int xrow = t >> 3, xcol = (t & 7) * 8;
  for (int kc0 = kc_begin; kc0 < kc_end; kc0 += BKC2) {
    {
      const int kr0 = 2 * kc0 + akr;              // real K index of this thread's chunk
      const int kr_end = 2 * kc_end;
      uint4 h0 = make_uint4(0, 0, 0, 0), h1 = h0, l0 = h0, l1 = h0;
      if (gi < g.M) {
        const int64_t off = (int64_t)gi * 2 * g.lda + kr0;
        if (kr0 + 16 <= kr_end) {
          h0 = *reinterpret_cast<const uint4*>(g.Ahi + off);
          h1 = *reinterpret_cast<const uint4*>(g.Ahi + off + 8);
          l0 = *reinterpret_cast<const uint4*>(g.Alo + off);
          l1 = *reinterpret_cast<const uint4*>(g.Alo + off + 8);
        } else {
          unsigned short hb[16], lb[16];
          for (int q = 0; q < 16; ++q) {
            const bool in = kr0 + q < kr_end;
            hb[q] = in ? g.Ahi[off + q] : (unsigned short)0;
            lb[q] = in ? g.Alo[off + q] : (unsigned short)0;
          }
          h0 = *reinterpret_cast<uint4*>(hb);
          h1 = *reinterpret_cast<uint4*>(hb + 8);
          l0 = *reinterpret_cast<uint4*>(lb);
          l1 = *reinterpret_cast<uint4*>(lb + 8);
        }
      }
      *reinterpret_cast<uint4*>(&Ah[arow][akr]) = h0;
      *reinterpret_cast<uint4*>(&Ah[arow][akr + 8]) = h1;
      *reinterpret_cast<uint4*>(&Al[arow][akr]) = l0;
      *reinterpret_cast<uint4*>(&Al[arow][akr + 8]) = l1;
    }
    {
      const int kx = kc0 + xrow;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int b = b0 + xcol + q;
        float2 v = make_float2(0.f, 0.f);
        if (kx < kc_end && b < g.ncols) v = g.X[(int64_t)kx * g.ldx + b];
        const unsigned short rh = f2bf(v.x), ih = f2bf(v.y);
        const unsigned short rl = f2bf(v.x - bf2f(rh)), il = f2bf(v.y - bf2f(ih));
        const unsigned short nih = ih ^ 0x8000u, nil = il ^ 0x8000u;  // -Im, exact
        const int c = xcol + q, kr = 2 * xrow;
        // real expansion: [2k][b] = re, [2k+1][b] = -im, [2k][64+b] = im, [2k+1][64+b] = re
        *reinterpret_cast<unsigned int*>(&Xh[c][kr]) = (unsigned int)rh | ((unsigned int)nih << 16);
        *reinterpret_cast<unsigned int*>(&Xh[BNI + c][kr]) = (unsigned int)ih | ((unsigned int)rh << 16);
        *reinterpret_cast<unsigned int*>(&Xl[c][kr]) = (unsigned int)rl | ((unsigned int)nil << 16);
        *reinterpret_cast<unsigned int*>(&Xl[BNI + c][kr]) = (unsigned int)il | ((unsigned int)rl << 16);
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KR; ks += 16) {
      const int kb = ks + 8 * (lane >> 5);
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&Ah[wr + (lane & 31)][kb]);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(&Al[wr + (lane & 31)][kb]);
      const bf16x8 xh0 = *reinterpret_cast<const bf16x8*>(&Xh[wc + (lane & 31)][kb]);
      const bf16x8 xl0 = *reinterpret_cast<const bf16x8*>(&Xl[wc + (lane & 31)][kb]);
      const bf16x8 xh1 = *reinterpret_cast<const bf16x8*>(&Xh[wc + 32 + (lane & 31)][kb]);
      const bf16x8 xl1 = *reinterpret_cast<const bf16x8*>(&Xl[wc + 32 + (lane & 31)][kb]);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh0, acc0, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl0, acc0, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh1, acc1, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl1, acc1, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh1, acc1, 0, 0, 0);
    }
    __syncthreads();
  }

  float* Yf = reinterpret_cast<float*>(g.Y + s * g.y_slice_stride);
  const int part = wc >> 6;
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

// ---- BF16 split-precision product, tiling 1 ---------------------------------
// X is split once per product into XB (bf16 bits, the layout of bf16x2.h:
// the real-part rows of its expansion, K-blocked), so 8 consecutive K of one
// instance are one 16-byte read and 64 instances' chunks are contiguous.
using tdg::XB_ROWS;
static_assert(tdg::XB_TILE == BNI, "split operand tiles hold one block's instances");

__global__ void __launch_bounds__(256) expand_bf16x2_kernel(const float2* __restrict__ X, int64_t ldx, int Kc,
                                                            int ncols, unsigned short* __restrict__ XB,
                                                            int64_t ldxb) {
  // 32 complex K rows x 64 instances through LDS: read along instances, write along K
  __shared__ float2 tile[32][BNI + 1];
  const int ct = blockIdx.y, k0 = blockIdx.x * 32, t = threadIdx.x;
  for (int i = t; i < 32 * BNI; i += 256) {
    const int r = i / BNI, b = i % BNI;
    const int k = k0 + r, bb = ct * BNI + b;
    tile[r][b] = (k < Kc && bb < ncols) ? X[(int64_t)k * ldx + bb] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  // one 16-byte chunk (4 complex K of one instance) per thread and pass;
  // consecutive threads write consecutive instances' chunks
  for (int i = t; i < 2 * 8 * BNI; i += 256) {
    const int c = i % BNI, j = (i / BNI) % 8, p = i / (8 * BNI);
    uint4 w;
    w.x = xb_word(tile[4 * j][c].x, tile[4 * j][c].y, p);
    w.y = xb_word(tile[4 * j + 1][c].x, tile[4 * j + 1][c].y, p);
    w.z = xb_word(tile[4 * j + 2][c].x, tile[4 * j + 2][c].y, p);
    w.w = xb_word(tile[4 * j + 3][c].x, tile[4 * j + 3][c].y, p);
    *reinterpret_cast<uint4*>(&XB[xb_index(ct, p, c, 2 * (k0 + 4 * j), ldxb)]) = w;
  }
}

// Blocks take their (row tile, instance tile, K slice) XCD-aware: the row
// tiles of one slice, which read the same slice of X, run on one XCD and
// share its L2, so X is fetched about once per product.
//
// 128 rows x 64 instances per block, 16 complex K columns per LDS stage; wave
// w owns rows 64*(w/2) .. +63 and real columns 64*(w%2) .. +63 as 2 x 2 MFMA
// accumulators, so each 16-byte fragment read from LDS feeds six products.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// A word of two bf16 at positions e, e + 1: those at or past `end` zeroed.
__device__ inline unsigned int bf16_pair_mask(unsigned int w, int e, int end) {
  return e >= end ? 0u : (e + 1 >= end ? (w & 0xffffu) : w);
}

constexpr int BM3 = 128;
constexpr int BKC3 = 16;
constexpr int KR3 = 2 * BKC3;
constexpr int LPAD3 = 8;

// KR: real K per LDS stage, 32 (tiling 1) or 64 (tiling 3: rows
// are read in 128-byte pieces per plane instead of 64-byte ones, two blocks
// per CU by LDS).
template <int KR>
__global__ void __launch_bounds__(256) cgemm_bf16x2_mfma_v2(GemmBf16Args g, const unsigned short* __restrict__ XB,
                                                             int64_t ldxb) {
  constexpr int CH = KR / 8;       // 16-byte chunks per row and plane
  constexpr int RPI = 256 / CH;    // rows one pass of the block's threads covers
  constexpr int IT = 2 * BM3 / RPI;  // passes over both planes of A
  constexpr int ITX = IT / 2;        // of the stored (real-part) rows of X
  __shared__ __align__(16) unsigned short As[2][BM3][KR + LPAD3];
  __shared__ __align__(16) unsigned short Xs[2][XB_ROWS][KR + LPAD3];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int bx, ct, s;
  tdg::xcd_block3(bx, ct, s);
  const int m0 = bx * BM3, b0 = ct * BNI;
  const int kc_begin = s * g.kslice;
  const int kc_end = min(g.Kc, kc_begin + g.kslice);
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  floatx16 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // Tile loads go into registers (the next stage's while the current one is
  // multiplied); bf16 past the slice's K are zeroed when the tile is written to
  // LDS.  A chunk of 8 bf16 (4 complex) never crosses a split-K boundary
  // (slices are multiples of 16 complex) and stays inside its row (ld % 4 == 0).
  const int kr_end = 2 * kc_end;
  u32x4 ra[IT], rx[ITX];
  auto load_tile = [&](int kc0) {
    const int kr0 = 2 * kc0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      // chunk q of row `row` in plane p (the first IT / 2 passes: hi plane)
      const int q = t % CH, row = ((t / CH) + RPI * it) & (BM3 - 1), p = it / (IT / 2);
      const int kr = kr0 + 8 * q, gi = m0 + row;
      ra[it] = u32x4{0u, 0u, 0u, 0u};
      if (gi < g.M && kr < kr_end)
        ra[it] = *reinterpret_cast<const u32x4*>((p ? g.Alo : g.Ahi) + (int64_t)gi * 2 * g.lda + kr);
    }
#pragma unroll
    for (int it = 0; it < ITX; ++it) {
      // X: chunk q of stored row `row` in plane p, a wave taking one chunk of
      // all 64 rows (1 KB contiguous); zero past the padded row (a 64-K stage
      // that starts 16 columns past a multiple of 32 can reach beyond ldxb;
      // the padding itself is zero)
      const int u = t / BNI + 4 * it, row = t % BNI, q = u % CH, p = u / CH;
      const int kr = kr0 + 8 * q;
      rx[it] = u32x4{0u, 0u, 0u, 0u};
      if (kr < ldxb) rx[it] = *reinterpret_cast<const u32x4*>(XB + xb_index(ct, p, row, kr, ldxb));
    }
  };
  auto store_tile = [&](int kc0) {
    const int kr0 = 2 * kc0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int q = t % CH, row = ((t / CH) + RPI * it) & (BM3 - 1), p = it / (IT / 2);
      const int kr = kr0 + 8 * q;
      u32x4 v = ra[it];
      // keep bf16 e of the chunk only while kr + e < kr_end (two per 32-bit word)
      v.x = bf16_pair_mask(v.x, kr, kr_end);
      v.y = bf16_pair_mask(v.y, kr + 2, kr_end);
      v.z = bf16_pair_mask(v.z, kr + 4, kr_end);
      v.w = bf16_pair_mask(v.w, kr + 6, kr_end);
      *reinterpret_cast<u32x4*>(&As[p][row][8 * q]) = v;
    }
#pragma unroll
    for (int it = 0; it < ITX; ++it) {
      // the stored row and the imaginary-part row it gives
      const int u = t / BNI + 4 * it, row = t % BNI, q = u % CH, p = u / CH;
      const u32x4 v = rx[it];
      *reinterpret_cast<u32x4*>(&Xs[p][row][8 * q]) = v;
      *reinterpret_cast<u32x4*>(&Xs[p][BNI + row][8 * q]) = u32x4{xb_imag(v.x), xb_imag(v.y), xb_imag(v.z), xb_imag(v.w)};
    }
  };

  if (kc_begin < kc_end) {
    load_tile(kc_begin);
    store_tile(kc_begin);
  }
  __syncthreads();
  for (int kc0 = kc_begin; kc0 < kc_end; kc0 += KR / 2) {
    const bool more = kc0 + KR / 2 < kc_end;
    if (more) load_tile(kc0 + KR / 2);
#pragma unroll
    for (int ks = 0; ks < KR; ks += 16) {
      const int kb = ks + 8 * (lane >> 5);
      bf16x8 ah[2], al[2], xh[2], xl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ah[i] = *reinterpret_cast<const bf16x8*>(&As[0][wr + 32 * i + (lane & 31)][kb]);
        al[i] = *reinterpret_cast<const bf16x8*>(&As[1][wr + 32 * i + (lane & 31)][kb]);
        xh[i] = *reinterpret_cast<const bf16x8*>(&Xs[0][wc + 32 * i + (lane & 31)][kb]);
        xl[i] = *reinterpret_cast<const bf16x8*>(&Xs[1][wc + 32 * i + (lane & 31)][kb]);
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the products
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], xh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], xl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], xh[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
    if (more) store_tile(kc0 + KR / 2);
    __syncthreads();
  }

  // real column wc + 32 j + lane % 32: instance 32 j + lane % 32 of the tile, part wc / 64
  float* Yf = reinterpret_cast<float*>(g.Y + s * g.y_slice_stride);
  const int part = wc >> 6;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + wr + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (row >= g.M) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int b = b0 + 32 * j + (lane & 31);
        if (b < g.ncols) Yf[2 * ((int64_t)row * g.ldy + b) + part] = acc[i][j][r];
      }
    }
}

// ---- BF16 split-precision product, tilings 2 and 4 -------------------------
// BMT rows x 64 instances per block.  BMT = 256 (tiling 2): wave w owns
// rows 64 w .. +63 and all 128 real columns as 2 x 4 MFMA accumulators, so a
// fragment read from LDS feeds two (X) or four (A) products.  BMT = 128
// (tiling 4): wave w owns rows 64 (w / 2) .. +63 and the real or the
// imaginary output parts of the 64 instances (alternating between blocks) as
// 2 x 2 accumulators.
// A (both planes) and the stored rows of the split X are copied straight into
// LDS by 16-byte direct-to-LDS loads, into a ring of three stages of 16
// complex K: the loads of the next two stages are in flight while one is
// multiplied, with no registers held.  The imaginary-part columns' X
// fragments are formed from the real-part ones after they are read
// (xb_imag).  Blocks are placed on the XCDs as for tiling 1.  The
// ring takes 120 KB of LDS at BMT = 256 (one block per CU) and 72 KB at 128
// (two).
// In a stage, row r of a plane of A is 4 chunks of 8 bf16 (64 bytes); chunk c
// sits at slot c ^ ((r / 2) % 4), so the 32 rows of a fragment read spread
// over all banks.  X is kept as in memory, [plane][chunk][64 rows] (16 bytes
// each): one copy instruction moves one chunk of all rows.  Rows past M read
// row M - 1 and K past the product reads chunk 0 of the row: both multiply
// zeros of X or land in outputs never stored (X is zero from K = Kc on, and
// the row's own columns Kc .. lda - 1 are).
constexpr int KR4 = 32;                          // real K per stage
constexpr int ST4 = 3;                           // stages in the ring
constexpr int X4_BYTES = 2 * BNI * KR4 * 2;      // the stored X rows of a stage
constexpr int X4_COPIES = X4_BYTES / (256 * 16);  // 16-byte copies per lane and stage
// s_waitcnt immediate with vmcnt = n (gfx9 encoding: bits 3:0 and 15:14),
// expcnt and lgkmcnt at their maxima (no wait)
constexpr int waitcnt_vm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x0F70; }

typedef __attribute__((address_space(1))) void gsrc_t;
typedef __attribute__((address_space(3))) void ldst_t;

__device__ inline int swz(int row, int c) { return c ^ ((row >> 1) & 3); }

// xb_imag on each word of an X fragment
__device__ inline bf16x8 imag_fragment(bf16x8 f) {
  u32x4 v = __builtin_bit_cast(u32x4, f);
  v = u32x4{xb_imag(v.x), xb_imag(v.y), xb_imag(v.z), xb_imag(v.w)};
  return __builtin_bit_cast(bf16x8, v);
}

template <int BMT>
__global__ void __launch_bounds__(256) cgemm_bf16x2_mfma_v3(GemmBf16Args g, const unsigned short* __restrict__ XB,
                                                             int64_t ldxb) {
  static_assert(BMT == 256 || BMT == 128, "tile rows");
  constexpr int A_BYTES = 2 * BMT * KR4 * 2;       // both planes of a stage
  constexpr int A_COPIES = A_BYTES / (256 * 16);   // 16-byte copies per lane and stage
  constexpr int A_INS = BMT / 16;                  // copy instructions per plane (16 rows each)
  constexpr int NJ = BMT == 256 ? 4 : 2;           // column fragments per wave
  __shared__ __align__(16) unsigned char lds[ST4 * (A_BYTES + X4_BYTES)];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int bx, ct, s;
  tdg::xcd_block3(bx, ct, s);
  const int m0 = bx * BMT, b0 = ct * BNI;
  const int wr = BMT == 256 ? 64 * w : 64 * (w >> 1);  // the wave's first row
  // BMT = 128: imaginary output parts; which waves form the imaginary-part
  // fragments alternates with the block, so that work is not always on the
  // same SIMDs of a CU
  const int half = BMT == 256 ? 0 : ((w ^ bx ^ s) & 1);
  const int kc_begin = s * g.kslice;
  const int kc_end = min(g.Kc, kc_begin + g.kslice);
  const int nst = (kc_end - kc_begin + KR4 / 2 - 1) / (KR4 / 2);
  const int64_t row_bf = 2 * g.lda;  // bf16 per row of a plane (columns Kc .. lda - 1 hold zeros)

  // issue the direct-to-LDS copies of stage `st` (K from kc0) into ring slot q:
  // instruction ins copies A rows 16 (ins % A_INS) .. +15 of plane ins / A_INS
  // (A_COPIES per wave; lane l fills slot l % 4 of row l / 4), and each wave
  // two chunks of X (lane l: row l)
  auto issue = [&](int st, int q) {
    const int kr0 = 2 * (kc_begin + st * (KR4 / 2));
    unsigned char* abase = lds + q * (A_BYTES + X4_BYTES);
    unsigned char* xbase = abase + A_BYTES;
    const int rl = lane >> 2, sl = lane & 3;
#pragma unroll
    for (int j = 0; j < A_COPIES; ++j) {
      const int ins = w * A_COPIES + j, p = ins / A_INS, row = 16 * (ins % A_INS) + rl;
      const int gi = min(m0 + row, g.M - 1);
      int kr = kr0 + 8 * swz(row, sl);
      if (kr + 8 > row_bf) kr = 0;  // past the row: any finite chunk (X is zero there)
      const unsigned short* src = (p ? g.Alo : g.Ahi) + (int64_t)gi * row_bf + kr;
      __builtin_amdgcn_global_load_lds((gsrc_t*)src, (ldst_t*)(abase + (p * BMT + 16 * (ins % A_INS)) * 64), 16, 0,
                                       0);
    }
#pragma unroll
    for (int j = 0; j < X4_COPIES; ++j) {
      const int ins = w * X4_COPIES + j, p = ins >> 2, c = ins & 3;
      const unsigned short* src = XB + xb_index(ct, p, lane, kr0 + 8 * c, ldxb);
      __builtin_amdgcn_global_load_lds((gsrc_t*)src, (ldst_t*)(xbase + (p * 4 + c) * BNI * 16), 16, 0, 0);
    }
  };

  floatx16 acc[2][NJ];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  if (nst > 0) issue(0, 0);
  if (nst > 1) issue(1, 1);
  for (int st = 0; st < nst; ++st) {
    // this wave's copies of stage st have landed (those of st + 1 may not);
    // the barrier makes every wave's copies visible and frees slot (st + 2) % 3
    if (st + 1 < nst)
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(A_COPIES + X4_COPIES));
    else
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    // a plain barrier: the waits above are the only ones the copies need (a
    // __syncthreads fence would also wait for the next stage's copies)
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(63) & ~0x0F00);  // lgkmcnt(0): this wave's LDS reads are done
    __builtin_amdgcn_s_barrier();
    if (st + 2 < nst) issue(st + 2, (st + 2) % ST4);
    const unsigned char* abase = lds + (st % ST4) * (A_BYTES + X4_BYTES);
    const unsigned char* xbase = abase + A_BYTES;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int c = 2 * ks + (lane >> 5);
      bf16x8 ah[2], al[2], xh[NJ], xl[NJ];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wr + 32 * i + (lane & 31);
        const int off = (row * 4 + swz(row, c)) * 16;
        ah[i] = *reinterpret_cast<const bf16x8*>(abase + off);
        al[i] = *reinterpret_cast<const bf16x8*>(abase + BMT * 64 + off);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int off = (c * BNI + 32 * j + (lane & 31)) * 16;
        xh[j] = *reinterpret_cast<const bf16x8*>(xbase + off);
        xl[j] = *reinterpret_cast<const bf16x8*>(xbase + 4 * BNI * 16 + off);
      }
      __builtin_amdgcn_sched_barrier(0);
      // the imaginary-part columns from the real-part ones: fragments 2 and 3
      // (BMT = 256), or the wave's two fragments (BMT = 128, odd waves)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (BMT == 256) {
          xh[j + 2] = imag_fragment(xh[j]);
          xl[j + 2] = imag_fragment(xl[j]);
        } else if (half) {
          xh[j] = imag_fragment(xh[j]);
          xl[j] = imag_fragment(xl[j]);
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], xh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], xl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], xh[j], acc[i][j], 0, 0, 0);
        }
    }
  }

  // fragment j: instance 32 (j % 2) + lane % 32 of the tile; output part j / 2
  // (BMT = 256) or the wave's half (BMT = 128)
  float* Yf = reinterpret_cast<float*>(g.Y + s * g.y_slice_stride);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + wr + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (row >= g.M) continue;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int b = b0 + 32 * (j & 1) + (lane & 31);
        const int part = BMT == 256 ? (j >> 1) : half;
        if (b < g.ncols) Yf[2 * ((int64_t)row * g.ldy + b) + part] = acc[i][j][r];
      }
    }
}

// The split X of tilings 1 to 4 (the layout of bf16x2.h, as written by
// expand_bf16x2_kernel) straight from split-K slices of a product: x[k][b] =
// sum over slices s in order of in[s stride + k ldx + b], for k < Kc and b <
// ncols, zero elsewhere in [Kc rounded][tiles x 64].  Thread (pair o, slice
// group g) of a block sums slices g, g + 4, ... of two instances; the four
// group sums are added in order and written as bf16 hi / lo words.
__global__ void __launch_bounds__(256) sum_expand_bf16x2_kernel(const float4* __restrict__ in, int slices,
                                                                int64_t stride2, int Kc, int64_t ldx2, int ncols,
                                                                int tiles, unsigned short* __restrict__ XB,
                                                                int64_t ldxb) {
  __shared__ float4 red[4][64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + o;  // pair index over (k, instance pair)
  const int pairs_per_k = tiles * (BNI / 2);
  const int64_t npairs = (ldxb / 2) * (int64_t)pairs_per_k;
  const int k = (int)(i / pairs_per_k), bp = (int)(i % pairs_per_k), b = 2 * bp;
  const bool live = i < npairs && k < Kc && b < ncols;
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (live) v = group_slice_sum(in, slices, stride2, (int64_t)k * ldx2 + bp, g);
  red[g][o] = v;
  __syncthreads();
  if (g != 0 || i >= npairs) return;
  float4 r = red[0][o];
  for (int q = 1; q < 4; ++q) {
    const float4 a = red[q][o];
    r.x += a.x; r.y += a.y; r.z += a.z; r.w += a.w;
  }
  for (int h = 0; h < 2; ++h) {
    const int bb = b + h, ct = bb / BNI, c = bb % BNI;
    const float re = (live && bb < ncols) ? (h ? r.z : r.x) : 0.f, im = (live && bb < ncols) ? (h ? r.w : r.y) : 0.f;
    for (int p = 0; p < 2; ++p)
      *reinterpret_cast<unsigned int*>(&XB[xb_index(ct, p, c, 2 * k, ldxb)]) = xb_word(re, im, p);
  }
}

// dst (TDG_BF16X2, [rows][ld_dst]) <- src complex (float or double, [rows][ld_src]);
// columns cols .. ld_dst-1 of dst are zero-filled.
template <typename S>
__global__ void split_bf16x2_kernel(const S* __restrict__ src, int64_t ld_src, int64_t rows, int64_t cols,
                                    unsigned short* __restrict__ dst, int64_t ld_dst) {
  const int64_t plane = rows * ld_dst * 2;
  const int64_t i = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ld_dst; c += (int64_t)gridDim.x * blockDim.x) {
    float re = 0.f, im = 0.f;
    if (c < cols) {
      re = (float)src[i * ld_src + c].x;
      im = (float)src[i * ld_src + c].y;
    }
    const unsigned short rh = f2bf(re), ih = f2bf(im);
    const int64_t o = (i * ld_dst + c) * 2;
    dst[o] = rh;
    dst[o + 1] = ih;
    dst[plane + o] = f2bf(re - bf2f(rh));
    dst[plane + o + 1] = f2bf(im - bf2f(ih));
  }
}

}  // namespace

namespace tdg {

size_t cgemm_bf16x2_work_bytes(int Kc, int ncols) {
  const int64_t ldxb = 2 * (((int64_t)Kc + 31) / 32 * 32);
  return (size_t)((ncols + BNI - 1) / BNI) * 2 * BNI * ldxb * sizeof(unsigned short);
}

void expand_bf16x2(hipStream_t stream, const void* X, int64_t ldx, int Kc, int ncols, void* work) {
  const int64_t ldxb = 2 * (((int64_t)Kc + 31) / 32 * 32);
  const int tiles = (ncols + BNI - 1) / BNI;
  hipLaunchKernelGGL(expand_bf16x2_kernel, dim3((unsigned)(ldxb / 64), (unsigned)tiles), dim3(256), 0, stream,
                     (const float2*)X, ldx, Kc, ncols, (unsigned short*)work, ldxb);
}

void sum_expand_bf16x2(hipStream_t stream, const void* in, int slices, int64_t stride, int Kc, int64_t ldx, int ncols,
                       void* work) {
  const int64_t ldxb = 2 * (((int64_t)Kc + 31) / 32 * 32);
  const int tiles = (ncols + BNI - 1) / BNI;
  const int64_t npairs = (ldxb / 2) * (int64_t)tiles * (BNI / 2);
  hipLaunchKernelGGL(sum_expand_bf16x2_kernel, dim3((unsigned)((npairs + 63) / 64)), dim3(256), 0, stream,
                     (const float4*)in, slices, stride / 2, Kc, ldx / 2, ncols, tiles, (unsigned short*)work, ldxb);
}

// variant 0: 64-row tiles, X split while staged; variants 1 to 4: X split
// once into `work` (cgemm_bf16x2_work_bytes), then 128-row tiles (variant 1),
// 256-row tiles staged by direct-to-LDS loads (variant 2), 128-row tiles of
// 64 real K per stage (variant 3), or 128-row tiles staged by direct-to-LDS
// loads (variant 4).
// With x_expanded, `work` already holds that expansion (sum_expand_bf16x2)
// and X is not read.
void cgemm_bf16x2(hipStream_t stream, const void* A, int64_t lda, int M, int Kc, const void* X, int64_t ldx,
                  void* Y, int64_t ldy, int64_t y_slice_stride, int ncols, int kslice, int variant, void* work,
                  bool x_expanded) {
  GemmBf16Args g;
  g.Ahi = (const unsigned short*)A;
  g.Alo = (const unsigned short*)A + (int64_t)M * lda * 2;
  g.lda = lda;
  g.M = M;
  g.Kc = Kc;
  g.X = (const float2*)X;
  g.ldx = ldx;
  g.Y = (float2*)Y;
  g.ldy = ldy;
  g.y_slice_stride = y_slice_stride;
  g.ncols = ncols;
  g.kslice = kslice;
  const int splits = (Kc + kslice - 1) / kslice;
  if (variant >= 1 && variant <= 4 && work) {
    const int64_t ldxb = 2 * (((int64_t)Kc + 31) / 32 * 32);
    const int tiles = (ncols + BNI - 1) / BNI;
    if (!x_expanded) expand_bf16x2(stream, X, ldx, Kc, ncols, work);
    if (variant == 3) {
      const dim3 grid((M + BM3 - 1) / BM3, tiles, splits);
      hipLaunchKernelGGL(cgemm_bf16x2_mfma_v2<64>, grid, dim3(256), 0, stream, g, (const unsigned short*)work, ldxb);
      return;
    }
    if (variant == 2) {
      const dim3 grid((M + 255) / 256, tiles, splits);
      hipLaunchKernelGGL(cgemm_bf16x2_mfma_v3<256>, grid, dim3(256), 0, stream, g, (const unsigned short*)work, ldxb);
      return;
    }
    if (variant == 4) {
      const dim3 grid((M + 127) / 128, tiles, splits);
      hipLaunchKernelGGL(cgemm_bf16x2_mfma_v3<128>, grid, dim3(256), 0, stream, g, (const unsigned short*)work, ldxb);
      return;
    }
    const dim3 grid((M + BM3 - 1) / BM3, tiles, splits);
    hipLaunchKernelGGL(cgemm_bf16x2_mfma_v2<32>, grid, dim3(256), 0, stream, g, (const unsigned short*)work, ldxb);
    return;
  }
  const dim3 grid((M + BM - 1) / BM, (ncols + BNI - 1) / BNI, splits);
  hipLaunchKernelGGL(cgemm_bf16x2_mfma, grid, dim3(256), 0, stream, g);
}

void split_bf16x2(hipStream_t stream, const void* src, int src_is_double, int64_t ld_src, int64_t rows, int64_t cols,
                  void* dst, int64_t ld_dst) {
  const dim3 grid((unsigned)std::min<int64_t>(64, (ld_dst + 255) / 256), (unsigned)rows);
  if (src_is_double)
    hipLaunchKernelGGL(split_bf16x2_kernel<double2>, grid, dim3(256), 0, stream, (const double2*)src, ld_src, rows,
                       cols, (unsigned short*)dst, ld_dst);
  else
    hipLaunchKernelGGL(split_bf16x2_kernel<float2>, grid, dim3(256), 0, stream, (const float2*)src, ld_src, rows,
                       cols, (unsigned short*)dst, ld_dst);
}

}  // namespace tdg
