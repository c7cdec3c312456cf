// BF16 split precision (TDG_BF16X2): a float is carried as a bf16 hi part
// (round to nearest even) and a bf16 lo part (the rounded remainder), and the
// products accumulate hi*hi + hi*lo + lo*hi in FP32.  Shared by the product
// kernels and by the batched stage kernel, which writes the split operand of
// the next product directly.
//
// Split operand layout (product tilings 1 to 4): the stored part of X's real
// expansion is the rows that give the real parts of the outputs, holding
// (re, -im) of x[k][XB_TILE ct + c] at real K index kr = (2k, 2k + 1), for
// tile ct of XB_TILE instances, plane p (0 = hi, 1 = lo) and instance c <
// XB_TILE.  The rows that give the imaginary parts, (im, re), are the same
// words with their halves swapped and one sign flipped (xb_imag), formed by
// the product kernels.  The array is K-blocked: chunk j = kr / 8 of instance
// c is 8 bf16 (16 bytes) at xb_index(ct, p, c, 8 j, ldxb), and the chunks of
// the tile's 64 instances for one (p, j) are contiguous (1 KB).  ldxb is 2 Kc
// rounded up to 64, and the entries from 2 Kc up to ldxb are zeros (of either
// sign).
#pragma once

#include <hip/hip_runtime.h>

namespace tdg {

constexpr int XB_TILE = 64;            // instances per tile
constexpr int XB_ROWS = 2 * XB_TILE;   // rows of the real expansion per tile and plane

__device__ inline unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// Element offset of real K index kr of instance c (tile ct, plane p).
__host__ __device__ inline int64_t xb_index(int ct, int p, int c, int64_t kr, int64_t ldxb) {
  return (((int64_t)(ct * 2 + p) * (ldxb / 8) + kr / 8) * XB_TILE + c) * 8 + kr % 8;
}

// The stored word (two bf16) of x = re + i im at K pair (2k, 2k + 1) of plane
// p: (re, -im), the part's bf16 hi (p = 0) or the bf16 of its remainder (p = 1).
__device__ inline unsigned int xb_word(float re, float im, int p) {
  const unsigned short rh = f2bf(re), ih = f2bf(im);
  const unsigned short r = p ? f2bf(re - bf2f(rh)) : rh, i = p ? f2bf(im - bf2f(ih)) : ih;
  return (unsigned int)r | ((unsigned int)(i ^ 0x8000u) << 16);
}

// The word of the imaginary-part row, (im, re), from a stored word (re, -im):
// halves swapped, then the sign of the new low half flipped.  The split is
// symmetric under negation, so this is exact in both planes.
__device__ inline unsigned int xb_imag(unsigned int w) { return ((w >> 16) | (w << 16)) ^ 0x8000u; }

}  // namespace tdg
