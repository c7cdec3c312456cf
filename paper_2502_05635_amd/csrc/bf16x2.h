// BF16 split precision (TDG_BF16X2): a float is carried as a bf16 hi part
// (round to nearest even) and a bf16 lo part (the rounded remainder), and the
// products accumulate hi*hi + hi*lo + lo*hi in FP32.  Shared by the product
// kernels and by the batched stage kernel, which writes the split operand of
// the next product directly.
//
// Split operand layout (the second and third product tilings): for tile ct of
// XB_TILE instances, plane p (0 = hi, 1 = lo), row c < XB_ROWS and real K
// index kr, XB[((ct * 2 + p) * XB_ROWS + c) * ldxb + kr] holds the real
// expansion of x[k][XB_TILE ct + (c % XB_TILE)]: rows c < XB_TILE (real parts
// of the outputs) carry (re, -im) at kr = (2k, 2k + 1), rows c >= XB_TILE
// (imaginary parts) carry (im, re).  ldxb is 2 Kc rounded up to 64, and the
// entries from 2 Kc up to ldxb are zero.
#pragma once

#include <hip/hip_runtime.h>

namespace tdg {

constexpr int XB_TILE = 64;            // instances per tile
constexpr int XB_ROWS = 2 * XB_TILE;   // rows per tile and plane

__device__ inline unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// The word (two bf16) of x = re + i im at K pair (2k, 2k + 1) of plane p, in a
// row of real parts (imag_row false: (re, -im)) or of imaginary parts (im, re).
__device__ inline unsigned int xb_word(float re, float im, int p, bool imag_row) {
  const unsigned short rh = f2bf(re), ih = f2bf(im);
  const unsigned short r = p ? f2bf(re - bf2f(rh)) : rh, i = p ? f2bf(im - bf2f(ih)) : ih;
  return imag_row ? ((unsigned int)i | ((unsigned int)r << 16)) : ((unsigned int)r | ((unsigned int)(i ^ 0x8000u) << 16));
}

}  // namespace tdg
