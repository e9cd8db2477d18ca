// Stream-K schedule arithmetic, shared by the host library and the kernels.
//
// The report (Background section) describes Stream-K as dividing the total
// multiply-accumulate work of a GEMM into even-sized units spread over all
// cores, instead of handing each core whole output tiles and leaving some
// idle when the tile count does not divide evenly.  This file fixes the
// concrete rules used by this library:
//
//  * tiles:      tm = ceil(M/BM), tn = ceil(N/BN), T_p = tm*tn per problem,
//                I_p = max(1, ceil(K/BK)) MAC iterations per tile (a K = 0
//                problem keeps one empty iteration so that its tiles still run
//                the epilogue);
//  * tile order: problem-major; row-major inside a problem, or bands of
//                group_m tile rows walked down the band first;
//  * split:      Stream-K tiles [0,S), data-parallel tiles [S,T);
//  * balance:    W Stream-K iterations over g workgroups, q = W/g, rho = W%g,
//                workgroup x owns [x*q + min(x,rho), ... + q + (x<rho));
//  * fixup:      the workgroup that runs a split tile's iteration 0 finishes
//                it after the partial tiles of workgroups x+1..y, where y owns
//                the tile's last iteration.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define SK_HD __host__ __device__ __forceinline__
#else
#define SK_HD inline
#endif

namespace sk {

SK_HD int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
SK_HD int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
SK_HD int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

// Local tile index u -> (tile row, tile column).
SK_HD void tile_coords(int64_t u, int32_t tm, int32_t tn, int32_t group_m,
                       int32_t* r, int32_t* c) {
  if (group_m <= 0) {
    *r = (int32_t)(u / tn);
    *c = (int32_t)(u % tn);
    return;
  }
  int64_t band_tiles = (int64_t)group_m * tn;
  int64_t band = u / band_tiles;
  int64_t h = imin(group_m, tm - band * group_m);
  int64_t v = u - band * band_tiles;
  *r = (int32_t)(band * group_m + v % h);
  *c = (int32_t)(v / h);
}

// Cost of one partial tile (store, wait, load, add) in MAC iterations of
// the same tile, measured on MI355X.  16-bit and e4m3 iterations (64 / 128
// K-values): about 4 up to 256x128 tiles, about 8 for 256x256.  An FP32
// iteration (32 K-values on the FP32 matrix cores) takes ~4.5x as long
// (2.5 vs 0.55 us for a lone 128x128 workgroup), so there a partial tile
// costs about one iteration.
SK_HD int64_t fixup_iters(int64_t bm, int64_t bn, int64_t bk) {
  return bk == 32 ? imax(1, bm * bn / 32768) : imax(4, bm * bn / 8192);
}

// Split point S for T tiles on g workgroups.  Hybrid (mode 0) and auto
// (mode 3, whose host policy may then keep S = 0): the two-tile rule, S = 0
// when T is a multiple of g, else min(T, T mod g + g).  All Stream-K (mode
// 1): S = T.  dp_tiles >= 0 overrides: S = T - dp_tiles.
SK_HD int64_t split_point(int64_t T, int64_t g, int32_t mode, int64_t dp_tiles) {
  int64_t S;
  if (mode == 2) return 0;                 // baseline DP grid
  if (mode == 1) S = T;                    // all Stream-K
  else S = (g <= 0 || T % g == 0) ? 0 : imin(T, T % g + g);
  if (dp_tiles >= 0) S = T - imin(dp_tiles, T);
  return S;
}

// First iteration of workgroup x under the balanced split.
SK_HD int64_t range_begin(int64_t x, int64_t q, int64_t rho) {
  return x * q + imin(x, rho);
}

// Workgroup owning global Stream-K iteration `it` (inverse of range_begin).
SK_HD int64_t iter_owner(int64_t it, int64_t q, int64_t rho) {
  int64_t big = rho * (q + 1);             // iterations owned by x < rho
  if (it < big) return it / (q + 1);
  return rho + (it - big) / q;
}

// Logical workgroup id of hardware workgroup b.
SK_HD int64_t logical_id(int64_t b, int64_t g, int32_t xcd_remap, int32_t reverse) {
  if (reverse) return g - 1 - b;
  if (xcd_remap && g % 8 == 0) return (b % 8) * (g / 8) + b / 8;
  return b;
}

// Elements of K per MAC iteration: 128 bytes of K for every input type
// (MXFP4: 256 elements of half a byte), except MXFP6: 128 elements, 96
// bytes (four blocks of 32 six-bit values).
SK_HD int32_t k_per_iter(int32_t dtype_ab) {
  return dtype_ab == 0 ? 32 : dtype_ab == 5 ? 256 : dtype_ab >= 3 ? 128 : 64;
}

// Bytes per element of the kernels' view of an operand (MXFP4 and MXFP6
// operands are seen as bytes: two, or four per three, elements).
SK_HD int32_t elem_bytes(int32_t dtype) {
  return dtype == 0 ? 4 : dtype >= 3 ? 1 : 2;
}

// Bytes of n elements (n even for MXFP4, a multiple of 4 for MXFP6; a
// count past those rounds up to the byte holding the last element's bits).
SK_HD int64_t elems_to_bytes(int32_t dtype, int64_t n) {
  if (dtype == 5) return (n + 1) / 2;
  if (dtype == 6 || dtype == 7) return (3 * n + 3) / 4;
  return n * elem_bytes(dtype);
}

}  // namespace sk
