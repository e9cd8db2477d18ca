// Launch-time model of the library's auto policy (host only).
//
// The report names a predictive model of block-to-time behaviour as future
// work (Results, the Block2Time paragraph; Future Work).  This model predicts
// the time of a launch from its schedule: each workgroup's time is the sum
// over its segments (Stream-K segments first, then its whole tiles) of
//
//     t_tile + iterations * t_it(n) * (1 + l2 for Stream-K iterations)
//     + t_cin            when the segment runs the epilogue and beta != 0
//     + t_store          for a PARTIAL segment (store and publish)
//     + npeers * t_peer  for a FINISH segment, which first waits until each
//                        peer's partial tile has been published,
//
// and the launch takes t_launch plus its slowest workgroup.  t_it(n) is the
// time of one MAC iteration with n workgroups running at once, interpolated
// between a light load (64) and a full load (256 workgroups): the L2 feeds
// each CU more slowly as more CUs share it.  l2 is the share of an iteration
// lost when the workgroups of an XCD walk K at different k-phases (Stream-K)
// rather than in step (data-parallel waves).  A data-parallel grid of T
// tiles takes ceil(T / CUs) waves of one tile each.
//
// The constants are measured on MI355X per input type and tile by
// paper_2407_00044_amd/calibrate.py (f16 uses the bf16 rows, MXFP8 the e4m3
// rows and MXFP4 the bf16 rows: the same data path per iteration).  They are policy: no result depends on them, only which
// launch the auto mode picks.
#pragma once

#include <stdint.h>

namespace sk {

struct CostRow {
  int32_t dt, bm, bn;
  float t_launch, t_tile, t_it_full, t_it_light, t_store, t_peer, l2, t_cin;   // us
};

// clang-format off
static const CostRow kCostTable[] = {
    {0, 128, 128, 6.230f, 3.484f, 2.0634f, 1.9028f, 2.138f, 1.753f, 0.0000f, 2.031f},
    {2, 256, 256, 6.324f, 9.941f, 1.5960f, 1.0280f, 3.616f, 4.852f, 0.0000f, 10.291f},
    {2, 256, 128, 7.311f, 3.484f, 0.8967f, 0.5808f, 2.023f, 2.059f, 0.0000f, 5.420f},
    {2, 128, 128, 7.169f, 1.162f, 0.5284f, 0.3663f, 4.539f, 1.101f, 0.0000f, 1.376f},
    {3, 256, 256, 5.651f, 12.693f, 1.5662f, 1.1314f, 8.360f, 4.088f, 0.0460f, 10.279f},
    {3, 256, 128, 6.626f, 3.902f, 0.8283f, 0.5625f, 2.085f, 2.269f, 0.0000f, 5.109f},
    {3, 128, 128, 7.240f, 1.309f, 0.5099f, 0.3593f, 4.852f, 0.900f, 0.0000f, 1.363f},
    {3, 64, 128, 7.308f, 0.000f, 0.3465f, 0.2892f, 8.106f, 0.467f, 0.0000f, 0.689f},
};
// clang-format on

// The auto mode splits tiles only when the launch without splits is
// predicted to take more than this factor times the Stream-K launch.  For
// the 16- and 8-bit kernels the model's error reaches 6-13% on its
// calibration launches, and on the BF16 shape sweep the splits that lost
// were predicted at most 5% faster (256x256 tiles, every tile split), while
// the 8192x11008x4096 products of a linear layer gain 2-3% where it
// predicts 7.2-7.5%.  The FP32 kernels are bound by the matrix cores rather
// than by the L2, and the model fits their calibration launches within
// 2.9%.
constexpr double kAutoMargin = 1.07;
constexpr double kAutoMarginF32 = 1.03;
inline double auto_margin(int32_t dt) { return dt == 0 ? kAutoMarginF32 : kAutoMargin; }

// Row of (input type, tile); f16 takes bf16's.  A tile without a row takes
// the row of the same type whose tile area is closest.
inline const CostRow* cost_row(int32_t dt, int32_t bm, int32_t bn) {
  // f16 and MXFP4 (four 16-byte steps per iteration) as bf16, MXFP8 (both
  // element formats), per-tensor e5m2 and MXFP6 (two steps) as e4m3
  const int32_t d = (dt == 1 || dt == 5) ? 2 : dt >= 4 ? 3 : dt;
  const CostRow* best = nullptr;
  int64_t best_gap = 0;
  for (const CostRow& r : kCostTable) {
    if (r.dt != d) continue;
    if (r.bm == bm && r.bn == bn) return &r;
    const int64_t a = (int64_t)r.bm * r.bn - (int64_t)bm * bn;
    const int64_t gap = a < 0 ? -a : a;
    if (best == nullptr || gap < best_gap) {
      best = &r;
      best_gap = gap;
    }
  }
  return best;
}

// Time of one MAC iteration with n workgroups running at once.
inline double iter_time(const CostRow& c, int64_t n) {
  double f = (double)(n - 64) / 192.0;
  f = f < 0.0 ? 0.0 : f > 1.0 ? 1.0 : f;
  return c.t_it_light + (c.t_it_full - c.t_it_light) * f;
}

}  // namespace sk
