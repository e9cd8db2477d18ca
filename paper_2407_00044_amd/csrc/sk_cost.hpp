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
    {0, 128, 128, 6.590f, 3.119f, 2.0501f, 1.8695f, 0.917f, 2.121f, 0.0000f, 1.903f},
    {2, 256, 256, 7.952f, 7.297f, 1.5793f, 1.0144f, 2.626f, 4.771f, 0.0000f, 11.593f},
    {2, 256, 128, 7.462f, 3.340f, 0.9197f, 0.6548f, 2.148f, 1.754f, 0.0000f, 5.178f},
    {2, 128, 128, 6.817f, 1.410f, 0.5496f, 0.4100f, 3.987f, 1.133f, 0.0000f, 1.413f},
    {3, 256, 256, 5.986f, 10.699f, 1.5708f, 1.1121f, 6.846f, 3.966f, 0.0531f, 9.834f},
    {3, 256, 128, 6.552f, 3.516f, 0.8382f, 0.5553f, 2.398f, 1.754f, 0.0000f, 5.168f},
    {3, 128, 128, 7.307f, 1.038f, 0.5018f, 0.3684f, 5.347f, 0.778f, 0.0000f, 1.344f},
    {3, 64, 128, 7.072f, 0.092f, 0.3521f, 0.2931f, 8.152f, 0.379f, 0.0000f, 0.838f},
};
// clang-format on

// The auto mode splits tiles only when the launch without splits is
// predicted to take more than this factor times the Stream-K launch.  For
// the 16- and 8-bit kernels the model's error reaches 5-12% on its
// calibration launches and ~5% either way on the BF16 shape sweep, where a
// smaller margin let two splits lose.  The FP32 kernels are bound by the
// matrix cores rather than by the L2, and the model fits their calibration
// launches within 2.6%.
constexpr double kAutoMargin = 1.08;
constexpr double kAutoMarginF32 = 1.03;
inline double auto_margin(int32_t dt) { return dt == 0 ? kAutoMarginF32 : kAutoMargin; }

// Row of (input type, tile); f16 takes bf16's.  A tile without a row takes
// the row of the same type whose tile area is closest.
inline const CostRow* cost_row(int32_t dt, int32_t bm, int32_t bn) {
  // f16 and MXFP4 (four 16-byte steps per iteration) as bf16, MXFP8 as e4m3
  const int32_t d = (dt == 1 || dt == 5) ? 2 : dt == 4 ? 3 : dt;
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
