// Kernel argument structures shared by the host launcher and the kernels.
#pragma once

#include <stdint.h>

#include "../../include/streamk.h"

namespace sk {

// One GEMM problem as the kernels see it.  For a grouped launch an array of
// these lives in device memory (written by sk_grouped_prepare).
struct ProbDesc {
  const void* A;
  const void* B;
  const void* Cin;
  void* Cout;
  int64_t M, N, K;
  int64_t lda, ldb, ldc;     // elements
  float alpha_s;             // alpha * scale_a * scale_b
  float beta;
  int32_t tm, tn;            // tile grid
  int32_t I;                 // MAC iterations per tile
  int32_t aligned;           // 16-byte loads allowed for A and B
  int64_t tile_start;        // first global tile of this problem
  int64_t iter_start;        // global Stream-K iteration of that tile
                             // (W when the problem has no Stream-K tile)
};

struct KParams {
  ProbDesc prob;             // single-problem launch
  const ProbDesc* group;     // grouped launch: device array, else nullptr
  int32_t nprobs;
  int32_t dtype_c;
  int64_t T, S, W, g, q, rho;
  int32_t group_m;
  int32_t xcd_remap;
  int32_t dp_grid;           // 1: baseline grid, hardware workgroup -> tile
  int32_t reverse_ids;
  int32_t* err;              // device error word
  int32_t* flags;            // one arrival counter per Stream-K tile
  float* slots;              // g partial tiles of BM*BN floats
  int64_t spin_limit;
  // debug hooks (nullptr when unused)
  sk_segment* trace;
  int64_t trace_cap;
  int64_t* trace_count;
  int32_t* cover;
  int64_t cover_stride;
  int32_t partial_delay;
};

// Workspace layout: [256 B header: error word][flags, S int32, padded to
// 256 B][g slots of BM*BN floats].
inline int64_t ws_flags_offset() { return 256; }
inline int64_t ws_slots_offset(int64_t S) { return 256 + ((S * 4 + 255) / 256) * 256; }
inline int64_t ws_bytes(int64_t S, int64_t g, int64_t bm, int64_t bn) {
  return ws_slots_offset(S) + g * bm * bn * 4;
}

}  // namespace sk
