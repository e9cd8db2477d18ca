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
  int32_t user_index;        // index of the problem in the caller's array
  int32_t act;               // sk_activation of the epilogue
  const void* sA;            // MXFP8: E8M0 scales of A, row i at sA + i * ldsa
  const void* sB;            //        and of B, column j at sB + j * ldsb
  int64_t ldsa, ldsb;        //        (bytes; one scale per 32 K-values)
  const float* bias;         // N FP32 values added before the activation, or null
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
  uint32_t* epoch;           // launches completed on this workspace
  uint32_t* done;            // workgroups of the running launch that ended
  uint32_t* tokens;          // per workgroup: launch tag of its partial tile
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

// Workspace layout (every offset fixed, none depends on the problem):
//   [0, 256)            header: error word, epoch word, done counter
//   [256, 256 + 4*kMaxWG)  one 32-bit token per persistent workgroup
//   [kSlotsOffset, ...)  g partial tiles of BM*BN floats
// A contributor publishes its partial tile by writing the launch's tag into
// its own token; the tag is the epoch word plus one, and the last workgroup
// of every launch advances the epoch, so tokens of earlier launches never
// match and nothing has to be cleared between launches.
constexpr int64_t kMaxWG = 4096;                       // persistent workgroups
constexpr int64_t kHeaderBytes = 256;
constexpr int64_t kTokensOffset = kHeaderBytes;
constexpr int64_t kSlotsOffset = kTokensOffset + 4 * kMaxWG;   // 16640
inline int64_t ws_bytes(int64_t S, int64_t g, int64_t bm, int64_t bn) {
  return S > 0 ? kSlotsOffset + g * bm * bn * 4 : kHeaderBytes;
}

}  // namespace sk
