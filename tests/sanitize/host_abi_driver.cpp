// Host-only driver of libstreamk's planning entry points, built together
// with csrc/sk_api.hip under AddressSanitizer and UndefinedBehaviorSanitizer
// (host code only) by tests/test_sanitizers.py.  No GPU is needed: the tile
// menu is registered by hand (kernel handles that are never launched) and
// every call passes num_cu > 0.  Exits non-zero on any contract violation;
// the sanitizers abort on memory or undefined-behaviour errors.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/streamk.h"
#include "../../paper_2407_00044_amd/csrc/sk_registry.hpp"

static int failures = 0;
#define EXPECT(c)                                                     \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__,    \
              __LINE__, #c);                                          \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64() {   // splitmix64
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }

static const int kDummy = 0;

static void register_menu() {
  const int tiles[][2] = {{256, 256}, {256, 128}, {128, 128}, {64, 128}};
  for (int la = 0; la < 2; ++la)
    for (int lb = 0; lb < 2; ++lb) {
      sk::register_kernel({0, la, lb, 128, 128, 2, 256, &kDummy});
      for (int dt = 1; dt <= 3; ++dt)
        for (int t = 0; t < 4; ++t) {
          if (t == 3 && dt != 3) continue;
          sk::register_kernel({dt, la, lb, tiles[t][0], tiles[t][1], 2, 512, &kDummy});
        }
    }
}

static sk_problem problem(int64_t M, int64_t N, int64_t K, int dt, int la, int lb) {
  sk_problem p;
  memset(&p, 0, sizeof(p));
  p.M = M; p.N = N; p.K = K;
  p.layout_a = la; p.layout_b = lb;
  p.lda = la == SK_ROW_MAJOR ? (K > 0 ? K : 1) : (M > 0 ? M : 1);
  p.ldb = lb == SK_ROW_MAJOR ? (N > 0 ? N : 1) : (K > 0 ? K : 1);
  p.ldc = N > 0 ? N : 1;
  p.dtype_ab = dt; p.dtype_c = SK_F32;
  p.alpha = 1.f; p.beta = 0.f; p.scale_a = 1.f; p.scale_b = 1.f;
  return p;
}

static sk_config config(int dt, int bm, int bn, int cus, int mode) {
  sk_config c;
  memset(&c, 0, sizeof(c));
  c.block_m = bm; c.block_n = bn;
  c.block_k = dt == SK_F32 ? 32 : dt == SK_F8E4M3 ? 128 : 64;
  c.num_cu = cus; c.mode = mode; c.dp_tiles = -1; c.group_m = -1; c.xcd_remap = 1;
  return c;
}

// Schedule of a problem set: every (tile, k) of the Stream-K tiles and every
// data-parallel tile covered exactly once.
static int planned = 0;

static void check_schedule(const std::vector<sk_problem>& ps, const sk_config& c) {
  sk_plan_info info;
  if (sk_plan(ps.data(), (int32_t)ps.size(), &c, &info) != SK_OK) return;
  ++planned;
  int64_t count = 0;
  EXPECT(sk_schedule(ps.data(), (int32_t)ps.size(), &c, nullptr, 0, &count) == SK_OK);
  std::vector<sk_segment> segs((size_t)count + 1);
  if (count > 0) {
    int64_t small = 0;
    EXPECT(sk_schedule(ps.data(), (int32_t)ps.size(), &c, segs.data(), count - 1, &small) ==
           SK_ERR_CAPACITY);
  }
  EXPECT(sk_schedule(ps.data(), (int32_t)ps.size(), &c, segs.data(), count, &count) == SK_OK);
  std::vector<int32_t> order(ps.size());
  EXPECT(sk_plan_order(ps.data(), (int32_t)ps.size(), &c, order.data()) == SK_OK);
  std::vector<std::vector<int32_t>> cover((size_t)info.T);
  for (int64_t t = 0; t < info.T; ++t) cover[(size_t)t].assign((size_t)info.max_iters, 0);
  for (int64_t i = 0; i < count; ++i) {
    const sk_segment& s = segs[(size_t)i];
    EXPECT(s.tile >= 0 && s.tile < info.T);
    EXPECT(s.k_begin >= 0 && s.k_begin < s.k_end && s.k_end <= info.max_iters);
    if (s.tile < 0 || s.tile >= info.T || s.k_end > info.max_iters || s.k_begin < 0) continue;
    for (int k = s.k_begin; k < s.k_end; ++k) cover[(size_t)s.tile][(size_t)k] += 1;
  }
  for (int64_t t = 0; t < info.T; ++t) {
    int32_t first = cover[(size_t)t][0];
    EXPECT(first == 1);
    for (int32_t v : cover[(size_t)t]) EXPECT(v == 0 || v == 1);
  }
  size_t ws = 0;
  EXPECT(sk_workspace_size(ps.data(), (int32_t)ps.size(), &c, &ws) == SK_OK);
  EXPECT((int64_t)ws == info.workspace_bytes);
}

int main() {
  register_menu();
  for (int code = -8; code <= 0; ++code) EXPECT(sk_status_string(code) != nullptr);
  int32_t n = 0;
  EXPECT(sk_supported_tiles(SK_F8E4M3, nullptr, 0, &n) == SK_OK && n == 4);
  std::vector<int32_t> tl(3 * (size_t)n);
  EXPECT(sk_supported_tiles(SK_F8E4M3, tl.data(), n, &n) == SK_OK);
  EXPECT(sk_supported_tiles(SK_F8E4M3, tl.data(), n - 1, &n) == SK_ERR_CAPACITY);

  const int bms[] = {256, 256, 128};
  const int bns[] = {256, 128, 128};
  for (int iter = 0; iter < 400; ++iter) {
    const int dt = (int)uniform(0, 3);
    const int ti = dt == SK_F32 ? 2 : (int)uniform(0, 2);
    const int mode = (int)uniform(0, 3);
    const int cus = (int)uniform(1, 256);
    const int np = iter % 5 == 0 ? (int)uniform(2, 9) : 1;
    std::vector<sk_problem> ps;
    const int la = (int)uniform(0, 1), lb = (int)uniform(0, 1);
    for (int i = 0; i < np; ++i)
      ps.push_back(problem(uniform(0, 3000), uniform(0, 3000), uniform(0, 9000), dt, la, lb));
    sk_config c = config(dt, bms[ti], bns[ti], cus, mode);
    c.group_m = (int)uniform(-1, 9);
    c.min_iters = (int)uniform(0, 3);
    c.wg_per_cu = (int)uniform(0, 2);
    if (iter % 7 == 0) c.dp_tiles = uniform(0, 40);
    check_schedule(ps, c);
  }

  EXPECT(planned >= 300);

  // invalid arguments never read past what they describe
  sk_problem p = problem(100, 100, 100, SK_BF16, SK_ROW_MAJOR, SK_COL_MAJOR);
  sk_config c = config(SK_BF16, 128, 128, 8, SK_MODE_SK);
  sk_plan_info info;
  EXPECT(sk_plan(nullptr, 1, &c, &info) == SK_ERR_INVALID_ARG);
  EXPECT(sk_plan(&p, 0, &c, &info) == SK_ERR_INVALID_ARG);
  EXPECT(sk_plan(&p, 1, nullptr, &info) == SK_ERR_INVALID_ARG);
  EXPECT(sk_plan(&p, 1, &c, nullptr) == SK_ERR_INVALID_ARG);
  sk_problem bad = p;
  bad.lda = 99;
  EXPECT(sk_plan(&bad, 1, &c, &info) == SK_ERR_INVALID_ARG);
  bad = p;
  bad.M = -1;
  EXPECT(sk_plan(&bad, 1, &c, &info) == SK_ERR_INVALID_ARG);
  bad = p;
  bad.dtype_ab = 7;
  EXPECT(sk_plan(&bad, 1, &c, &info) == SK_ERR_UNSUPPORTED);
  sk_config cb = c;
  cb.block_k = 32;
  EXPECT(sk_plan(&p, 1, &cb, &info) == SK_ERR_UNSUPPORTED);
  cb = c;
  cb.mode = 9;
  EXPECT(sk_plan(&p, 1, &cb, &info) == SK_ERR_INVALID_ARG);
  size_t dsz = 0;
  EXPECT(sk_grouped_desc_size(0, &dsz) == SK_ERR_INVALID_ARG);
  EXPECT(sk_grouped_desc_size(48, &dsz) == SK_OK && dsz > 0);
  // sk_transpose: argument checks (before any launch), extreme sizes in the
  // overlap test's address arithmetic
  void* pa = (void*)(uintptr_t)0x100000;
  void* pb = (void*)(uintptr_t)0x900000;
  EXPECT(sk_transpose(pa, 4, 5, 5, pb, 4, 3, nullptr) == SK_ERR_INVALID_ARG);
  EXPECT(sk_transpose(pa, 4, 5, 4, pb, 4, 2, nullptr) == SK_ERR_INVALID_ARG);
  EXPECT(sk_transpose(pa, 4, 5, 5, pb, 3, 2, nullptr) == SK_ERR_INVALID_ARG);
  EXPECT(sk_transpose(nullptr, 4, 5, 5, pb, 4, 2, nullptr) == SK_ERR_INVALID_ARG);
  EXPECT(sk_transpose(pa, 4, 5, 5, (char*)pa + 8, 4, 2, nullptr) == SK_ERR_INVALID_ARG);
  EXPECT(sk_transpose(pa, (int64_t)1 << 20, (int64_t)1 << 20, (int64_t)1 << 20, pa, (int64_t)1 << 20,
                      4, nullptr) == SK_ERR_INVALID_ARG);
  EXPECT(sk_transpose(pa, (int64_t)1 << 40, 3, (int64_t)1 << 40, pb, (int64_t)1 << 40, 1,
                      nullptr) == SK_ERR_INVALID_ARG);
  EXPECT(sk_transpose(nullptr, 0, 9, 9, nullptr, 1, 1, nullptr) == SK_OK);

  if (failures) {
    fprintf(stderr, "%d expectation(s) failed\n", failures);
    return 1;
  }
  printf("host ABI driver: ok (%d problem sets planned and scheduled)\n", planned);
  return 0;
}
