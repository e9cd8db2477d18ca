// C ABI of the Stream-K GEMM library: validation, planning, schedule
// enumeration and kernel launches.  See include/streamk.h for the contract of
// every entry point.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/streamk.h"
#include "sk_cost.hpp"
#include "sk_params.hpp"
#include "sk_registry.hpp"
#include "sk_sched.hpp"

namespace sk {

static std::vector<KernelEntry>& registry() {
  static std::vector<KernelEntry> r;
  return r;
}

bool register_kernel(const KernelEntry& e) {
  registry().push_back(e);
  return true;
}

static const KernelEntry* find_kernel(int dt, int la, int lb, int bm, int bn) {
  for (const KernelEntry& e : registry())
    if (e.dt == dt && e.la == la && e.lb == lb && e.bm == bm && e.bn == bn) return &e;
  return nullptr;
}

static bool tile_built(int dt, int bm, int bn) {
  for (const KernelEntry& e : registry())
    if (e.dt == dt && e.bm == bm && e.bn == bn) return true;
  return false;
}

// Default fixup-wait bound: polls of ~128 clocks of s_sleep plus an L2 round
// trip each, a few seconds in all.
constexpr int64_t kDefaultSpinLimit = int64_t(1) << 22;
constexpr int64_t kMaxIndex = (int64_t(1) << 31) - 1;

struct Plan {
  int64_t T = 0, S = 0, W = 0, g = 0, q = 0, rho = 0, max_iters = 0;
  int64_t ws_bytes = 0;
  int32_t group_m = 0;           // resolved tile order
  bool dp_grid = false;          // one workgroup per tile, no fixup
  double pred_us = 0.0;          // launch-time model: this launch
  double pred_dp_us = 0.0;       // ... and the data-parallel grid of the problems
  std::vector<ProbDesc> descs;   // operand pointers left null by plan_problems
  std::vector<int32_t> order;    // descs[i] describes caller problem order[i]
};

// Per-device facts are queried once and cached (these runtime queries cost
// microseconds, more than a small GEMM).
static std::mutex g_cache_mu;
static std::map<int, int> g_cus;                                   // device -> CUs
static std::map<std::pair<int, const void*>, int> g_resident;      // (device, kernel) -> WGs/CU

static sk_status device_cus(int32_t* n) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SK_ERR_HIP;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cus.find(dev);
    if (it != g_cus.end()) {
      *n = it->second;
      return SK_OK;
    }
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return SK_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cus[dev] = v;
  *n = v;
  return SK_OK;
}

// Workgroups of kernel `ke` that fit on one CU at once.
static sk_status resident_per_cu(const KernelEntry* ke, int* per_cu) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SK_ERR_HIP;
  const auto key = std::make_pair(dev, ke->fn);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_resident.find(key);
    if (it != g_resident.end()) {
      *per_cu = it->second;
      return SK_OK;
    }
  }
  int v = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, ke->fn, ke->nt, 0) != hipSuccess)
    return SK_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_resident[key] = v;
  *per_cu = v;
  return SK_OK;
}

static sk_status check_problem(const sk_problem& p) {
  if (p.M < 0 || p.N < 0 || p.K < 0) return SK_ERR_INVALID_ARG;
  if (p.M > kMaxIndex || p.N > kMaxIndex || p.K > kMaxIndex) return SK_ERR_UNSUPPORTED;
  if (p.dtype_ab < 0 || p.dtype_ab > 9) return SK_ERR_UNSUPPORTED;
  if (p.dtype_c < 0 || p.dtype_c > 2) return SK_ERR_UNSUPPORTED;
  if ((p.layout_a != SK_ROW_MAJOR && p.layout_a != SK_COL_MAJOR) ||
      (p.layout_b != SK_ROW_MAJOR && p.layout_b != SK_COL_MAJOR))
    return SK_ERR_INVALID_ARG;
  const int64_t need_a = p.layout_a == SK_ROW_MAJOR ? p.K : p.M;
  const int64_t need_b = p.layout_b == SK_ROW_MAJOR ? p.N : p.K;
  if (p.lda < std::max<int64_t>(1, need_a)) return SK_ERR_INVALID_ARG;
  if (p.ldb < std::max<int64_t>(1, need_b)) return SK_ERR_INVALID_ARG;
  if (p.ldc < std::max<int64_t>(1, p.N)) return SK_ERR_INVALID_ARG;
  if (p.activation < SK_ACT_NONE || p.activation > SK_ACT_SILU || p.reserved != 0)
    return SK_ERR_INVALID_ARG;
  if (((uintptr_t)p.bias & 3) != 0) return SK_ERR_INVALID_ARG;
  return SK_OK;
}

// Resolves g and checks the config against the tile menu.
static sk_status resolve_config(const sk_config* cfg, int32_t dtype_ab, int64_t* g_out,
                                int64_t* cus_out) {
  if (cfg == nullptr) return SK_ERR_INVALID_ARG;
  if (cfg->mode < 0 || cfg->mode > 3) return SK_ERR_INVALID_ARG;
  if (cfg->block_k != k_per_iter(dtype_ab)) return SK_ERR_UNSUPPORTED;
  if (!tile_built(dtype_ab, cfg->block_m, cfg->block_n)) return SK_ERR_UNSUPPORTED;
  if (cfg->group_m < -1 || cfg->wg_per_cu < 0 || cfg->num_cu < 0) return SK_ERR_INVALID_ARG;
  if (cfg->dp_tiles < -1) return SK_ERR_INVALID_ARG;
  if (cfg->spin_limit < 0 || cfg->min_iters < 0) return SK_ERR_INVALID_ARG;
  int32_t cus = cfg->num_cu;
  if (cus == 0) {
    sk_status st = device_cus(&cus);
    if (st != SK_OK) return st;
  }
  const int64_t wpc = cfg->wg_per_cu == 0 ? 1 : cfg->wg_per_cu;
  *g_out = (int64_t)cus * wpc;
  *cus_out = cus;
  return SK_OK;
}

// The kernels address a tile's operands and output with 32-bit byte offsets
// from the tile's first element (buffer instructions); every offset a tile
// can form must stay below 2^31.
static bool offsets_fit(const sk_problem& p, int64_t bm, int64_t bn) {
  const int64_t ec = p.dtype_c == SK_F32 ? 4 : 2;
  const int64_t rm = std::min<int64_t>(std::max<int64_t>(p.M, 1), bm);
  const int64_t rn = std::min<int64_t>(std::max<int64_t>(p.N, 1), bn);
  const int64_t k = std::max<int64_t>(p.K, 1);
  auto bytes = [&](int64_t n) { return elems_to_bytes(p.dtype_ab, n); };
  const int64_t span_a = p.layout_a == SK_ROW_MAJOR ? bytes((rm - 1) * p.lda + k)
                                                    : bytes((k - 1) * p.lda + bm);
  const int64_t span_b = p.layout_b == SK_COL_MAJOR ? bytes((rn - 1) * p.ldb + k)
                                                    : bytes((k - 1) * p.ldb + bn);
  const int64_t span_c = ((rm - 1) * p.ldc + bn) * ec;
  return span_a <= kMaxIndex && span_b <= kMaxIndex && span_c <= kMaxIndex;
}

// Grid floor: with m = min_iters > 1 a Stream-K launch of a small problem
// uses max(1, W_all / m) < g workgroups.  Automatic m (min_iters = 0): one
// partial tile costs about f = fixup_iters(BM, BN, BK) MAC iterations of the
// finisher's time, so a tile of I iterations split into c pieces takes
// about I/c + f(c-1) iteration times; c is the largest integer >= 1 with
// f c^2 <= I_mean and m = ceil(I_mean/c).
static int64_t grid_floor(int64_t g, int64_t T, int64_t W_all, int32_t min_iters, int64_t f) {
  if (T == 0 || W_all == 0) return g;
  int64_t m = min_iters;
  if (m == 0) {
    const int64_t i_mean = cdiv(W_all, T);
    int64_t c = 1;
    while (f * (c + 1) * (c + 1) <= i_mean) ++c;
    m = cdiv(i_mean, c);
  }
  if (m <= 1) return g;
  return std::min<int64_t>(g, std::max<int64_t>(1, W_all / m));
}

// Automatic tile order (group_m = -1).  Under the balanced split workgroup x
// starts at iteration x*q, i.e. at k-phase x*q mod I of its first tile, and
// workgroups x and x + I/gcd(q, I) start at the same phase, so they walk K
// in step; their first tiles lie D = q/gcd(q, I) apart.  In bands of G
// tile rows walked down the band first, tiles t and t + D sit side by side
// in one tile row whenever G divides D, so such workgroups read the same A
// panel slices at the same time and share them in L2, as the workgroups of
// a data-parallel wave do.  G is the largest divisor of D not above the
// tile-row count tm.  Without Stream-K tiles: bands of 8 rows (the
// data-parallel wave's tiles on one XCD then form a compact block).
static int64_t gcd64(int64_t a, int64_t b) {
  while (b != 0) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

static int32_t resolve_group_m(int32_t group_m, const Plan& P) {
  if (group_m >= 0) return group_m;
  if (P.S > 0 && P.q > 0) {
    for (const ProbDesc& d : P.descs) {
      if ((int64_t)d.tm * d.tn == 0) continue;
      const int64_t D = P.q / gcd64(P.q, d.I);
      int64_t G = std::min<int64_t>(D, d.tm);
      while (D % G != 0) --G;
      return (int32_t)G;
    }
  }
  return 8;
}

// Iteration space, even split, workspace and tile order of a plan whose
// problems, tiles, g and S are set.
static sk_status finish_plan(Plan* P, const sk_config* cfg, int64_t bm, int64_t bn) {
  // Stream-K iteration offsets (problem-major, so J is monotone in p).
  int64_t J = 0;
  for (ProbDesc& d : P->descs) {
    const int64_t ti = (int64_t)d.tm * d.tn;
    d.iter_start = J;
    const int64_t sk_tiles = std::max<int64_t>(0, std::min<int64_t>(ti, P->S - d.tile_start));
    J += sk_tiles * d.I;
  }
  if (J > kMaxIndex) return SK_ERR_UNSUPPORTED;
  P->W = J;
  P->q = P->rho = 0;
  if (!P->dp_grid && P->g > 0) {
    P->q = P->W / P->g;
    P->rho = P->W % P->g;
  }
  P->ws_bytes = P->dp_grid ? 0 : ws_bytes(P->S, P->S > 0 ? P->g : 0, bm, bn);
  // the fixup addresses all partial slots with 32-bit buffer offsets, and
  // the workspace holds one token per persistent workgroup
  if (P->S > 0 && P->g * bm * bn * 4 > kMaxIndex) return SK_ERR_UNSUPPORTED;
  if (!P->dp_grid && P->g > kMaxWG) return SK_ERR_UNSUPPORTED;
  P->group_m = resolve_group_m(cfg->group_m, *P);
  return SK_OK;
}

static double predict_us(const Plan& P, const CostRow& c, int64_t cus);

// Tile counts, split point, iteration space and per-problem offsets.  With
// `predict`, the launch-time model's predictions of the resolved launch and
// of the data-parallel grid are filled in (SK_MODE_AUTO always uses them).
static sk_status plan_problems(const sk_problem* probs, int32_t n, const sk_config* cfg,
                               Plan* out, bool predict = false) {
  if (probs == nullptr || n <= 0) return SK_ERR_INVALID_ARG;
  for (int32_t i = 0; i < n; ++i) {
    sk_status st = check_problem(probs[i]);
    if (st != SK_OK) return st;
    if (probs[i].dtype_ab != probs[0].dtype_ab || probs[i].dtype_c != probs[0].dtype_c ||
        probs[i].layout_a != probs[0].layout_a || probs[i].layout_b != probs[0].layout_b)
      return SK_ERR_UNSUPPORTED;
  }
  int64_t g = 0, cus = 0;
  sk_status st = resolve_config(cfg, probs[0].dtype_ab, &g, &cus);
  if (st != SK_OK) return st;
  const int64_t bm = cfg->block_m, bn = cfg->block_n, bk = cfg->block_k;
  for (int32_t i = 0; i < n; ++i)
    if (!offsets_fit(probs[i], bm, bn)) return SK_ERR_UNSUPPORTED;

  // Global tile order of a grouped persistent launch: problems by MAC
  // iterations per tile, most first, ties in the caller's order.  Whole
  // tiles left to the persistent round-robin then alternate evenly between
  // the workgroups (longest-first list scheduling); an even Stream-K split
  // does not depend on the order.  The data-parallel grid keeps the
  // caller's order (the hardware hands its workgroups out as CUs free up).
  Plan P;
  P.order.resize(n);
  for (int32_t i = 0; i < n; ++i) P.order[i] = i;
  auto iters_of = [&](int32_t i) { return std::max<int64_t>(1, cdiv(probs[i].K, bk)); };
  if (cfg->mode != SK_MODE_DP)
    std::stable_sort(P.order.begin(), P.order.end(),
                     [&](int32_t a, int32_t b) { return iters_of(a) > iters_of(b); });
  P.descs.resize(n);
  int64_t T = 0;
  for (int32_t i = 0; i < n; ++i) {
    const sk_problem& p = probs[P.order[i]];
    ProbDesc& d = P.descs[i];
    memset(&d, 0, sizeof(d));
    d.M = p.M; d.N = p.N; d.K = p.K;
    d.lda = p.lda; d.ldb = p.ldb; d.ldc = p.ldc;
    d.alpha_s = p.alpha * p.scale_a * p.scale_b;
    d.beta = p.beta;
    d.tm = (int32_t)(p.M > 0 ? cdiv(p.M, bm) : 0);
    d.tn = (int32_t)(p.N > 0 ? cdiv(p.N, bn) : 0);
    d.I = (int32_t)std::max<int64_t>(1, cdiv(p.K, bk));
    d.user_index = P.order[i];
    d.act = p.activation;
    d.bias = p.bias;
    d.tile_start = T;
    T += (int64_t)d.tm * d.tn;
    P.max_iters = std::max<int64_t>(P.max_iters, d.I);
    if (p.dtype_ab == SK_MXF4E2M1 || p.dtype_ab == SK_MXF6E2M3 || p.dtype_ab == SK_MXF6E3M2) {
      // the kernels see MXFP4 and MXFP6 operands as bytes
      d.K = elems_to_bytes(p.dtype_ab, d.K);
      d.lda = elems_to_bytes(p.dtype_ab, d.lda);
      d.ldb = elems_to_bytes(p.dtype_ab, d.ldb);
    }
  }
  if (T > kMaxIndex) return SK_ERR_UNSUPPORTED;
  P.T = T;
  if (cfg->mode == SK_MODE_DP) {
    P.S = 0;
    P.g = T;
    P.dp_grid = true;
  } else {
    int64_t W_all = 0;
    for (int32_t i = 0; i < n; ++i) W_all += (int64_t)P.descs[i].tm * P.descs[i].tn * P.descs[i].I;
    P.g = grid_floor(g, T, W_all, cfg->min_iters, fixup_iters(bm, bn, bk));
    P.S = split_point(T, P.g, cfg->mode, cfg->dp_tiles);
  }
  st = finish_plan(&P, cfg, bm, bn);
  if (st != SK_OK) return st;

  const bool is_auto = cfg->mode == SK_MODE_AUTO;
  if (is_auto || predict) {
    const CostRow& c = *cost_row(probs[0].dtype_ab, (int32_t)bm, (int32_t)bn);
    // the data-parallel grid of the same problems (one workgroup per tile)
    Plan D = P;
    D.S = 0;
    D.g = T;
    D.dp_grid = true;
    st = finish_plan(&D, cfg, bm, bn);
    if (st != SK_OK) return st;
    P.pred_us = predict_us(P, c, cus);
    P.pred_dp_us = predict_us(D, c, cus);
    if (is_auto && P.S > 0) {
      // SK_MODE_AUTO: split tiles only if the model predicts the launch
      // without splits (the data-parallel grid for one problem, whole tiles
      // on the persistent workgroups for several) to be auto_margin times
      // slower
      Plan A = P;
      if (n == 1) {
        A = D;
        A.pred_us = P.pred_dp_us;
      } else {
        A.S = 0;
        st = finish_plan(&A, cfg, bm, bn);
        if (st != SK_OK) return st;
        A.pred_us = predict_us(A, c, cus);
      }
      A.pred_dp_us = P.pred_dp_us;
      if (!(A.pred_us > auto_margin(probs[0].dtype_ab) * P.pred_us)) P = std::move(A);
    } else if (is_auto && P.S == 0 && n == 1) {
      // nothing to split on one problem: the data-parallel grid itself (the
      // hardware hands out tiles as workgroups finish, which beats a fixed
      // round-robin of whole tiles over persistent workgroups)
      const double dp = P.pred_dp_us;
      P = std::move(D);
      P.pred_us = P.pred_dp_us = dp;
    }
  }
  *out = std::move(P);
  return SK_OK;
}

// Host mirror of the kernel's tile lookups.
static int32_t host_find_problem(const Plan& P, int64_t key, bool by_iter) {
  int32_t lo = 0, hi = (int32_t)P.descs.size() - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    int64_t s = by_iter ? P.descs[mid].iter_start : P.descs[mid].tile_start;
    if (s <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

static void host_segments(const Plan& P, const sk_config* cfg, std::vector<sk_segment>* out) {
  auto emit = [&](int64_t x, int32_t p, int64_t t, int64_t u, int kb, int ke, int role,
                  int npeers) {
    const ProbDesc& d = P.descs[p];
    sk_segment s;
    s.wg = (int32_t)x;
    s.problem = P.order[p];
    s.tile = (int32_t)t;
    tile_coords(u, d.tm, d.tn, P.group_m, &s.tile_m, &s.tile_n);
    s.k_begin = kb;
    s.k_end = ke;
    s.role = role;
    s.npeers = npeers;
    out->push_back(s);
  };
  if (P.dp_grid) {
    for (int64_t t = 0; t < P.T; ++t) {
      int32_t p = host_find_problem(P, t, false);
      emit(t, p, t, t - P.descs[p].tile_start, 0, P.descs[p].I, SK_ROLE_DP, 0);
    }
    return;
  }
  for (int64_t x = 0; x < P.g; ++x) {
    const int64_t s = range_begin(x, P.q, P.rho);
    const int64_t e = s + P.q + (x < P.rho ? 1 : 0);
    int64_t it = s;
    while (it < e) {
      int32_t p = host_find_problem(P, it, true);
      const ProbDesc& d = P.descs[p];
      int64_t u = (it - d.iter_start) / d.I;
      int64_t J = d.iter_start + u * d.I;
      int kb = (int)(it - J);
      int ke = (int)(std::min(e, J + d.I) - J);
      int role, npeers = 0;
      if (kb > 0) role = SK_ROLE_PARTIAL;
      else if (ke == d.I) role = SK_ROLE_FULL;
      else {
        role = SK_ROLE_FINISH;
        npeers = (int)(iter_owner(J + d.I - 1, P.q, P.rho) - x);
      }
      emit(x, p, d.tile_start + u, u, kb, ke, role, npeers);
      it = J + ke;
    }
    for (int64_t r = 0;; ++r) {          // position x, or g-1-x in odd rounds
      const int64_t t = P.S + r * P.g + ((r & 1) ? P.g - 1 - x : x);
      if (t >= P.T) break;
      int32_t p = host_find_problem(P, t, false);
      emit(x, p, t, t - P.descs[p].tile_start, 0, P.descs[p].I, SK_ROLE_DP, 0);
    }
  }
}

// Predicted time in microseconds of the launch P under the launch-time
// model (sk_cost.hpp): every workgroup's segments walked as the kernel walks
// them; the launch ends with its slowest workgroup.
static double predict_us(const Plan& P, const CostRow& c, int64_t cus) {
  if (P.T == 0) return 0.0;
  cus = std::max<int64_t>(1, cus);
  auto tile_cost = [&](const ProbDesc& d, double it) {
    return c.t_tile + d.I * it + (d.beta != 0.f ? c.t_cin : 0.0);
  };
  if (P.dp_grid) {
    const double it = iter_time(c, std::min<int64_t>(P.T, cus));
    if (P.descs.size() == 1) return c.t_launch + (double)cdiv(P.T, cus) * tile_cost(P.descs[0], it);
    double sum = 0.0, mx = 0.0;   // several problems: work over the CUs, or the longest tile
    for (const ProbDesc& d : P.descs) {
      const int64_t tiles = (int64_t)d.tm * d.tn;
      if (tiles == 0) continue;
      const double tc = tile_cost(d, it);
      sum += (double)tiles * tc;
      mx = std::max(mx, tc);
    }
    return c.t_launch + std::max(mx, sum / (double)cus);
  }
  const int64_t g = P.g;
  const double it = iter_time(c, std::min<int64_t>(g, cus));
  const double it_sk = it * (1.0 + c.l2);
  auto range = [&](int64_t x, int64_t* s, int64_t* e) {
    *s = range_begin(x, P.q, P.rho);
    *e = *s + P.q + (x < P.rho ? 1 : 0);
  };
  // a PARTIAL segment is its workgroup's first: when its partial is published
  std::vector<double> ready((size_t)g, 0.0);
  for (int64_t x = 0; x < g; ++x) {
    int64_t s, e;
    range(x, &s, &e);
    if (s >= e) continue;
    const ProbDesc& d = P.descs[host_find_problem(P, s, true)];
    const int64_t J = d.iter_start + (s - d.iter_start) / d.I * d.I;
    if (s > J)
      ready[(size_t)x] = c.t_tile + (double)(std::min(e, J + d.I) - s) * it_sk + c.t_store;
  }
  double worst = 0.0;
  for (int64_t x = 0; x < g; ++x) {
    int64_t s, e;
    range(x, &s, &e);
    double t = 0.0;
    for (int64_t i = s; i < e;) {
      const ProbDesc& d = P.descs[host_find_problem(P, i, true)];
      const int64_t J = d.iter_start + (i - d.iter_start) / d.I * d.I;
      const int64_t kb = i - J, ke = std::min(e, J + d.I) - J;
      t += c.t_tile + (double)(ke - kb) * it_sk;
      if (kb > 0) {
        t += c.t_store;                                   // PARTIAL
      } else {
        if (ke < d.I) {                                   // FINISH
          const int64_t last = iter_owner(J + d.I - 1, P.q, P.rho);
          for (int64_t y = x + 1; y <= last; ++y) t = std::max(t, ready[(size_t)y]);
          t += (double)(last - x) * c.t_peer;
        }
        if (d.beta != 0.f) t += c.t_cin;
      }
      i = J + ke;
    }
    for (int64_t r = 0;; ++r) {          // whole tiles: position x, or g-1-x in odd rounds
      const int64_t tt = P.S + r * g + ((r & 1) ? g - 1 - x : x);
      if (tt >= P.T) break;
      t += tile_cost(P.descs[host_find_problem(P, tt, false)], it);
    }
    worst = std::max(worst, t);
  }
  return c.t_launch + worst;
}

__global__ void fill_zero_kernel(uint32_t* p, int64_t words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

static sk_status launch(const Plan& P, const sk_config* cfg, int32_t dt, int32_t la, int32_t lb,
                        int32_t dtype_c, const ProbDesc* single, const ProbDesc* dev_group,
                        int32_t nprobs, void* ws, size_t ws_len, const sk_debug* dbg,
                        hipStream_t stream) {
  const KernelEntry* ke = find_kernel(dt, la, lb, cfg->block_m, cfg->block_n);
  if (ke == nullptr) return SK_ERR_UNSUPPORTED;
  if (P.T == 0) return SK_OK;
  if (!P.dp_grid) {
    if (ws == nullptr || (int64_t)ws_len < P.ws_bytes) return SK_ERR_WORKSPACE;
    int32_t cus = 0;
    sk_status st = device_cus(&cus);
    if (st != SK_OK) return st;
    if (cfg->num_cu > cus) return SK_ERR_INVALID_ARG;
    int per_cu = 0;
    st = resident_per_cu(ke, &per_cu);
    if (st != SK_OK) return st;
    // Stream-K workgroups wait for each other: all must be resident at once.
    if (P.g > (int64_t)cus * per_cu) return SK_ERR_OCCUPANCY;
  }
  KParams kp;
  memset(&kp, 0, sizeof(kp));
  if (single) kp.prob = *single;
  kp.group = dev_group;
  kp.nprobs = nprobs;
  kp.dtype_c = dtype_c;
  kp.T = P.T; kp.S = P.S; kp.W = P.W; kp.g = P.g; kp.q = P.q; kp.rho = P.rho;
  kp.group_m = P.group_m;
  kp.xcd_remap = cfg->xcd_remap;
  kp.dp_grid = P.dp_grid ? 1 : 0;
  kp.spin_limit = cfg->spin_limit > 0 ? cfg->spin_limit : kDefaultSpinLimit;
  if (ws) {
    char* w = (char*)ws;
    kp.err = (int32_t*)w;
    kp.epoch = (uint32_t*)(w + 4);
    kp.done = (uint32_t*)(w + 8);
    kp.tokens = (uint32_t*)(w + kTokensOffset);
    kp.slots = (float*)(w + kSlotsOffset);
  }
  if (dbg) {
    kp.trace = dbg->trace;
    kp.trace_cap = dbg->trace_capacity;
    kp.trace_count = dbg->trace_count;
    kp.cover = dbg->cover;
    kp.cover_stride = dbg->cover_stride;
    kp.partial_delay = dbg->partial_delay;
    kp.reverse_ids = dbg->reverse_ids;
    if (kp.trace && !kp.trace_count) return SK_ERR_INVALID_ARG;
    if (kp.cover && kp.cover_stride < P.max_iters) return SK_ERR_INVALID_ARG;
  }
  void* args[] = {&kp};
  const int64_t grid = P.dp_grid ? P.T : P.g;
  if (hipLaunchKernel(ke->fn, dim3((unsigned)grid), dim3((unsigned)ke->nt), args, 0, stream) != hipSuccess)
    return SK_ERR_HIP;
  return SK_OK;
}

// MXFP8 block scales of one problem (sk_gemm_mx).
struct MxScales {
  const void* sA;
  int64_t ldsa;
  const void* sB;
  int64_t ldsb;
};

// An MXFP8 problem and its operands and block scales: the kernels are built
// for K-contiguous operands, whole 128-element iterations and 16-byte loads,
// and read the scales as 4-byte words, 4 per iteration.
static sk_status check_mx(const sk_problem& p, const void* A, const void* B, const MxScales& mx) {
  if (p.layout_a != SK_ROW_MAJOR || p.layout_b != SK_COL_MAJOR ||
      p.K % k_per_iter(p.dtype_ab) != 0)
    return SK_ERR_UNSUPPORTED;
  if (p.M == 0 || p.N == 0 || p.K == 0) return SK_OK;
  // rows of a multiple of 16 bytes (MXFP4: 32 elements)
  const int64_t row_align = p.dtype_ab == SK_MXF4E2M1 ? 32
                            : (p.dtype_ab == SK_MXF6E2M3 || p.dtype_ab == SK_MXF6E3M2) ? 64 : 16;
  if (!aligned16(A) || !aligned16(B) || p.lda % row_align != 0 || p.ldb % row_align != 0)
    return SK_ERR_UNSUPPORTED;
  if (mx.sA == nullptr || mx.sB == nullptr || ((uintptr_t)mx.sA & 3) != 0 ||
      ((uintptr_t)mx.sB & 3) != 0 || mx.ldsa % 4 != 0 || mx.ldsb % 4 != 0 ||
      mx.ldsa < p.K / 32 || mx.ldsb < p.K / 32)
    return SK_ERR_INVALID_ARG;
  if ((p.M - 1) * mx.ldsa + p.K / 32 > kMaxIndex || (p.N - 1) * mx.ldsb + p.K / 32 > kMaxIndex)
    return SK_ERR_UNSUPPORTED;
  return SK_OK;
}

static sk_status gemm_common(const sk_problem* p, const void* A, const void* B, const void* Cin,
                             void* Cout, void* ws, size_t ws_bytes_, const sk_config* cfg,
                             const sk_debug* dbg, void* stream, const MxScales* mx = nullptr) {
  if (p == nullptr) return SK_ERR_INVALID_ARG;
  if (p->dtype_ab < 0 || p->dtype_ab > SK_F8E5M2) return SK_ERR_UNSUPPORTED;
  // MX inputs need their block scales (sk_gemm_mx); others take none
  const bool is_mx = p->dtype_ab >= SK_MXF8E4M3 && p->dtype_ab <= SK_MXF8E5M2;
  if (is_mx != (mx != nullptr)) return SK_ERR_INVALID_ARG;
  Plan P;
  sk_status st = plan_problems(p, 1, cfg, &P);
  if (st != SK_OK) return st;
  if (mx) {
    st = check_mx(*p, A, B, *mx);
    if (st != SK_OK) return st;
  }
  if (p->M == 0 || p->N == 0) return SK_OK;
  if (Cout == nullptr) return SK_ERR_INVALID_ARG;
  if (p->K > 0 && (A == nullptr || B == nullptr)) return SK_ERR_INVALID_ARG;
  if (p->beta != 0.f && Cin == nullptr) return SK_ERR_INVALID_ARG;
  ProbDesc& d = P.descs[0];
  d.A = A; d.B = B; d.Cin = Cin; d.Cout = Cout;
  if (mx) {
    d.sA = mx->sA; d.sB = mx->sB;
    d.ldsa = mx->ldsa; d.ldsb = mx->ldsb;
  }
  d.aligned = aligned16(A) && aligned16(B) && elems_to_bytes(p->dtype_ab, p->lda) % 16 == 0 &&
              elems_to_bytes(p->dtype_ab, p->ldb) % 16 == 0;
  return launch(P, cfg, p->dtype_ab, p->layout_a, p->layout_b, p->dtype_c, &d, nullptr, 1, ws,
                ws_bytes_, dbg, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Workspace of sk_gemm_noalloc: a file-scope device array, one copy per GPU,
// held until the process ends.  Its size covers every tile of the menu up to
// 256x256 on 256 persistent workgroups.  In host code `scratch` names a
// host-side stand-in, never the device array: the device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr int64_t kScratchBytes = kSlotsOffset + (int64_t)256 * 256 * 256 * 4;
static_assert(kScratchBytes == SK_NOALLOC_SCRATCH_BYTES, "scratch size in the header");
static_assert(sizeof(sk_problem) == 96, "sk_problem layout of the header");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch;   // device -> address of its scratch

// Address of the current device's scratch.  With setup, the first call on a
// device looks the address up and clears the header and tokens (error word,
// epoch, done counter, arrival tokens) with a fill kernel on `stream`;
// without, a device not yet set up yields nullptr.
static sk_status device_scratch(hipStream_t stream, bool setup, void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SK_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) {
    *out = it->second;
    return SK_OK;
  }
  *out = nullptr;
  if (!setup) return SK_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
    return SK_ERR_HIP;
  const int64_t words = kSlotsOffset / 4;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0,
                     stream, (uint32_t*)ptr, words);
  if (hipGetLastError() != hipSuccess) return SK_ERR_HIP;
  g_scratch[dev] = ptr;
  *out = ptr;
  return SK_OK;
}

}  // namespace sk

using namespace sk;

extern "C" {

const char* sk_status_string(int32_t status) {
  switch (status) {
    case SK_OK: return "success";
    case SK_ERR_INVALID_ARG: return "invalid argument";
    case SK_ERR_UNSUPPORTED: return "unsupported dtype, layout or tile";
    case SK_ERR_WORKSPACE: return "workspace missing or too small";
    case SK_ERR_OCCUPANCY: return "more persistent workgroups than can be resident";
    case SK_ERR_HIP: return "HIP runtime error";
    case SK_ERR_CAPACITY: return "output array too small";
    case SK_ERR_DEVICE_TIMEOUT: return "a fixup wait on the device timed out";
    default: return "unknown status";
  }
}

sk_status sk_device_query(int32_t* num_cu, int32_t* max_wg_per_cu, const sk_config* cfg,
                          int32_t dtype_ab) {
  int32_t cus = 0;
  sk_status st = device_cus(&cus);
  if (st != SK_OK) return st;
  if (num_cu) *num_cu = cus;
  if (max_wg_per_cu) {
    if (cfg == nullptr) return SK_ERR_INVALID_ARG;
    const KernelEntry* ke = nullptr;
    for (int la = 0; la < 2 && !ke; ++la)
      for (int lb = 0; lb < 2 && !ke; ++lb)
        ke = find_kernel(dtype_ab, la, lb, cfg->block_m, cfg->block_n);
    if (ke == nullptr) return SK_ERR_UNSUPPORTED;
    int per_cu = 0;
    st = resident_per_cu(ke, &per_cu);
    if (st != SK_OK) return st;
    *max_wg_per_cu = per_cu;
  }
  return SK_OK;
}

sk_status sk_supported_tiles(int32_t dtype_ab, int32_t* out, int32_t capacity, int32_t* count) {
  if (count == nullptr) return SK_ERR_INVALID_ARG;
  std::vector<std::pair<int, int>> tiles;
  for (const KernelEntry& e : registry())
    if (e.dt == dtype_ab &&
        std::find(tiles.begin(), tiles.end(), std::make_pair(e.bm, e.bn)) == tiles.end())
      tiles.push_back({e.bm, e.bn});
  std::sort(tiles.begin(), tiles.end());
  *count = (int32_t)tiles.size();
  if (out == nullptr) return SK_OK;
  if (capacity < (int32_t)tiles.size()) return SK_ERR_CAPACITY;
  for (size_t i = 0; i < tiles.size(); ++i) {
    out[3 * i] = tiles[i].first;
    out[3 * i + 1] = tiles[i].second;
    out[3 * i + 2] = k_per_iter(dtype_ab);
  }
  return SK_OK;
}

sk_status sk_plan(const sk_problem* probs, int32_t nprobs, const sk_config* cfg,
                  sk_plan_info* info) {
  if (info == nullptr) return SK_ERR_INVALID_ARG;
  Plan P;
  sk_status st = plan_problems(probs, nprobs, cfg, &P, true);
  if (st != SK_OK) return st;
  info->T = P.T; info->S = P.S; info->W = P.W; info->g = P.g;
  info->predicted_us = P.pred_us;
  info->predicted_dp_us = P.pred_dp_us;
  info->q = P.q; info->rho = P.rho;
  info->workspace_bytes = P.ws_bytes;
  info->max_iters = P.max_iters;
  info->group_m = P.group_m;
  info->dp_grid = P.dp_grid ? 1 : 0;
  return SK_OK;
}

sk_status sk_plan_order(const sk_problem* probs, int32_t nprobs, const sk_config* cfg,
                        int32_t* order) {
  if (order == nullptr) return SK_ERR_INVALID_ARG;
  Plan P;
  sk_status st = plan_problems(probs, nprobs, cfg, &P);
  if (st != SK_OK) return st;
  for (int32_t i = 0; i < nprobs; ++i) order[i] = P.order[i];
  return SK_OK;
}

sk_status sk_cost_model(int32_t dtype_ab, int32_t block_m, int32_t block_n, float* constants,
                        int32_t n) {
  if (constants == nullptr || n < 10 || dtype_ab < 0 || dtype_ab > 3) return SK_ERR_INVALID_ARG;
  const CostRow* c = cost_row(dtype_ab, block_m, block_n);
  if (c == nullptr) return SK_ERR_UNSUPPORTED;
  const float v[10] = {c->t_launch, c->t_tile, c->t_it_full, c->t_it_light, c->t_store,
                       c->t_peer, c->l2, c->t_cin, (float)auto_margin(dtype_ab),
                       (float)(c->bm * 65536 + c->bn)};
  for (int i = 0; i < 10; ++i) constants[i] = v[i];
  return SK_OK;
}

sk_status sk_schedule(const sk_problem* probs, int32_t nprobs, const sk_config* cfg,
                      sk_segment* out, int64_t capacity, int64_t* count) {
  if (count == nullptr) return SK_ERR_INVALID_ARG;
  Plan P;
  sk_status st = plan_problems(probs, nprobs, cfg, &P);
  if (st != SK_OK) return st;
  std::vector<sk_segment> segs;
  host_segments(P, cfg, &segs);
  *count = (int64_t)segs.size();
  if (out == nullptr) return SK_OK;
  if (capacity < (int64_t)segs.size()) return SK_ERR_CAPACITY;
  if (!segs.empty()) memcpy(out, segs.data(), segs.size() * sizeof(sk_segment));
  return SK_OK;
}

sk_status sk_workspace_size(const sk_problem* probs, int32_t nprobs, const sk_config* cfg,
                            size_t* bytes) {
  if (bytes == nullptr) return SK_ERR_INVALID_ARG;
  Plan P;
  sk_status st = plan_problems(probs, nprobs, cfg, &P);
  if (st != SK_OK) return st;
  *bytes = (size_t)P.ws_bytes;
  return SK_OK;
}

sk_status sk_workspace_init(void* workspace, size_t bytes, void* stream) {
  if (bytes == 0) return SK_OK;
  if (workspace == nullptr || !aligned16(workspace) || bytes % 4 != 0) return SK_ERR_INVALID_ARG;
  const int64_t words = (int64_t)(bytes / 4);
  const int64_t blocks = std::min<int64_t>(1024, (words + 255) / 256);
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     (hipStream_t)stream, (uint32_t*)workspace, words);
  return hipGetLastError() == hipSuccess ? SK_OK : SK_ERR_HIP;
}

sk_status sk_gemm(const sk_problem* p, const void* A, const void* B, const void* C_in,
                  void* C_out, void* workspace, size_t ws_bytes_, const sk_config* cfg,
                  void* stream) {
  return gemm_common(p, A, B, C_in, C_out, workspace, ws_bytes_, cfg, nullptr, stream);
}

sk_status sk_gemm_mx(const sk_problem* p, const void* A, const void* B, const void* scale_a,
                     int64_t ld_scale_a, const void* scale_b, int64_t ld_scale_b,
                     const void* C_in, void* C_out, void* workspace, size_t ws_bytes_,
                     const sk_config* cfg, void* stream) {
  const MxScales mx{scale_a, ld_scale_a, scale_b, ld_scale_b};
  return gemm_common(p, A, B, C_in, C_out, workspace, ws_bytes_, cfg, nullptr, stream, &mx);
}

sk_status sk_gemm_debug(const sk_problem* p, const void* A, const void* B, const void* C_in,
                        void* C_out, void* workspace, size_t ws_bytes_, const sk_config* cfg,
                        const sk_debug* dbg, void* stream) {
  if (dbg == nullptr) return SK_ERR_INVALID_ARG;
  return gemm_common(p, A, B, C_in, C_out, workspace, ws_bytes_, cfg, dbg, stream);
}

sk_status sk_gemm_noalloc(const sk_problem* p, const void* A, const void* B, const void* C_in,
                          void* C_out, const sk_config* cfg, void* stream) {
  void* ws = nullptr;
  sk_status st = device_scratch((hipStream_t)stream, true, &ws);
  if (st != SK_OK) return st;
  return gemm_common(p, A, B, C_in, C_out, ws, (size_t)kScratchBytes, cfg, nullptr, stream);
}

sk_status sk_check_device_error(void* workspace, size_t ws_bytes_, int32_t* code,
                                void* stream) {
  if (workspace == nullptr) {
    // the scratch of sk_gemm_noalloc on the current device
    sk_status st = device_scratch((hipStream_t)stream, false, &workspace);
    if (st != SK_OK) return st;
    if (workspace == nullptr) {
      if (code) *code = 0;
      return SK_OK;
    }
    ws_bytes_ = (size_t)kScratchBytes;
  }
  if (ws_bytes_ < 4) return SK_ERR_INVALID_ARG;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SK_ERR_HIP;
  int32_t v = 0;
  if (hipMemcpy(&v, workspace, 4, hipMemcpyDeviceToHost) != hipSuccess) return SK_ERR_HIP;
  if (v != 0) {
    int32_t z = 0;
    if (hipMemcpy(workspace, &z, 4, hipMemcpyHostToDevice) != hipSuccess) return SK_ERR_HIP;
  }
  if (code) *code = v;
  return v != 0 ? SK_ERR_DEVICE_TIMEOUT : SK_OK;
}

sk_status sk_grouped_desc_size(int32_t nprobs, size_t* bytes) {
  if (bytes == nullptr || nprobs <= 0) return SK_ERR_INVALID_ARG;
  *bytes = (size_t)nprobs * sizeof(ProbDesc);
  return SK_OK;
}

// sk_grouped_prepare and, with the block scales of every problem,
// sk_grouped_prepare_mx.
static sk_status grouped_prepare(const sk_problem* probs, const void* const* A,
                                 const void* const* B, const void* const* sA,
                                 const int64_t* ldsa, const void* const* sB,
                                 const int64_t* ldsb, const void* const* C_in,
                                 void* const* C_out, int32_t nprobs, const sk_config* cfg,
                                 void* dev_desc, size_t desc_bytes, sk_grouped_plan* plan,
                                 void* stream) {
  if (plan == nullptr || A == nullptr || B == nullptr || C_out == nullptr || dev_desc == nullptr)
    return SK_ERR_INVALID_ARG;
  Plan P;
  sk_status st = plan_problems(probs, nprobs, cfg, &P);
  if (st != SK_OK) return st;
  // MX problems need their block scales (sk_grouped_prepare_mx); others take none
  const bool mx = probs[0].dtype_ab >= SK_MXF8E4M3 && probs[0].dtype_ab <= SK_MXF8E5M2;
  if (mx != (sA != nullptr && ldsa != nullptr && sB != nullptr && ldsb != nullptr))
    return SK_ERR_INVALID_ARG;
  if (desc_bytes < (size_t)nprobs * sizeof(ProbDesc)) return SK_ERR_WORKSPACE;
  const int32_t dt = probs[0].dtype_ab;
  int32_t all_aligned = 1;
  for (int32_t i = 0; i < nprobs; ++i) {
    const int32_t j = P.order[i];
    const sk_problem& p = probs[j];
    ProbDesc& d = P.descs[i];
    d.A = A[j]; d.B = B[j]; d.Cout = C_out[j];
    d.Cin = C_in ? C_in[j] : nullptr;
    const bool empty = p.M == 0 || p.N == 0;
    if (!empty) {
      if (d.Cout == nullptr) return SK_ERR_INVALID_ARG;
      if (p.K > 0 && (d.A == nullptr || d.B == nullptr)) return SK_ERR_INVALID_ARG;
      if (p.beta != 0.f && d.Cin == nullptr) return SK_ERR_INVALID_ARG;
    }
    if (mx) {
      const MxScales m{sA[j], ldsa[j], sB[j], ldsb[j]};
      st = check_mx(p, d.A, d.B, m);
      if (st != SK_OK) return st;
      d.sA = m.sA; d.sB = m.sB;
      d.ldsa = m.ldsa; d.ldsb = m.ldsb;
    }
    d.aligned = aligned16(d.A) && aligned16(d.B) && elems_to_bytes(dt, p.lda) % 16 == 0 &&
                elems_to_bytes(dt, p.ldb) % 16 == 0;
    all_aligned &= d.aligned;
  }
  if (hipMemcpyAsync(dev_desc, P.descs.data(), (size_t)nprobs * sizeof(ProbDesc),
                     hipMemcpyHostToDevice, (hipStream_t)stream) != hipSuccess)
    return SK_ERR_HIP;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SK_ERR_HIP;
  memset(plan, 0, sizeof(*plan));
  plan->nprobs = nprobs;
  plan->mode = cfg->mode;
  plan->dtype_ab = probs[0].dtype_ab;
  plan->dtype_c = probs[0].dtype_c;
  plan->layout_a = probs[0].layout_a;
  plan->layout_b = probs[0].layout_b;
  plan->block_m = cfg->block_m;
  plan->block_n = cfg->block_n;
  plan->block_k = cfg->block_k;
  plan->T = P.T; plan->S = P.S; plan->W = P.W; plan->g = P.g;
  plan->q = P.q; plan->rho = P.rho;
  plan->workspace_bytes = P.ws_bytes;
  plan->xcd_remap = cfg->xcd_remap;
  plan->group_m = P.group_m;
  plan->spin_limit = cfg->spin_limit;
  plan->all_aligned = all_aligned;
  plan->max_iters = P.max_iters;
  return SK_OK;
}

sk_status sk_grouped_prepare(const sk_problem* probs, const void* const* A,
                             const void* const* B, const void* const* C_in, void* const* C_out,
                             int32_t nprobs, const sk_config* cfg, void* dev_desc,
                             size_t desc_bytes, sk_grouped_plan* plan, void* stream) {
  return grouped_prepare(probs, A, B, nullptr, nullptr, nullptr, nullptr, C_in, C_out, nprobs,
                         cfg, dev_desc, desc_bytes, plan, stream);
}

sk_status sk_grouped_prepare_mx(const sk_problem* probs, const void* const* A,
                                const void* const* B, const void* const* scale_a,
                                const int64_t* ld_scale_a, const void* const* scale_b,
                                const int64_t* ld_scale_b, const void* const* C_in,
                                void* const* C_out, int32_t nprobs, const sk_config* cfg,
                                void* dev_desc, size_t desc_bytes, sk_grouped_plan* plan,
                                void* stream) {
  if (scale_a == nullptr || ld_scale_a == nullptr || scale_b == nullptr || ld_scale_b == nullptr)
    return SK_ERR_INVALID_ARG;
  return grouped_prepare(probs, A, B, scale_a, ld_scale_a, scale_b, ld_scale_b, C_in, C_out,
                         nprobs, cfg, dev_desc, desc_bytes, plan, stream);
}

static sk_status grouped_common(const sk_grouped_plan* plan, const void* dev_desc,
                                void* workspace, size_t ws_bytes_, const sk_debug* dbg,
                                void* stream) {
  if (plan == nullptr || dev_desc == nullptr || plan->nprobs <= 0) return SK_ERR_INVALID_ARG;
  if (plan->mode < 0 || plan->mode > 3) return SK_ERR_INVALID_ARG;
  Plan P;
  P.T = plan->T; P.S = plan->S; P.W = plan->W; P.g = plan->g;
  P.q = plan->q; P.rho = plan->rho;
  P.ws_bytes = plan->workspace_bytes;
  P.group_m = plan->group_m;
  P.max_iters = plan->max_iters;
  P.dp_grid = plan->mode == SK_MODE_DP ||
              (plan->mode == SK_MODE_AUTO && plan->S == 0 && plan->nprobs == 1);
  sk_config cfg;
  memset(&cfg, 0, sizeof(cfg));
  cfg.block_m = plan->block_m;
  cfg.block_n = plan->block_n;
  cfg.block_k = plan->block_k;
  cfg.xcd_remap = plan->xcd_remap;
  cfg.group_m = plan->group_m;
  cfg.spin_limit = plan->spin_limit;
  cfg.mode = plan->mode;
  return launch(P, &cfg, plan->dtype_ab, plan->layout_a, plan->layout_b, plan->dtype_c, nullptr,
                (const ProbDesc*)dev_desc, plan->nprobs, workspace, ws_bytes_, dbg,
                (hipStream_t)stream);
}

sk_status sk_gemm_grouped(const sk_grouped_plan* plan, const void* dev_desc, void* workspace,
                          size_t ws_bytes_, void* stream) {
  return grouped_common(plan, dev_desc, workspace, ws_bytes_, nullptr, stream);
}

sk_status sk_gemm_grouped_debug(const sk_grouped_plan* plan, const void* dev_desc,
                                void* workspace, size_t ws_bytes_, const sk_debug* dbg,
                                void* stream) {
  if (dbg == nullptr) return SK_ERR_INVALID_ARG;
  return grouped_common(plan, dev_desc, workspace, ws_bytes_, dbg, stream);
}

}  // extern "C"
