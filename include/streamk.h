/*
 * streamk.h -- C ABI of the MI355X (gfx950) Stream-K GEMM library
 * (libstreamk.so).
 *
 * The library computes the general matrix product the report studies
 * (Introduction, Background; measured as M x N x K problems in Results,
 * Table 1):
 *
 *     C_out = alpha * scale_a * scale_b * (A x B) + beta * C_in
 *
 * with A of size M x K, B of size K x N and C of size M x N, using Stream-K's
 * work-centric decomposition (Background section): the multiply-accumulate
 * (MAC) loop iterations of all output tiles are counted together and split
 * evenly over one persistent workgroup per compute unit -- the report's
 * "Compute Units" launch parameter (Methodology) -- and a tile whose
 * iterations straddle two or more workgroups is finished by a partial-sum
 * fixup.  A data-parallel (one tile per workgroup) + Stream-K hybrid covers
 * the tile count's remainder, and a plain data-parallel grid is available as
 * the baseline the method is compared with.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.     Every data pointer (A, B, C_in, C_out, workspace, device
 *               descriptors) is caller-owned device memory of the current HIP
 *               device.  The library never allocates or frees device memory
 *               and never keeps a pointer after a call returns; its only
 *               device memory of its own is the static scratch array of
 *               sk_gemm_noalloc.
 * Streams.      `hip_stream` is a hipStream_t passed as void* (NULL = the
 *               null stream).  Launch entry points only enqueue work and
 *               return; they do not synchronise.
 * Errors.       Every entry point returns an sk_status; nothing aborts and no
 *               C++ exception crosses the ABI.  On an error return no work has
 *               been enqueued.  Errors raised inside a kernel (a fixup wait
 *               that exceeded its spin limit) are reported later by
 *               sk_check_device_error.
 * Threads.      Entry points are thread-safe; concurrent launches must use
 *               distinct workspaces.
 * Layout.       Element (i,k) of A is a[i*lda + k] (SK_ROW_MAJOR) or
 *               a[k*lda + i] (SK_COL_MAJOR); element (k,j) of B is
 *               b[k*ldb + j] (row-major) or b[j*ldb + k] (column-major);
 *               C is always row-major: c[i*ldc + j].  Leading dimensions are
 *               in elements.  C_in and C_out share ldc and dtype_c and may
 *               alias (in-place update).
 * Padding.      Problems are not padded (the report's padding study, Results
 *               and Table 1): out-of-range rows/columns/k-elements of a tile
 *               read as zero and out-of-range outputs are not written.
 * Alignment.    Any element-aligned pointer and leading dimension works.  The
 *               fast 16-byte load path is used when A and B start on 16-byte
 *               boundaries and lda*size, ldb*size are multiples of 16 bytes;
 *               otherwise the element-wise path is used (same results).
 */
#ifndef STREAMK_H
#define STREAMK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SK_OK = 0,
  SK_ERR_INVALID_ARG = -1,    /* a dimension, leading dimension, pointer or
                                 config field is out of range */
  SK_ERR_UNSUPPORTED = -2,    /* dtype / tile / layout combination not built */
  SK_ERR_WORKSPACE = -3,      /* workspace missing or smaller than required */
  SK_ERR_OCCUPANCY = -4,      /* more persistent workgroups than the device
                                 can keep resident at once */
  SK_ERR_HIP = -5,            /* a HIP runtime call failed */
  SK_ERR_CAPACITY = -6,       /* an output array is too small */
  SK_ERR_DEVICE_TIMEOUT = -7  /* a fixup wait gave up (see spin_limit) */
} sk_status;

/* Input (A, B) element types.  SK_F8E4M3 is the OCP 8-bit e4m3 "fn" format
 * (finite, max 448) that gfx950 matrix cores consume.  SK_MXF8E4M3 is OCP
 * MXFP8: e4m3 elements, and for every 32 consecutive K-values of each row of
 * A and each column of B an E8M0 scale byte e (value 2^(e-127), e = 255 NaN)
 * that multiplies them (sk_gemm_mx only).  SK_MXF4E2M1 is OCP MXFP4: E2M1
 * elements (sign, 2 exponent bits with bias 1, 1 mantissa bit: magnitudes
 * 0, 0.5, 1, 1.5, 2, 3, 4, 6) packed two per byte, element 2j of a row in
 * the low nibble of byte j, with the same E8M0 block scales.  SK_MXF6E2M3
 * and SK_MXF6E3M2 are OCP MXFP6: six-bit elements (sign, then 2 exponent
 * bits with bias 1 and 3 mantissa bits, max 7.5; or 3 exponent bits with
 * bias 3 and 2 mantissa bits, max 28; no infinities or NaNs) packed
 * little-endian, element k of a row at bits 6k .. 6k+5 of the row's bytes
 * (a block of 32 elements is 24 bytes), with the same E8M0 block scales.
 * SK_F8E5M2 is OCP e5m2 with per-tensor scales, taken as SK_F8E4M3 is
 * (every layout, the same tiles).
 * SK_MXF8E5M2 is OCP MXFP8 with e5m2 elements (sign, 5 exponent bits with
 * bias 15, 2 mantissa bits; exponent 31 holds infinities and NaNs; max
 * finite 57344), one byte each, with the same block scales.
 * Sizes and leading dimensions count elements.  Accumulation is FP32 for
 * every input type. */
typedef enum {
  SK_F32 = 0, SK_F16 = 1, SK_BF16 = 2, SK_F8E4M3 = 3, SK_MXF8E4M3 = 4, SK_MXF4E2M1 = 5,
  SK_MXF6E2M3 = 6, SK_MXF6E3M2 = 7, SK_MXF8E5M2 = 8, SK_F8E5M2 = 9
} sk_dtype;
typedef enum { SK_ROW_MAJOR = 0, SK_COL_MAJOR = 1 } sk_layout;

/* How output tiles are distributed (Background section):
 *   SK_MODE_HYBRID  data-parallel + Stream-K: tiles [S, T) are whole tiles
 *                   dealt to the persistent workgroups in rounds of g
 *                   (position x, or g-1-x in odd rounds), tiles
 *                   [0, S) are split by MAC iterations; S = 0 when T is a
 *                   multiple of g, else min(T, T mod g + g) ("two-tile" rule),
 *                   unless sk_config.dp_tiles >= 0 sets S = T - dp_tiles.
 *   SK_MODE_SK      every tile is a Stream-K tile (S = T).
 *   SK_MODE_DP      baseline data-parallel grid: one workgroup per tile,
 *                   no persistence, no fixup, no workspace.
 *   SK_MODE_AUTO    SK_MODE_HYBRID, except that S = 0 (no tile is split)
 *                   unless the launch-time model (sk_cost_model) predicts
 *                   the launch without splits to be more than `margin`
 *                   times slower (1.07; FP32 inputs, whose kernels the
 *                   model fits more closely, 1.03); with nothing split on one problem
 *                   the launch is the data-parallel grid itself.  The
 *                   model's constants are measured on MI355X; not in the
 *                   report. */
typedef enum {
  SK_MODE_HYBRID = 0, SK_MODE_SK = 1, SK_MODE_DP = 2, SK_MODE_AUTO = 3
} sk_mode;

/* Role of a schedule segment (what a workgroup does with one tile). */
typedef enum {
  SK_ROLE_FULL = 0,     /* all MAC iterations of the tile, then the epilogue */
  SK_ROLE_FINISH = 1,   /* iterations [0, k_end), then waits for npeers
                           partial tiles, sums them and runs the epilogue */
  SK_ROLE_PARTIAL = 2,  /* iterations [k_begin, k_end) with k_begin > 0;
                           stores the partial tile and signals its owner */
  SK_ROLE_DP = 3        /* a whole data-parallel tile */
} sk_role;

/* Activation of the fused epilogue (beyond the report, whose GEMM is the
 * bare product: the epilogue of a linear layer, the deep-learning use its
 * Introduction names).  Computed in FP32 on the FP32 sum of the epilogue:
 *   SK_ACT_RELU  max(v, 0) (NaN passes through)
 *   SK_ACT_GELU  v * Phi(v) = 0.5 v (1 + erf(v / sqrt 2)) (the erf form)
 *   SK_ACT_SILU  v / (1 + exp(-v)) */
typedef enum {
  SK_ACT_NONE = 0, SK_ACT_RELU = 1, SK_ACT_GELU = 2, SK_ACT_SILU = 3
} sk_activation;

/* One GEMM.  dtype_c is SK_F32, SK_F16 or SK_BF16 (results are rounded to
 * nearest-even from FP32).  scale_a / scale_b are the per-tensor scales of
 * FP8 inputs (use 1 otherwise).  beta == 0 means C_in is never read.
 *
 * Fused epilogue: with bias and activation left zero (a zeroed tail, as a
 * caller that predates these fields leaves it) the output is the product
 * above.  Otherwise
 *   C_out[i][j] = act(alpha*scale_a*scale_b*(A B)[i][j] + beta*C_in[i][j]
 *                     + bias[j])
 * with bias a device array of N FP32 values, 4-byte aligned (NULL: no bias),
 * applied once per output element by the workgroup that finishes the tile
 * (partial tiles hold raw sums).  Unknown activation codes are
 * SK_ERR_INVALID_ARG.  The planning calls ignore both fields. */
typedef struct {
  int64_t M, N, K;
  int32_t layout_a, layout_b;   /* sk_layout */
  int64_t lda, ldb, ldc;        /* elements */
  int32_t dtype_ab;             /* sk_dtype of A and B */
  int32_t dtype_c;              /* sk_dtype of C_in / C_out */
  float alpha, beta, scale_a, scale_b;
  const float* bias;            /* device, N values, or NULL */
  int32_t activation;           /* sk_activation */
  int32_t reserved;             /* 0 */
} sk_problem;

/* Launch configuration.  block_m x block_n x block_k must be a tile built
 * for dtype_ab (sk_supported_tiles); block_k is the number of K elements of
 * one MAC-loop iteration, which is 128 bytes of K: 32 (f32), 64 (f16, bf16)
 * or 128 (e4m3).  A zeroed struct plus a tile is a valid default. */
typedef struct {
  int32_t block_m, block_n, block_k;
  int32_t num_cu;      /* compute units to use, 1..device CUs; 0 = all
                          (the report's "Compute Units" argument) */
  int32_t wg_per_cu;   /* persistent workgroups per CU; 0 means 1.
                          g = num_cu * wg_per_cu persistent workgroups */
  int32_t mode;        /* sk_mode */
  int64_t dp_tiles;    /* -1: hybrid rule; >= 0: S = T - min(dp_tiles, T)
                          (ignored in SK_MODE_DP) */
  int32_t group_m;     /* 0: row-major tile order; > 0: bands of group_m
                          tile rows, walked down the band first; -1:
                          automatic (with Stream-K tiles, bands of the
                          largest divisor of q/gcd(q, I) not above the tile
                          rows, so that workgroups starting at the same
                          k-phase work on one tile row; otherwise bands of
                          8 rows) */
  int32_t xcd_remap;   /* 1: hardware workgroup b runs logical id
                          (b mod 8)*(g/8) + b/8 (when g mod 8 == 0) so
                          consecutive logical ids share an XCD's L2 */
  int64_t spin_limit;  /* polls a fixup wait makes before giving up and
                          raising SK_ERR_DEVICE_TIMEOUT; 0 = default (about
                          four seconds) */
  int32_t min_iters;   /* grid floor m for every mode but SK_MODE_DP: the
                          launch uses g' = min(g, max(1, W_all / m))
                          workgroups, W_all = MAC iterations of all tiles, so
                          that a split tile has few contributors when the
                          problem is small.  0 = automatic: m =
                          ceil(I / c), I = ceil(W_all / T), c the largest
                          integer >= 1 with f c^2 <= I, f the fixup cost
                          of SK_MODE_AUTO; 1 = keep g.
                          sk_plan_info.g reports g'. */
} sk_config;

/* One schedule segment (sk_schedule output, and the device trace). */
typedef struct {
  int32_t wg;        /* logical workgroup id (tile id for SK_MODE_DP) */
  int32_t problem;   /* index into the problem array */
  int32_t tile;      /* global tile index (problem-major, problems in the
                        grouped order of sk_plan) */
  int32_t tile_m, tile_n;   /* tile coordinates inside the problem */
  int32_t k_begin, k_end;   /* MAC iterations [k_begin, k_end) of the tile */
  int32_t role;      /* sk_role */
  int32_t npeers;    /* FINISH: number of partial tiles it waits for */
} sk_segment;

/* Schedule parameters of a problem set under a config. */
typedef struct {
  int64_t T;         /* output tiles */
  int64_t S;         /* Stream-K tiles [0, S); data-parallel tiles [S, T) */
  int64_t W;         /* MAC iterations of the Stream-K tiles */
  int64_t g;         /* workgroups launched (T for SK_MODE_DP) */
  int64_t q, rho;    /* workgroup x owns q + (x < rho) iterations */
  int64_t workspace_bytes;
  int64_t max_iters; /* largest per-tile iteration count */
  int64_t group_m;   /* tile order used (group_m = -1 resolved) */
  int64_t dp_grid;   /* 1: the launch is the data-parallel grid (one
                        workgroup per tile: SK_MODE_DP, or SK_MODE_AUTO with
                        nothing to split on one problem) */
  double predicted_us;     /* launch-time model (sk_cost_model): this launch */
  double predicted_dp_us;  /* ... and the data-parallel grid of the problems */
} sk_plan_info;

/* Returns a static English description of a status code (library
 * mechanism; no passage of the report). */
const char* sk_status_string(int32_t status);

/* Device facts for the current HIP device: number of compute units, and the
 * number of workgroups of the kernel selected by (cfg tile, dtype_ab) that
 * can be resident on one CU at once.  Either output may be NULL.  (The
 * persistent grid is sized from the CU count: the report's "Compute Units"
 * argument, Methodology.) */
sk_status sk_device_query(int32_t* num_cu, int32_t* max_wg_per_cu,
                          const sk_config* cfg, int32_t dtype_ab);

/* Lists the tiles built for dtype_ab as (block_m, block_n, block_k)
 * triples in `out` (3*capacity ints; may be NULL to count).  `count`
 * receives the number of tiles.  (A small menu per precision: the report's
 * Background argues one Stream-K configuration per precision suffices.) */
sk_status sk_supported_tiles(int32_t dtype_ab, int32_t* out, int32_t capacity,
                             int32_t* count);

/* Host-only.  Schedule parameters of `nprobs` problems under `cfg`: tiles,
 * iterations, the split point of the data-parallel + Stream-K hybrid and the
 * even share q, rho of each workgroup (Background: even work units over all
 * cores; Methodology: "Compute Units").  The
 * problems are concatenated as in a grouped launch: ordered by MAC
 * iterations per tile, ceil(K / block_k), largest first, ties in the given
 * order, so that the whole tiles dealt to the persistent workgroups (in
 * rounds of g, at position x in even rounds and g-1-x in odd ones) balance
 * (SK_MODE_DP keeps the given order; a reading for grouped launches, which
 * the report does not treat).  cfg->num_cu must be > 0
 * when no HIP device is present. */
sk_status sk_plan(const sk_problem* probs, int32_t nprobs,
                  const sk_config* cfg, sk_plan_info* info);

/* Host-only.  Constants of the launch-time model that SK_MODE_AUTO uses
 * (the report names a predictive block-to-time model as future work:
 * Results, the Block2Time paragraph; Future Work).  A launch's predicted time
 * is t_launch plus its slowest workgroup's time; a workgroup's time sums,
 * over its segments in the order of sk_schedule,
 *   t_tile + iterations * t_it(n) * (1 + l2 for Stream-K segments)
 *   + t_cin (epilogue with beta != 0) + t_store (PARTIAL)
 *   + npeers * t_peer (FINISH, after every peer's PARTIAL has been stored),
 * with t_it(n) = t_it_light + (t_it_full - t_it_light) * clamp((n-64)/192,
 * 0, 1) for n workgroups at once; a data-parallel grid of T tiles on C CUs
 * takes ceil(T / C) waves (several problems: max(longest tile, work / C)).
 * SK_MODE_AUTO splits tiles only when the launch without splits is
 * predicted `margin` times slower.  constants[0..9] = t_launch, t_tile,
 * t_it_full, t_it_light, t_store, t_peer (microseconds), l2, t_cin
 * (microseconds), margin, and the table row's tile as block_m * 65536 +
 * block_n (the row of the same type with the nearest tile area when
 * (block_m, block_n) has none; f16 uses bf16's).  n >= 10.  Measured on
 * MI355X per type and tile (paper_2407_00044_amd/calibrate.py). */
sk_status sk_cost_model(int32_t dtype_ab, int32_t block_m, int32_t block_n,
                        float* constants, int32_t n);

/* Host-only.  The order in which a launch concatenates the problems:
 * order[i] is the caller's index of the i-th problem (nprobs entries). */
sk_status sk_plan_order(const sk_problem* probs, int32_t nprobs,
                        const sk_config* cfg, int32_t* order);

/* Host-only.  The complete schedule (Background: the MAC iterations of all
 * tiles split evenly, a tile crossing a boundary finished by a fixup; Figure
 * 1's data-parallel comparison is SK_MODE_DP): for each logical workgroup in order,
 * its Stream-K segments in processing order, then its data-parallel tiles
 * in increasing tile order.  With out == NULL only *count is set; with too
 * small a capacity *count is set and SK_ERR_CAPACITY returned. */
sk_status sk_schedule(const sk_problem* probs, int32_t nprobs,
                      const sk_config* cfg, sk_segment* out, int64_t capacity,
                      int64_t* count);

/* Bytes of workspace a launch of `probs` under `cfg` needs: room for the
 * partial tiles of the fixup that finishes split tiles (Background).  The layout
 * has fixed offsets, the same for every problem and config:
 *   [0, 256)        header: error word, epoch word, done counter;
 *   [256, 16640)    one 32-bit token per persistent workgroup (at most 4096);
 *   [16640, ...)    g FP32 partial tiles of block_m x block_n.
 * A workgroup that leaves a partial tile writes the launch's tag (epoch + 1)
 * into its token; the tile's finisher waits for that tag; the last workgroup
 * of a launch advances the epoch.  Tokens of earlier launches therefore
 * never match, whatever problems, tiles or workgroup counts the workspace
 * served before.  Only launches that split tiles (S > 0) use more than the
 * 256-byte header: 0 for SK_MODE_DP and the auto mode's data-parallel grid.
 */
sk_status sk_workspace_size(const sk_problem* probs, int32_t nprobs,
                            const sk_config* cfg, size_t* bytes);

/* Zeroes `bytes` of workspace on `hip_stream` with a fill kernel (safe to
 * record into a HIP graph).  Required once before a workspace's first use;
 * afterwards every launch leaves the header consistent by itself, also one
 * whose fixup wait timed out (SK_ERR_DEVICE_TIMEOUT: that launch's output is
 * invalid, later launches on the workspace are not affected). */
sk_status sk_workspace_init(void* workspace, size_t bytes, void* hip_stream);

/* One GEMM: C_out = alpha*scale_a*scale_b*A*B + beta*C_in (the product the
 * report studies: Introduction, Background; its M x N x K problems, Results,
 * Table 1), on the schedule of sk_schedule.
 * workspace/ws_bytes: at least sk_workspace_size bytes, initialised once by
 * sk_workspace_init; not shared with a concurrent launch.  May be NULL for
 * SK_MODE_DP.  M == 0 or N == 0 is a no-op; K == 0 gives beta*C_in.
 * Asynchronous on hip_stream; capturable into a HIP graph. */
sk_status sk_gemm(const sk_problem* p, const void* A, const void* B,
                  const void* C_in, void* C_out, void* workspace,
                  size_t ws_bytes, const sk_config* cfg, void* hip_stream);

/* One MX GEMM (dtype_ab = SK_MXF8E4M3, SK_MXF8E5M2, SK_MXF4E2M1,
 * SK_MXF6E2M3 or SK_MXF6E3M2): as sk_gemm, with
 *   C_out[i][j] = alpha*scale_a*scale_b * sum_k A[i][k] * 2^(sa[i][k/32]-127)
 *                                   * B[k][j] * 2^(sb[j][k/32]-127) + beta*C_in
 * where A, B hold e4m3 / e5m2 codes (MXFP4, MXFP6: packed codes), sa[i][b] = ((const uint8_t*)scale_a)[i*ld_scale_a
 * + b] and sb[j][b] = ((const uint8_t*)scale_b)[j*ld_scale_b + b] (device
 * memory; one E8M0 byte per 32 K-values of row i of A / column j of B).
 * The block scales are applied by the matrix cores (gfx950 scaled MFMA),
 * products accumulate in FP32.  Block-scaled formats go beyond the report,
 * whose CK kernel is one configuration per precision (Background); the
 * scaled MX formats are the gfx950 matrix cores' own.
 * Requirements (else SK_ERR_UNSUPPORTED): A row-major and B column-major,
 * K a multiple of 128 (MXFP4: 256), A and B 16-byte aligned with rows of a
 * multiple of 16 bytes (lda, ldb multiples of 16; MXFP4: 32; MXFP6: 64).
 * scale_a/scale_b 4-byte aligned, ld_scale_a/ld_scale_b multiples of 4 and
 * >= K/32 (else SK_ERR_INVALID_ARG).  Grouped launches:
 * sk_grouped_prepare_mx; sk_gemm with an MX type returns
 * SK_ERR_INVALID_ARG. */
sk_status sk_gemm_mx(const sk_problem* p, const void* A, const void* B,
                     const void* scale_a, int64_t ld_scale_a, const void* scale_b,
                     int64_t ld_scale_b, const void* C_in, void* C_out,
                     void* workspace, size_t ws_bytes, const sk_config* cfg,
                     void* hip_stream);

/* Debug hooks of sk_gemm_debug (all device pointers may be NULL). */
typedef struct {
  sk_segment* trace;        /* device array: one record per segment run */
  int64_t trace_capacity;   /* records that fit in `trace` */
  int64_t* trace_count;     /* device counter, zeroed by the caller; receives
                               the number of records (may exceed capacity) */
  int32_t* cover;           /* device array [T * cover_stride], zeroed by the
                               caller; cover[t*cover_stride + k] counts the
                               runs of MAC iteration k of tile t */
  int64_t cover_stride;     /* >= sk_plan_info.max_iters */
  int32_t partial_delay;    /* sleep rounds (~64 clocks each) a PARTIAL
                               segment waits before publishing */
  int32_t reverse_ids;      /* 1: hardware workgroup b runs logical id
                               g-1-b (stress of the fixup ordering) */
} sk_debug;

/* sk_gemm with the debug hooks above: same arithmetic and schedule, plus
 * a device trace of the segments run and per-iteration coverage counts.
 * For tests; never used for timing. */
sk_status sk_gemm_debug(const sk_problem* p, const void* A, const void* B,
                        const void* C_in, void* C_out, void* workspace,
                        size_t ws_bytes, const sk_config* cfg,
                        const sk_debug* dbg, void* hip_stream);

/* Library mechanism (no passage of the report: its fixup wait is
 * unbounded).  Reads and clears the workspace's device error word (synchronises
 * hip_stream).  Returns SK_ERR_DEVICE_TIMEOUT if a fixup wait of an earlier
 * launch gave up, SK_OK otherwise; *code receives the raw word if non-NULL.
 * workspace NULL: the scratch of sk_gemm_noalloc on the current device
 * (SK_OK if that entry point has not run there); ws_bytes is then ignored. */
sk_status sk_check_device_error(void* workspace, size_t ws_bytes,
                                int32_t* code, void* hip_stream);

/* ---- Allocation-free GEMM ------------------------------------------------
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same problem, operands, config, arithmetic and schedule as
 * sk_gemm; the workspace is instead a static device array of
 * SK_NOALLOC_SCRATCH_BYTES per GPU (256 B header + 4096 arrival tokens +
 * 256 partial tiles of 256x256 FP32, i.e. 64 MiB + 16.25 KiB), held by the
 * library until the process ends.  No device memory is allocated or freed.
 * The first call on a device looks the array up and enqueues one fill
 * kernel on hip_stream that clears its header and tokens.
 * Errors: SK_ERR_WORKSPACE when the plan needs more than the array
 * (sk_workspace_size > SK_NOALLOC_SCRATCH_BYTES, e.g. more than 256
 * persistent workgroups at 256x256), otherwise as sk_gemm.  A fixup wait
 * that gives up is reported by sk_check_device_error(NULL, 0, ...).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or host threads without ordering) race and give
 * wrong results; calls ordered on one stream are safe. */
#define SK_NOALLOC_SCRATCH_BYTES ((size_t)16640 + (size_t)256 * 256 * 256 * 4)
sk_status sk_gemm_noalloc(const sk_problem* p, const void* A, const void* B,
                          const void* C_in, void* C_out, const sk_config* cfg,
                          void* hip_stream);

/* ---- Grouped GEMM: one persistent launch over several problems ----------
 * The MAC iterations of all problems' Stream-K tiles are counted together
 * and split evenly over the persistent workgroups (Background section: even
 * work units over all cores, here over the tiles of every problem).
 * Problems are concatenated in the order sk_plan_order reports: by MAC
 * iterations per tile, largest first, ties in the given order (SK_MODE_DP:
 * the given order).  All problems share dtype_ab, dtype_c, layout_a and
 * layout_b.  The launch entry point takes a host plan plus device
 * descriptors (rather than a bare descriptor array and a config) so that a
 * captured launch replays exactly the schedule that was prepared. */

/* Host-side plan of a grouped launch, filled by sk_grouped_prepare. */
typedef struct {
  int32_t nprobs;
  int32_t mode;                 /* sk_mode the plan was made for */
  int32_t dtype_ab, dtype_c, layout_a, layout_b;
  int32_t block_m, block_n, block_k;
  int64_t T, S, W, g, q, rho;
  int64_t workspace_bytes;
  int32_t xcd_remap, group_m;
  int64_t spin_limit;
  int32_t all_aligned;
  int64_t max_iters;            /* largest per-tile iteration count */
} sk_grouped_plan;

/* Bytes of device descriptor memory sk_grouped_prepare needs. */
sk_status sk_grouped_desc_size(int32_t nprobs, size_t* bytes);

/* Validates the problems, computes the plan and copies the per-problem
 * descriptors (pointers, sizes, strides, scales, tile and iteration
 * offsets) into `dev_desc` (device memory of at least sk_grouped_desc_size
 * bytes).  Synchronises hip_stream; not capturable.  The descriptor stays
 * valid while the pointed-to buffers do. */
sk_status sk_grouped_prepare(const sk_problem* probs, const void* const* A,
                             const void* const* B, const void* const* C_in,
                             void* const* C_out, int32_t nprobs,
                             const sk_config* cfg, void* dev_desc,
                             size_t desc_bytes, sk_grouped_plan* plan,
                             void* hip_stream);

/* sk_grouped_prepare for MX problems (dtype_ab = SK_MXF8E4M3 or
 * SK_MXF4E2M1 in every problem; beyond the report: OCP MX block scaling, as
 * sk_gemm_mx):
 * scale_a[i] / scale_b[i] are problem i's E8M0 scales (rows of A, columns
 * of B, one byte per 32 K-values, ld_scale_a[i] / ld_scale_b[i] bytes
 * apart), with sk_gemm_mx's requirements per problem (K-contiguous
 * operands, whole iterations, 16-byte aligned operands and rows, 4-byte
 * aligned scale rows of at least K/32 bytes).  sk_grouped_prepare with MX
 * problems returns SK_ERR_INVALID_ARG.
 * The plan launches with sk_gemm_grouped. */
sk_status sk_grouped_prepare_mx(const sk_problem* probs, const void* const* A,
                                const void* const* B, const void* const* scale_a,
                                const int64_t* ld_scale_a, const void* const* scale_b,
                                const int64_t* ld_scale_b, const void* const* C_in,
                                void* const* C_out, int32_t nprobs,
                                const sk_config* cfg, void* dev_desc,
                                size_t desc_bytes, sk_grouped_plan* plan,
                                void* hip_stream);

/* Launches one grouped GEMM described by plan + dev_desc.  Launch only:
 * asynchronous and capturable into a HIP graph. */
sk_status sk_gemm_grouped(const sk_grouped_plan* plan, const void* dev_desc,
                          void* workspace, size_t ws_bytes, void* hip_stream);

/* sk_gemm_grouped with the debug hooks of sk_gemm_debug: a device trace of
 * the segments run (segment.problem is the caller's problem index) and
 * per-iteration coverage counts (cover_stride >= plan->max_iters).  For
 * tests; never used for timing. */
sk_status sk_gemm_grouped_debug(const sk_grouped_plan* plan, const void* dev_desc,
                                void* workspace, size_t ws_bytes, const sk_debug* dbg,
                                void* hip_stream);

/* ---- Operand packing -----------------------------------------------------
 * Library mechanism (the report's GEMMs take their operands as laid out).
 * Out-of-place transpose: `in` is a rows x cols row-major matrix (element
 * (i, j) at in[i*ld_in + j], ld_in >= max(1, cols)), `out` receives the
 * cols x rows row-major matrix out[j*ld_out + i] = in[i*ld_in + j] (ld_out
 * >= max(1, rows)); elements of elem_bytes = 1, 2 or 4 bytes are copied bit
 * for bit.  A column-major operand viewed as its row-major transpose gives,
 * through this, the K-contiguous copy that the GEMM kernels read with plain
 * 16-byte LDS reads (M- or N-major operands are read with transposing LDS
 * reads, which take two instructions per 16-bit fragment and four per
 * e4m3 fragment).  Device pointers, not overlapping; asynchronous on
 * hip_stream and capturable.  Errors: SK_ERR_INVALID_ARG for another
 * elem_bytes, negative sizes, a leading dimension below its minimum, NULL
 * pointers with rows * cols > 0, a matrix of 2^58 elements or more
 * (rows * ld_in or cols * ld_out), or overlapping matrices; SK_ERR_HIP if the
 * launch fails.  rows or cols 0: nothing is enqueued. */
sk_status sk_transpose(const void* in, int64_t rows, int64_t cols, int64_t ld_in,
                       void* out, int64_t ld_out, int32_t elem_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* STREAMK_H */
