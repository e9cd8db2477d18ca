// Stream-K GEMM kernel for gfx950 (CDNA4).
//
// One kernel template serves every mode:
//  * persistent Stream-K / hybrid: g workgroups; logical workgroup x runs its
//    even share [s_x, e_x) of the Stream-K tiles' MAC iterations (Background
//    section: even work units over all cores), finishing or contributing to
//    split tiles through the FP32 partial-tile workspace, then its
//    data-parallel tiles S+x, S+x+g, ...;
//  * baseline data-parallel grid: one workgroup per tile.
//
// Tile datapath (per MAC iteration = 128 bytes of K):
//  * K-contiguous operands: global -> LDS with LDS-direct 16-byte copies,
//    tile rows of 128 bytes of K; the 16-byte chunk c of row r is stored at
//    position c ^ ((r & 7) ^ ((r >> 3) & 3)), which keeps 8, 16 or 32
//    consecutive rows reading the same chunk on distinct banks and repeats
//    every 32 rows (so per-lane LDS addresses are shared by all 32-row
//    blocks of a wave); LDS -> MFMA operands with 16-byte reads;
//  * M/N-contiguous f16/bf16/e4m3 operands: LDS-direct copies of k-rows as
//    they lie in memory (16-byte chunks swizzled per k-row), read into MFMA
//    operands with gfx950's transposing LDS reads (ds_read_b64_tr_b16 /
//    _tr_b8);
//  * M/N-contiguous f32 operands (and e4m3 tiles of 64 rows): 16-byte loads
//    into registers, transposed there and written to LDS as K-contiguous
//    rows;
//  * LDS multi-buffered; 32x32 MFMA blocks accumulate in FP32
//    (v_mfma_f32_32x32x2_f32, _32x32x16_f16/_bf16, and the block-scaled
//    32x32x64 f8f6f4 form with unit scales for e4m3).
//  A and B fragments are read with the same (lane, slot) -> k assignment, so
//  the product is independent of how the matrix core orders k inside one
//  instruction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_params.hpp"
#include "sk_sched.hpp"

namespace sk {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

enum { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2, DT_F8 = 3, DT_MX8 = 4, DT_MX4 = 5, DT_MX6 = 6,
       DT_MX6E3 = 7, DT_MX8E5 = 8, DT_F8E5 = 9 };
// 8-bit e4m3 elements: plain (per-tensor scales, applied in the epilogue) or
// MXFP8 (an E8M0 scale per 32 K-values of each row of A and column of B,
// applied by the matrix core)
constexpr bool is_mx8(int dt) { return dt == DT_MX8 || dt == DT_MX8E5; }
constexpr bool is_f8pt(int dt) { return dt == DT_F8 || dt == DT_F8E5; }   // per-tensor scales
constexpr bool is_f8(int dt) { return is_f8pt(dt) || is_mx8(dt); }
// MXFP4: E2M1 elements packed two per byte, with MXFP8's block scales.  The
// kernels see its operands as bytes (K, lda, ldb in bytes, 256 elements per
// 128-byte iteration).
constexpr bool is_mx6(int dt) { return dt == DT_MX6 || dt == DT_MX6E3; }
constexpr bool is_mx(int dt) { return is_mx8(dt) || dt == DT_MX4 || is_mx6(dt); }
enum { L_ROW = 0, L_COL = 1 };
enum { R_FULL = 0, R_FINISH = 1, R_PARTIAL = 2, R_DP = 3 };

// Values that are the same in every lane, moved to scalar registers (the
// compiler cannot always prove it, and a buffer descriptor in vector
// registers forces a loop over lanes around every load).
__device__ __forceinline__ int32_t uniform32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ const char* uniform_ptr(const char* p) {
  return (const char*)uniform64((int64_t)p);
}

__device__ __forceinline__ int swz(int r) { return (r & 7) ^ ((r >> 3) & 3); }

__device__ __forceinline__ int lds_off(int row, int chunk) {
  return row * 128 + ((chunk ^ swz(row)) << 4);
}

// ---------------------------------------------------------------------------
// Operand staging, global memory -> LDS.
//
// Every operand tile is a block of R rows (m for A, n for B) by 128 bytes of
// K.  Two paths fill it:
//  * fast: 16-byte buffer loads (buffer_load_dwordx4).  A chunk that lies
//    outside the matrix (rows past M or N, whole chunks past K) gets an
//    offset beyond the buffer's size, for which the hardware returns zeros,
//    so edges cost no branches.  Needs 16-byte-aligned rows and no chunk that
//    straddles the end of a row (K or M/N not a multiple of the chunk).
//  * slow: element-by-element copy with explicit bounds checks, any
//    alignment; used only for the iterations/tiles where the fast path's
//    conditions fail.
// Offsets in a buffer are 32-bit; the host checks that a tile's furthest
// element is below 2^31 bytes from its base.

constexpr uint32_t kOOB = 0x80000000u;     // offset past any buffer size used
constexpr int kRsrcWord3 = 0x00020000;     // buffer descriptor dword 3 (32-bit data format)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const char* base, int64_t bytes) {
  const int32_t n = bytes <= 0 ? 0 : bytes >= (int64_t)kOOB ? (int32_t)kOOB : (int32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc((void*)uniform_ptr(base), (short)0, uniform32(n),
                                           kRsrcWord3);
}

// Operand geometry for one tile.
struct OpTile {
  const char* X;       // matrix base
  int64_t ld_b;        // leading dimension in bytes
  int64_t row0;        // first tile row (m or n)
  int64_t rows;        // M or N
  int64_t K;
  bool aligned;        // base and ld_b are multiples of 16 bytes
};

// One element of EB bytes through a buffer resource; an out-of-range offset
// (kOOB) reads as zero.
template <int EB>
__device__ __forceinline__ uint32_t buf_elem(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  if constexpr (EB == 4) return __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0);
  else if constexpr (EB == 2) return __builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0);
  else return __builtin_amdgcn_raw_buffer_load_b8(rs, (int)off, 0, 0);
}

// Packs 16/EB elements (each in the low EB bytes of a word) into a chunk.
template <int EB>
__device__ __forceinline__ u32x4 pack_chunk(const uint32_t (&e)[16 / EB]) {
  u32x4 v;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if constexpr (EB == 4) v[w] = e[w];
    else if constexpr (EB == 2) v[w] = (e[2 * w] & 0xffffu) | (e[2 * w + 1] << 16);
    else v[w] = (e[4 * w] & 0xffu) | ((e[4 * w + 1] & 0xffu) << 8) |
                ((e[4 * w + 2] & 0xffu) << 16) | (e[4 * w + 3] << 24);
  }
  return v;
}

// K-contiguous operand ("row-major A" / "column-major B"): element (r, k) at
// X[(row0 + r) * ld + k]; tile row r is 8 chunks of 16 bytes.  The fast
// path copies global memory straight into LDS (buffer_load_dwordx4 ... lds):
// one wave instruction fills 1 KiB of LDS, i.e. 8 consecutive tile rows, and
// lane i writes the 16 bytes at position i%8 of row i/8, so it fetches the
// logical chunk that the swizzle puts there.  No registers hold the stage.
template <int R, int EB, int NT, int KB = 128>
struct KMajorStage {
  static constexpr int EPC = 16 / EB;        // elements per chunk
  static constexpr int KE = KB / EB;         // K elements per iteration
  // chunks of a 128-byte LDS row that hold data: all 8, or (MXFP6, 96
  // bytes of K per iteration) the first 6; the others read nothing and
  // hold zeros
  static constexpr int KC = KB / 16;
  static_assert(KB % 16 == 0 && KB <= 128, "bytes of K per iteration");
  static constexpr int NI = R / (NT / 8);    // 1 KiB copies per wave
  static_assert(R % (NT / 8) == 0, "tile rows");

  __device__ __forceinline__ static bool slow(const OpTile& o, int64_t k0) {
    return !o.aligned || ((o.K % EPC) != 0 && k0 + KE > o.K);
  }

  __device__ __forceinline__ void issue(char* L, const OpTile& o, int64_t k0, int tid) {
    const char* base = o.X + o.row0 * o.ld_b;
    const int64_t rows_left = o.rows - o.row0;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, (rows_left - 1) * o.ld_b + o.K * EB);
    const int wave = uniform32(tid >> 6);
    int lane = tid & 63;
    // per-lane offsets are formed at each issue (a few adds), not hoisted
    // into registers that would live across the MAC loop
    asm volatile("" : "+v"(lane));
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const uint32_t kb32 = (uint32_t)(k0 * EB);
    const int32_t rl = (int32_t)imin(rows_left, R);
    const int32_t kleft = (int32_t)imin(o.K - k0, KE);   // K elements left in this slab
    const int lr = lane >> 3;                             // row inside the 8-row copy
    // Instruction j covers rows rbase..rbase+7, rbase = 8*(wave*NI + j); the
    // swizzle of row rbase + lr is lr ^ ((wave*NI + j) & 3).
    const uint32_t lane_row = (uint32_t)lr * ld32;
    if (rl == R && kleft == KE) {
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int jj = wave * NI + j;
        const int c = (lane & 7) ^ lr ^ (jj & 3);
        const uint32_t off = (KC < 8 && c >= KC) ? kOOB
            : lane_row + (uint32_t)(c * 16) + ((uint32_t)(jj * 8) * ld32 + kb32);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(L + jj * 1024), 16, (int)off, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int jj = wave * NI + j;
        const int c = (lane & 7) ^ lr ^ (jj & 3);
        const bool ok = jj * 8 + lr < rl && c * EPC < kleft;
        const uint32_t off = ok ? lane_row + (uint32_t)(c * 16) + ((uint32_t)(jj * 8) * ld32 + kb32)
                                : kOOB;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(L + jj * 1024), 16, (int)off, 0, 0, 0);
      }
    }
  }

  __device__ __forceinline__ void commit(char*, int) const {}

  // Copies of whole iterations with the per-lane offsets formed once per
  // tile (prep) and the iteration's K offset k0*EB passed as the scalar
  // offset of the buffer instruction: an issue is one LDS base move and one
  // buffer_load per copy.  Rows past the matrix keep an out-of-range offset.
  uint32_t pre[NI];
  __amdgpu_buffer_rsrc_t prs;

  __device__ __forceinline__ void prep(const OpTile& o, int tid) {
    const char* base = o.X + o.row0 * o.ld_b;
    const int64_t rows_left = o.rows - o.row0;
    prs = make_rsrc(base, (rows_left - 1) * o.ld_b + o.K * EB);
    const int wave = uniform32(tid >> 6);
    const int lane = tid & 63;
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const int32_t rl = (int32_t)imin(rows_left, R);
    const int lr = lane >> 3;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int jj = wave * NI + j;
      const int c = (lane & 7) ^ lr ^ (jj & 3);
      const bool ok = jj * 8 + lr < rl && (KC == 8 || c < KC);
      pre[j] = ok ? (uint32_t)(jj * 8 + lr) * ld32 + (uint32_t)(c * 16) : kOOB;
    }
  }

  // Whole iteration starting at K element k0 (k0 + KE <= K).  With on ==
  // false every lane reads out of range: the copies only write zeros into L.
  __device__ __forceinline__ void issue_pre(char* L, int64_t k0, int tid, bool on) const {
    const int wave = uniform32(tid >> 6);
    const int kb32 = uniform32((int32_t)(k0 * EB));
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int jj = wave * NI + j;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          prs, (__attribute__((address_space(3))) void*)(L + jj * 1024), 16,
          (int)(on ? pre[j] : kOOB), kb32, 0, 0);
    }
  }

  // Copy j alone (kb32: the iteration's scalar offset, as in issue_pre).
  __device__ __forceinline__ void issue_one(char* L, int kb32, int tid, bool on, int j) const {
    const int jj = uniform32(tid >> 6) * NI + j;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        prs, (__attribute__((address_space(3))) void*)(L + jj * 1024), 16,
        (int)(on ? pre[j] : kOOB), kb32, 0, 0);
  }
  __device__ __forceinline__ int k_offset(int64_t k0) const { return uniform32((int32_t)(k0 * EB)); }

  __device__ __forceinline__ static bool whole(const OpTile& o, int64_t k0) {
    return k0 + KE <= o.K;
  }

  // Edge iterations.  Rows 16-byte aligned (K ends inside a chunk): every
  // chunk is one 16-byte load, and the elements at k >= K are zeroed in
  // registers.  The buffer then extends to the end of the 4-byte word that
  // holds the matrix's last element (a word with valid data lies in a mapped
  // page), so no load reaches past it; the bytes it does read past K are
  // row padding or that word's tail, both masked.
  // Otherwise (any alignment) every element of the thread's chunks is loaded
  // on its own with an out-of-range offset where it lies outside the
  // matrix; all loads are issued before the chunks are packed and written.
  __device__ static void copy_slow(char* L, const OpTile& o, int64_t k0, int tid) {
    constexpr int NCH = R * 8 / NT;
    const char* base = o.X + o.row0 * o.ld_b;
    const int64_t rows_left = o.rows - o.row0;
    const int32_t rl = (int32_t)imin(rows_left, R);
    const int32_t kleft = (int32_t)imin(o.K - k0, KE);
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const uint32_t kb32 = (uint32_t)(k0 * EB);
    const int c = tid & 7;
    if (o.aligned) {
      const __amdgpu_buffer_rsrc_t rw =
          make_rsrc(base, (rows_left - 1) * o.ld_b + ((o.K * EB + 3) & ~(int64_t)3));
      const int nb = (kleft - c * EPC) * EB;   // valid bytes of this lane's chunk
      u32x4 v[NCH];
#pragma unroll
      for (int j = 0; j < NCH; ++j) {
        const int r = (tid >> 3) + j * (NT / 8);
        const bool ok = r < rl && nb > 0;
        v[j] = __builtin_amdgcn_raw_buffer_load_b128(
            rw, (int)(ok ? (uint32_t)r * ld32 + kb32 + (uint32_t)(c * 16) : kOOB), 0, 0);
      }
      u32x4 keep;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int kb = nb - 4 * w;             // valid bytes of word w
        keep[w] = kb >= 4 ? 0xffffffffu : kb <= 0 ? 0u : (1u << (8 * kb)) - 1u;
      }
#pragma unroll
      for (int j = 0; j < NCH; ++j) {
        const int r = (tid >> 3) + j * (NT / 8);
        *(u32x4*)(L + lds_off(r, c)) = v[j] & keep;
      }
      return;
    }
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, (rows_left - 1) * o.ld_b + o.K * EB);
    uint32_t e[NCH][EPC];
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int r = (tid >> 3) + j * (NT / 8);
#pragma unroll
      for (int i = 0; i < EPC; ++i) {
        const int kk = c * EPC + i;
        const bool ok = r < rl && kk < kleft;
        e[j][i] = buf_elem<EB>(rs, ok ? (uint32_t)r * ld32 + kb32 + (uint32_t)(kk * EB) : kOOB);
      }
    }
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int r = (tid >> 3) + j * (NT / 8);
      *(u32x4*)(L + lds_off(r, c)) = pack_chunk<EB>(e[j]);
    }
  }
};

// Register-staged variant of the K-contiguous path (16-byte buffer loads
// into registers, then 16-byte LDS writes); selected at build time.
template <int R, int EB, int NT, int KB = 128>
struct KMajorStageReg {
  static_assert(KB == 128, "register staging: 128 bytes of K per iteration");
  static constexpr int EPC = 16 / EB;
  static constexpr int KE = 128 / EB;
  static constexpr int NCH = R * 8 / NT;     // chunks per thread
  static_assert(NCH >= 1 && (R * 8) % NT == 0, "tile rows");
  u32x4 v[NCH];

  __device__ __forceinline__ static bool slow(const OpTile& o, int64_t k0) {
    return KMajorStage<R, EB, NT>::slow(o, k0);
  }

  __device__ __forceinline__ void issue(char*, const OpTile& o, int64_t k0, int tid) {
    const char* base = o.X + o.row0 * o.ld_b;
    const int64_t rows_left = o.rows - o.row0;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, (rows_left - 1) * o.ld_b + o.K * EB);
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const uint32_t kb32 = (uint32_t)(k0 * EB);
    const int32_t rl = (int32_t)imin(rows_left, R);
    const int32_t kleft = (int32_t)imin(o.K - k0, KE);
    const int c = tid & 7;
    const bool kok = c * EPC < kleft;
    const uint32_t lane_off = (uint32_t)(tid >> 3) * ld32 + kb32 + (uint32_t)(c * 16);
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int r = (tid >> 3) + j * (NT / 8);
      const bool ok = kok && r < rl;
      const uint32_t off = ok ? lane_off + (uint32_t)(j * (NT / 8)) * ld32 : kOOB;
      v[j] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    }
  }

  __device__ __forceinline__ void commit(char* L, int tid) const {
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int r = (tid >> 3) + j * (NT / 8);
      *(u32x4*)(L + lds_off(r, tid & 7)) = v[j];
    }
  }

  __device__ static void copy_slow(char* L, const OpTile& o, int64_t k0, int tid) {
    KMajorStage<R, EB, NT>::copy_slow(L, o, k0, tid);
  }
};

#ifndef SK_KMAJOR_DMA
#define SK_KMAJOR_DMA 1
#endif

// Register transpose of a block: in[j] holds 16/EB consecutive elements
// (along M or N) of k-row j; out[i] holds the 16/EB k-values of element i.
template <int EB>
__device__ __forceinline__ void transpose_block(const u32x4 (&in)[16 / EB],
                                                u32x4 (&out)[16 / EB]) {
  constexpr int E = 16 / EB;
  union U {
    u32x4 v;
    uint8_t b[16];
    uint16_t h[8];
    uint32_t w[4];
  };
  U a[E], o[E];
#pragma unroll
  for (int j = 0; j < E; ++j) a[j].v = in[j];
#pragma unroll
  for (int i = 0; i < E; ++i) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if constexpr (EB == 4) o[i].w[j] = a[j].w[i];
      else if constexpr (EB == 2) o[i].h[j] = a[j].h[i];
      else o[i].b[j] = a[j].b[i];
    }
  }
#pragma unroll
  for (int i = 0; i < E; ++i) out[i] = o[i].v;
}

// M/N-contiguous operand ("column-major A" / "row-major B"): element (r, k)
// at X[k * ld + row0 + r].  A thread loads a block of EPC k-rows x EPC tile
// rows (one 16-byte chunk per k-row), transposes it in registers and writes
// EPC K-contiguous chunks to LDS.
template <int R, int EB, int NT>
struct MNMajorStage {
  static constexpr int EPC = 16 / EB;
  static constexpr int KE = 128 / EB;
  static constexpr int RB = R / EPC;          // row blocks
  static constexpr int NBLK = RB * 8;         // x 8 chunk columns of K
  static constexpr int BPT = (NBLK + NT - 1) / NT;
  static_assert(R % EPC == 0, "tile rows");
  u32x4 v[BPT][EPC];

  __device__ __forceinline__ static bool slow(const OpTile& o, int64_t) {
    return !o.aligned || ((o.rows % EPC) != 0 && o.row0 + R > o.rows);
  }

  __device__ __forceinline__ void issue(char*, const OpTile& o, int64_t k0, int tid) {
    const char* base = o.X + o.row0 * EB;
    const int64_t rows_left = o.rows - o.row0;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, (o.K - 1) * o.ld_b + rows_left * EB);
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const int32_t rl = (int32_t)imin(rows_left, R);
    const int32_t kleft = (int32_t)imin(o.K - k0, KE);
    const uint32_t kb32 = (uint32_t)k0 * ld32;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int bidx = tid + NT * b;
      if (NBLK % NT != 0 && bidx >= NBLK) continue;
      const int rb = bidx % RB;
      const int kc = bidx / RB;
      const bool rok = rb * EPC < rl;
#pragma unroll
      for (int j = 0; j < EPC; ++j) {
        const int kk = kc * EPC + j;
        const bool ok = rok && kk < kleft;
        const uint32_t off = ok ? kb32 + (uint32_t)kk * ld32 + (uint32_t)(rb * 16) : kOOB;
        v[b][j] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
      }
    }
  }

  __device__ __forceinline__ void commit(char* L, int tid) const {
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int bidx = tid + NT * b;
      if (NBLK % NT != 0 && bidx >= NBLK) continue;
      const int rb = bidx % RB;
      const int kc = bidx / RB;
      u32x4 w[EPC];
      transpose_block<EB>(v[b], w);
#pragma unroll
      for (int i = 0; i < EPC; ++i) *(u32x4*)(L + lds_off(rb * EPC + i, kc)) = w[i];
    }
  }

  // Element-wise path: like issue()/commit() but every element is loaded on
  // its own (any alignment, partial row chunks).
  __device__ static void copy_slow(char* L, const OpTile& o, int64_t k0, int tid) {
    const char* base = o.X + o.row0 * EB;
    const int64_t rows_left = o.rows - o.row0;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, (o.K - 1) * o.ld_b + rows_left * EB);
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const int32_t rl = (int32_t)imin(rows_left, R);
    const int32_t kleft = (int32_t)imin(o.K - k0, KE);
    const uint32_t kb32 = (uint32_t)k0 * ld32;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int bidx = tid + NT * b;
      if (NBLK % NT != 0 && bidx >= NBLK) continue;
      const int rb = bidx % RB;
      const int kc = bidx / RB;
      uint32_t e[EPC][EPC];     // [k-row j][element i]
#pragma unroll
      for (int j = 0; j < EPC; ++j) {
        const int kk = kc * EPC + j;
#pragma unroll
        for (int i = 0; i < EPC; ++i) {
          const int r = rb * EPC + i;
          const bool ok = r < rl && kk < kleft;
          e[j][i] = buf_elem<EB>(rs, ok ? kb32 + (uint32_t)kk * ld32 + (uint32_t)(r * EB) : kOOB);
        }
      }
      // element i of the chunk for tile row rb*EPC+i holds k-row j: transpose
#pragma unroll
      for (int i = 0; i < EPC; ++i) {
        uint32_t t[EPC];
#pragma unroll
        for (int j = 0; j < EPC; ++j) t[j] = e[j][i];
        *(u32x4*)(L + lds_off(rb * EPC + i, kc)) = pack_chunk<EB>(t);
      }
    }
  }
};

// M/N-contiguous f16/bf16/e4m3 operand copied into LDS as it lies in memory:
// the stage holds KE k-rows of R elements (PITCH bytes each).  16-byte chunk
// c of k-row k sits at position c ^ tr_swizzle(k), which spreads the k-rows
// that one transposing read spans over distinct bank groups (see
// FragReader).  One wave copy fills 1 KiB = 64 / CPR k-rows, lane i
// fetching the chunk that the swizzle puts at its position.  k-rows past K
// and chunks wholly past M (N) are out-of-range offsets (zeros); a chunk that
// straddles M (N) reads row padding or the next k-row into tile rows that no
// output uses, and the buffer ends at the 4-byte word holding the last
// element, so no copy reads past it.
// Chunk swizzle of a transposed stage: 16-bit elements, 4 k-rows per read,
// XOR on chunk bits 2-3; 8-bit, 8 k-rows per read, XOR on bits 1-3 (k-rows
// of 16 or more chunks) or on bits 1-2 by k/2 (8 chunks: two k-rows share a
// 256-byte bank period).
template <int EB, int CPR>
__device__ __forceinline__ int tr_swizzle(int kr) {
  if constexpr (EB == 2) return 4 * (kr & 3);
  else if constexpr (CPR >= 16) return 2 * (kr & 7);
  else return 2 * ((kr >> 1) & 3);
}

template <int R, int EB, int NT>
struct MNMajorDMAStage {
  static constexpr int EPC = 16 / EB;
  static constexpr int KE = 128 / EB;        // k-rows per stage
  static constexpr int PITCH = R * EB;       // bytes per k-row
  static constexpr int CPR = PITCH / 16;     // chunks per k-row
  static constexpr int RPC = 1024 / PITCH;   // k-rows per 1 KiB copy
  static constexpr int NI = R / (NT / 8);    // 1 KiB copies per wave
  static_assert(((EB == 2 && CPR >= 16) || (EB == 1 && CPR >= 8)) && CPR <= 64 &&
                    R % (NT / 8) == 0, "tile rows");

  __device__ __forceinline__ static bool slow(const OpTile& o, int64_t) { return !o.aligned; }

  __device__ __forceinline__ static __amdgpu_buffer_rsrc_t rsrc(const OpTile& o) {
    const int64_t rows_left = o.rows - o.row0;
    return make_rsrc(o.X + o.row0 * EB, ((o.K - 1) * o.ld_b + rows_left * EB + 3) & ~(int64_t)3);
  }

  __device__ __forceinline__ void issue(char* L, const OpTile& o, int64_t k0, int tid) {
    const __amdgpu_buffer_rsrc_t rs = rsrc(o);
    const int wave = uniform32(tid >> 6);
    int lane = tid & 63;
    asm volatile("" : "+v"(lane));
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const uint32_t kb32 = (uint32_t)k0 * ld32;
    const int32_t rl = (int32_t)imin(o.rows - o.row0, R);
    const int32_t kleft = (int32_t)imin(o.K - k0, KE);
    const int lk = lane / CPR;                 // k-row inside the copy
    const int pc = lane % CPR;                 // chunk position inside the k-row
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int jj = wave * NI + j;
      const int kr = jj * RPC + lk;
      const int c = pc ^ tr_swizzle<EB, CPR>(kr);
      const bool ok = kr < kleft && c * EPC < rl;
      const uint32_t off = ok ? kb32 + (uint32_t)kr * ld32 + (uint32_t)(c * 16) : kOOB;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rs, (__attribute__((address_space(3))) void*)(L + jj * 1024), 16, (int)off, 0, 0, 0);
    }
  }

  __device__ __forceinline__ void commit(char*, int) const {}

  // Hoisted copies of whole iterations (see KMajorStage::prep): the k-row
  // offset k0*ld is the scalar offset; chunks wholly past M (N) keep an
  // out-of-range offset.
  uint32_t pre[NI];
  uint32_t pld;
  __amdgpu_buffer_rsrc_t prs;

  __device__ __forceinline__ void prep(const OpTile& o, int tid) {
    prs = rsrc(o);
    pld = (uint32_t)uniform32((int32_t)o.ld_b);
    const int wave = uniform32(tid >> 6);
    const int lane = tid & 63;
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const int32_t rl = (int32_t)imin(o.rows - o.row0, R);
    const int lk = lane / CPR;
    const int pc = lane % CPR;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int jj = wave * NI + j;
      const int kr = jj * RPC + lk;
      const int c = pc ^ tr_swizzle<EB, CPR>(kr);
      pre[j] = c * EPC < rl ? (uint32_t)kr * ld32 + (uint32_t)(c * 16) : kOOB;
    }
  }

  __device__ __forceinline__ void issue_pre(char* L, int64_t k0, int tid, bool on) const {
    const int wave = uniform32(tid >> 6);
    const int kb32 = uniform32((int32_t)((uint32_t)k0 * pld));
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int jj = wave * NI + j;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          prs, (__attribute__((address_space(3))) void*)(L + jj * 1024), 16,
          (int)(on ? pre[j] : kOOB), kb32, 0, 0);
    }
  }

  // Copy j alone (kb32: the iteration's scalar offset, as in issue_pre).
  __device__ __forceinline__ void issue_one(char* L, int kb32, int tid, bool on, int j) const {
    const int jj = uniform32(tid >> 6) * NI + j;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        prs, (__attribute__((address_space(3))) void*)(L + jj * 1024), 16,
        (int)(on ? pre[j] : kOOB), kb32, 0, 0);
  }
  __device__ __forceinline__ int k_offset(int64_t k0) const { return uniform32((int32_t)((uint32_t)k0 * pld)); }

  __device__ __forceinline__ static bool whole(const OpTile& o, int64_t k0) {
    return k0 + KE <= o.K;
  }

  // Any alignment: every element loaded on its own (out-of-range offsets
  // read as zero), packed into chunks written at their swizzled positions.
  __device__ static void copy_slow(char* L, const OpTile& o, int64_t k0, int tid) {
    constexpr int NCH = KE * CPR / NT;
    static_assert((KE * CPR) % NT == 0, "chunks per thread");
    const char* base = o.X + o.row0 * EB;
    const int64_t rows_left = o.rows - o.row0;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, (o.K - 1) * o.ld_b + rows_left * EB);
    const uint32_t ld32 = (uint32_t)o.ld_b;
    const uint32_t kb32 = (uint32_t)k0 * ld32;
    const int32_t rl = (int32_t)imin(rows_left, R);
    const int32_t kleft = (int32_t)imin(o.K - k0, KE);
    uint32_t e[NCH][EPC];
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
      const int idx = tid + t * NT;
      const int kr = idx / CPR, c = idx % CPR;
#pragma unroll
      for (int i = 0; i < EPC; ++i) {
        const int m = c * EPC + i;
        const bool ok = kr < kleft && m < rl;
        e[t][i] = buf_elem<EB>(rs, ok ? kb32 + (uint32_t)kr * ld32 + (uint32_t)(m * EB) : kOOB);
      }
    }
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
      const int idx = tid + t * NT;
      const int kr = idx / CPR, c = idx % CPR;
      *(u32x4*)(L + kr * PITCH + ((c ^ tr_swizzle<EB, CPR>(kr)) << 4)) = pack_chunk<EB>(e[t]);
    }
  }
};

#ifndef SK_MN_TR
#define SK_MN_TR 1
#endif
#ifndef SK_RING_TR
#define SK_RING_TR 0
#endif

// Stage of an operand: K-contiguous, M/N-contiguous through transposing LDS
// reads (TR), or M/N-contiguous transposed in registers.
template <bool KMAJOR, bool TR, int R, int EB, int NT, int KB>
struct StageSel;
template <bool TR, int R, int EB, int NT, int KB>
struct StageSel<true, TR, R, EB, NT, KB> {
#if SK_KMAJOR_DMA
  using type = KMajorStage<R, EB, NT, KB>;
#else
  using type = KMajorStageReg<R, EB, NT, KB>;
#endif
};
template <int R, int EB, int NT, int KB>
struct StageSel<false, true, R, EB, NT, KB> { using type = MNMajorDMAStage<R, EB, NT>; };
template <int R, int EB, int NT, int KB>
struct StageSel<false, false, R, EB, NT, KB> { using type = MNMajorStage<R, EB, NT>; };

// ---------------------------------------------------------------------------
// Matrix-core step: one 32-byte (f32/f16/bf16) or 64-byte (e4m3) slice of K
// for one 32x32 output block.  Lane l reads tile row (l mod 32); lanes
// 0-31 and 32-63 read adjacent 16-byte (32-byte for e4m3) pieces of K.
template <int DT>
struct Frag { u32x4 c[is_f8(DT) ? 2 : 1]; };
// MXFP8: the lane's 32 K-values and the E8M0 scale of their block
template <>
struct Frag<DT_MX8> { u32x4 c[2]; int32_t s; };
template <>
struct Frag<DT_MX8E5> { u32x4 c[2]; int32_t s; };
// MXFP4: the lane's 32 K-values (16 bytes) and the scale of their block
template <>
struct Frag<DT_MX4> { u32x4 c[1]; int32_t s; };
// MXFP6 (e2m3 / e3m2): the lane's 32 six-bit K-values (24 bytes, element j
// at bits 6j .. 6j+5) and the scale of their block
template <>
struct Frag<DT_MX6> { u32x2 c[3]; int32_t s; };
template <>
struct Frag<DT_MX6E3> { u32x2 c[3]; int32_t s; };

// Per-lane LDS byte offset, inside a 32-row block, of the 16-byte piece
// `chunk` of the lane's row (lane mod 32).  The swizzle repeats every 32
// rows, so the same offset serves every 32-row block.
__device__ __forceinline__ int frag_lane_off(int l32, int chunk) {
  return l32 * 128 + ((chunk ^ swz(l32)) << 4);
}

template <int DT>
__device__ __forceinline__ Frag<DT> read_frag(const char* L, const int (&lo)[2]) {
  Frag<DT> f;
  f.c[0] = *(const u32x4*)(L + lo[0]);
  if constexpr (is_f8(DT)) f.c[1] = *(const u32x4*)(L + lo[1]);
  return f;
}

template <int DT>
__device__ __forceinline__ void mma(v16f& acc, const Frag<DT>& a, const Frag<DT>& b) {
  if constexpr (DT == DT_F32) {
    // element-wise copy: a bit cast of a vector-element expression reads
    // element 0, so each element is first moved into a scalar
    const v4f af = __builtin_bit_cast(v4f, a.c[0]);
    const v4f bf = __builtin_bit_cast(v4f, b.c[0]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float x = af[e], y = bf[e];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc, 0, 0, 0);
    }
  } else if constexpr (DT == DT_F16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a.c[0]),
                                                 __builtin_bit_cast(v8h, b.c[0]), acc, 0, 0, 0);
  } else if constexpr (DT == DT_BF16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a.c[0]),
                                                  __builtin_bit_cast(v8bf, b.c[0]), acc, 0, 0,
                                                  0);
  } else if constexpr (is_f8pt(DT)) {
    v8i av = __builtin_bit_cast(v8i, a.c);
    v8i bv = __builtin_bit_cast(v8i, b.c);
    // operand format 0 (e4m3) or 1 (e5m2) for A and B; E8M0 scale 127 = 2^0
    constexpr int F = DT == DT_F8 ? 0 : 1;
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc, F, F, 0, 127, 0, 127);
  } else if constexpr (is_mx8(DT)) {
    // MXFP8: each lane's 32 K-values (one block of its row of A / column of
    // B) carry that block's E8M0 scale; the matrix core multiplies every
    // product by 2^(sa-127) * 2^(sb-127)
    v8i av = __builtin_bit_cast(v8i, a.c);
    v8i bv = __builtin_bit_cast(v8i, b.c);
    // operand format 0 (e4m3) or 1 (e5m2)
    constexpr int F = DT == DT_MX8 ? 0 : 1;
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc, F, F, 0, a.s, 0, b.s);
  } else if constexpr (is_mx6(DT)) {
    // MXFP6 (operand format 2, e2m3, or 3, e3m2): 24 bytes per lane, the
    // lane's block of 32 K-values with its scale (the lane half's 32 values
    // form one block: checked on the device against random operands with
    // per-half scales)
    constexpr int F = DT == DT_MX6 ? 2 : 3;
    const v8i av = {(int)a.c[0][0], (int)a.c[0][1], (int)a.c[1][0], (int)a.c[1][1],
                    (int)a.c[2][0], (int)a.c[2][1], 0, 0};
    const v8i bv = {(int)b.c[0][0], (int)b.c[0][1], (int)b.c[1][0], (int)b.c[1][1],
                    (int)b.c[2][0], (int)b.c[2][1], 0, 0};
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc, F, F, 0, a.s, 0, b.s);
  } else {
    // MXFP4 (operand format 4, e2m1): 16 bytes per lane, the lane's block
    // of 32 K-values with its scale
    const v8i av = {(int)a.c[0][0], (int)a.c[0][1], (int)a.c[0][2], (int)a.c[0][3], 0, 0, 0, 0};
    const v8i bv = {(int)b.c[0][0], (int)b.c[0][1], (int)b.c[0][2], (int)b.c[0][3], 0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc, 4, 4, 0, a.s, 0, b.s);
  }
}

// ---------------------------------------------------------------------------
template <int DT_, int LA_, int LB_, int BM_, int BN_, int WGM_, int NW_>
struct Cfg {
  static constexpr int DT = DT_, LA = LA_, LB = LB_, BM = BM_, BN = BN_, WGM = WGM_;
  static constexpr int NW = NW_, NT = 64 * NW_;     // waves, threads per workgroup
  static constexpr int EB = DT == DT_F32 ? 4 : (is_f8(DT) || DT == DT_MX4 || is_mx6(DT)) ? 1 : 2;
  static constexpr bool MX = is_mx(DT);              // E8M0 block scales in the stage
  static constexpr int SB = DT == DT_MX4 ? 8 : 4;    // MX: scale bytes per row and iteration
  // K elements per iteration (MX formats: bytes of K); an LDS stage row is
  // 128 bytes, of which MXFP6 (128 six-bit values) fills 96
  static constexpr int KE = is_mx6(DT) ? 96 : 128 / EB;
  static constexpr int WGN = NW / WGM;
  static constexpr int WM = BM / WGM, WN = BN / WGN; // per-wave tile
  static constexpr int FM = WM / 32, FN = WN / 32;   // 32x32 blocks per wave
  static constexpr int STEPS = (is_f8(DT) || is_mx6(DT)) ? 2 : 4;   // matrix-core steps per iteration
  static constexpr int BOFF = BM * 128;              // B tile offset in a stage
  // MX: after the tiles, SB scale bytes (the iteration's SB blocks of 32
  // K-values) per row of A then per column of B, copied in 256-byte blocks,
  // SNI per wave
  static constexpr int SCL_A = (BM + BN) * 128;
  static constexpr int SCL_B = SCL_A + SB * BM;
  static constexpr int SNI = MX ? ((BM + BN) * SB + NW * 256 - 1) / (NW * 256) : 0;
  static constexpr int STAGE = (BM + BN) * 128 + SNI * NW * 256;   // LDS bytes per stage
  // M/N-contiguous 16-bit operands are read with transposing LDS reads
  // (e4m3: tiles of at least 128 rows)
  static constexpr bool TR16 = (DT == DT_F16 || DT == DT_BF16) && SK_MN_TR && SK_KMAJOR_DMA;
  static constexpr bool TR8 = is_f8pt(DT) && SK_MN_TR && SK_KMAJOR_DMA;
  static constexpr bool TRA = LA == L_COL && (TR16 || (TR8 && BM >= 128));
  static constexpr bool TRB = LB == L_ROW && (TR16 || (TR8 && BN >= 128));
  // Both operands copied LDS-direct: as many stages as fit in 160 KiB (at
  // most 4); otherwise double-buffered register staging.
  static constexpr bool DMA = (LA == L_ROW || TRA) && (LB == L_COL || TRB) && SK_KMAJOR_DMA;
  static constexpr int NS_FIT = (160 * 1024) / STAGE;
  static constexpr int NSTAGE = DMA ? (NS_FIT > 4 ? 4 : NS_FIT) : 2;
  // Stages refilled right after their last read (mac_loop_ring) when both
  // operands are K-contiguous.  Transposing LDS reads take twice the LDS
  // read instructions per step and need the two-step look-ahead of
  // mac_loop_dma (three or more stages) or mac_loop_fast (two).
  static constexpr bool RING = DMA && ((!TRA && !TRB) || (SK_RING_TR && STEPS == 4));
  // fragments read three matrix-core steps ahead for K-contiguous 16-bit
  // tiles below 256x256 (against one step: +4-5% at 256x128, +3% at
  // 128x128); the 256x256 tile, at the register limit, reads one step ahead
  // (two cost it 13-23%), and FP8 iterations have two steps only
  static constexpr int RING_LA = (TRA || TRB) ? 2 : (STEPS == 4 && BM * BN < 256 * 256) ? 3 : 1;
  // e4m3 fragments read with transposing LDS reads on the 256x256 tile:
  // two steps of fragments (96 registers) beside the 128 accumulator
  // registers exceed the 256 a wave of two per SIMD has, so the two-stage
  // loop reads each step's fragments just before its MFMAs
  static constexpr bool FRAG_LOOKAHEAD = !(is_f8(DT) && (TRA || TRB) && FM * FN >= 8);
  // LDS-direct copies issued per wave for one iteration
  static constexpr int NLOADS = (BM + BN) / (NT / 8) + SNI;
  static_assert(!MX || (LA == L_ROW && LB == L_COL && (BM * SB) % 256 == 0),
                "MX: K-contiguous operands, A's scale rows end on a 256-byte block");
  // LDS read instructions per matrix-core step
  static constexpr int RD_K = is_f8(DT) ? 2 : is_mx6(DT) ? 3 : 1;   // K-contiguous fragment
  static constexpr int RD_T = is_f8(DT) ? 4 : 2;    // transposed fragment
  static constexpr int NRD = FM * (TRA ? RD_T : RD_K) + FN * (TRB ? RD_T : RD_K);
  static_assert(WGM * WGN == NW && FM >= 1 && FN >= 1, "wave grid");
  static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile");
  using StageA = typename StageSel<LA == L_ROW, TRA, BM, EB, NT, KE * EB>::type;
  using StageB = typename StageSel<LB == L_COL, TRB, BN, EB, NT, KE * EB>::type;
};

template <typename C>
struct Acc { v16f a[C::FM][C::FN]; };

// MX block scales of one tile into the stage: the SB scale bytes of an
// iteration (its SB blocks of 32 K-values: 4 for MXFP8, 8 for MXFP4) for
// each row of A, then for each column of B, in 4-byte LDS-direct copies.
// The stage holds them as [rows of A | columns of B] x SB bytes; copy j of
// wave w fills bytes 256 (w + NW j) .. +255 of that (lane l: 4 bytes at
// 256 (w + NW j) + 4l), so A's and B's rows never share a copy (BM * SB is
// a multiple of 256).  A copy past the last row reads nothing (out-of-range
// offset) and zeroes its bytes, so every wave issues the same number of
// copies per stage.  Rows past M or N read as zero scales (their elements
// are zero too).
template <typename C>
struct ScaleStage {
  static constexpr int NI = C::SNI;
  uint32_t voff[NI > 0 ? NI : 1];
  __amdgpu_buffer_rsrc_t prs[NI > 0 ? NI : 1];

  __device__ __forceinline__ void prep(const ProbDesc& pd, int64_t m0, int64_t n0, int tid) {
    if constexpr (C::MX) {
      const int wave = uniform32(tid >> 6);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int blk = wave + C::NW * j;              // 256-byte block of the stage
        const int f = 256 * blk + 4 * (tid & 63);      // this lane's byte
        const int r = f / C::SB, part = (f % C::SB) / 4;
        if (256 * blk < C::SB * C::BM) {
          prs[j] = make_rsrc((const char*)pd.sA + m0 * pd.ldsa, (pd.M - m0) * pd.ldsa);
          voff[j] = (uint32_t)r * (uint32_t)pd.ldsa + 4 * part;
        } else if (256 * blk < C::SB * (C::BM + C::BN)) {
          prs[j] = make_rsrc((const char*)pd.sB + n0 * pd.ldsb, (pd.N - n0) * pd.ldsb);
          voff[j] = (uint32_t)(r - C::BM) * (uint32_t)pd.ldsb + 4 * part;
        } else {
          prs[j] = make_rsrc((const char*)pd.sA, 0);
          voff[j] = kOOB;
        }
      }
    }
  }

  // Copy j of iteration k's scale bytes into the stage at L (on == false:
  // zeros).
  __device__ __forceinline__ void issue_one(char* L, int64_t k, int tid, bool on, int j) const {
    if constexpr (C::MX) {
      const int wave = uniform32(tid >> 6);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          prs[j],
          (__attribute__((address_space(3))) void*)(L + C::SCL_A + 256 * (wave + C::NW * j)), 4,
          (int)(on ? voff[j] : kOOB), uniform32((int32_t)(C::SB * k)), 0, 0);
    }
  }

  // All of iteration k's scale bytes.
  __device__ __forceinline__ void issue(char* L, int64_t k, int tid, bool on) const {
#pragma unroll
    for (int j = 0; j < NI; ++j) issue_one(L, k, tid, on, j);
  }
};

template <typename C>
__device__ __forceinline__ void zero_acc(Acc<C>& acc) {
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc.a[i][j][r] = 0.f;
}

// LDS stage -> matrix cores: acc += A_slab * B_slab for one iteration.
// Lanes 0-31 and 32-63 read adjacent 16-byte (e4m3: 32-byte) pieces of K of
// rows lane mod 32; step s covers pieces 2s, 2s+1 (e4m3: 4s .. 4s+3).
// Software-pipelined: the fragments of step s+1 are read from LDS before the
// matrix-core instructions of step s are issued, so LDS latency overlaps
// with the previous step's MFMAs.
// Fragments of one operand out of an LDS stage, for the wave's 32-row
// blocks i = 0 .. NB-1 starting at tile row `rowbase`.
//  * K-contiguous stage: lane l reads the 16-byte (e4m3: 32-byte) piece
//    2s + l/32 (4s + 2(l/32), +1) of row rowbase + 32i + l%32.
//  * Transposed 16-bit stage (TR): a ds_read_b64_tr_b16 gives lane i of
//    each 16-lane group the (i mod 4)-th 16-bit element of the 8 bytes
//    addressed by lane 4j + i/4 of its group, j = 0..3.  Lane p of group g
//    addresses k-row k0 + 8(g/2) + p/4 at rows 16(g mod 2) + 4(p mod 4) ..
//    +3 of the block, so lane l receives row l%32, k-rows k0 + 8(l/32) +
//    0..3: the first half of its MFMA operand; a second read at k0 + 4 gives
//    the other half.  With the stage's chunk swizzle, each group's four
//    k-rows lie in distinct 64-byte bank groups and the two groups reading
//    one block take the two halves of each, so a 32-lane half-wave reads all
//    64 banks once.
//  * Transposed e4m3 stage: ds_read_b64_tr_b8 gives lane i the (i mod 8)-th
//    byte of the 8 bytes addressed by lane 2j + i/8, j = 0..7.  Lane p of
//    group g addresses k-row k0 + 32(g/2) + p/2 at rows 16(g mod 2) +
//    8(p mod 2) .. +7, so lane l receives row l%32, k-rows k0 + 32(l/32) +
//    0..7; four reads (k0 + 8r) give its 32 k-values.  The swizzle puts a
//    group pair's eight k-rows on eight distinct 32-byte bank groups.
//  * MXFP8 (K-contiguous): the scaled 32x32x64 matrix-core step forms block
//    b (32 K-values) of a row from bytes 16b .. 16b+15 of both lane halves
//    and takes its scale from lane half b (gfx950 lane layout, checked on
//    the device with an all-ones operand and one lane's scale doubled).  So
//    lane l takes the 16-byte pieces 4s + l/32 and 4s + 2 + l/32: block b of
//    the step is the pieces 4s + 2b, 4s + 2b + 1, the iteration's block
//    2s + b, whose scale lane half b reads: byte 2s + l/32 of the 4 scale
//    bytes the stage holds for the lane's row, SREL bytes past the operand
//    (row r's bytes at 4r).
template <typename C, bool TR, int NB, int R, int SREL>
struct FragReader {
  static constexpr int PITCH = R * C::EB;    // bytes per k-row (TR stage)
  int off[NB];
  int l32, half;
  int sb;                                    // MX: the SB scale bytes of this lane's row (block 0)

  __device__ __forceinline__ void init(int rowbase, int lane) {
    l32 = lane & 31;
    half = lane >> 5;
    if constexpr (C::MX) sb = SREL + C::SB * (rowbase + l32);
    if constexpr (TR && C::EB == 2) {
      static_assert(C::STEPS == 4, "16 k-values per step");
      const int p = lane & 15, g = lane >> 4, j = p >> 2, q = p & 3;
      const int part = (8 * (g >> 1) + j) * PITCH + 16 * (2 * (g & 1) + (q >> 1)) + 8 * (q & 1);
#pragma unroll
      for (int i = 0; i < NB; ++i) off[i] = part + 64 * ((rowbase / 32 + i) ^ j);
    } else if constexpr (TR) {
      static_assert(C::EB == 1 && C::STEPS == 2 && PITCH >= 128, "64 k-values per step");
      const int p = lane & 15, g = lane >> 4, j = p >> 1, q = p & 1;
      const int sw = PITCH >= 256 ? j : (j >> 1);   // chunk-pair XOR of the swizzle
      const int part = (32 * (g >> 1) + j) * PITCH + 16 * (g & 1) + 8 * q;
#pragma unroll
      for (int i = 0; i < NB; ++i) off[i] = part + 32 * ((rowbase / 32 + i) ^ sw);
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i) off[i] = (rowbase + 32 * i) * 128;
    }
  }

  // Fragment of block i for matrix-core step s (16 k-values for 16-bit types).
  __device__ __forceinline__ Frag<C::DT> read(const char* op, int i, int s) const {
    Frag<C::DT> f;
    if constexpr (TR && C::EB == 1) {
      const char* p = op + off[i] + 64 * s * PITCH;
      v2i r[4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        r[t] = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
            (__attribute__((address_space(3))) v2i*)(p + 8 * t * PITCH));
      f.c[0] = u32x4{(uint32_t)r[0][0], (uint32_t)r[0][1], (uint32_t)r[1][0], (uint32_t)r[1][1]};
      f.c[1] = u32x4{(uint32_t)r[2][0], (uint32_t)r[2][1], (uint32_t)r[3][0], (uint32_t)r[3][1]};
    } else if constexpr (TR) {
      const char* p = op + off[i] + 16 * s * PITCH;
      const u32x2 lo = __builtin_bit_cast(
          u32x2, __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                     (__attribute__((address_space(3))) v4s*)(p)));
      const u32x2 hi = __builtin_bit_cast(
          u32x2, __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                     (__attribute__((address_space(3))) v4s*)(p + 4 * PITCH)));
      f.c[0] = u32x4{lo[0], lo[1], hi[0], hi[1]};
    } else if constexpr (is_mx6(C::DT)) {
      // MXFP6: step s covers K bytes 48s .. 48s+47 of the row, lane half h
      // the 24 bytes 48s + 24h .. (its block of 32 values), read as three
      // 8-byte pieces of the swizzled 16-byte chunks; scales as MXFP8
      const char* p = op + off[i];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int u = 6 * s + 3 * half + t;   // 8-byte unit of the row
        f.c[t] = *(const u32x2*)(p + frag_lane_off(l32, u >> 1) + 8 * (u & 1));
      }
      f.s = (s & 1) ? 0 : (int32_t)(*(const uint32_t*)(op + sb + 128 * i) >> (8 * half));
    } else {
      int lo[2];
      if constexpr (is_mx8(C::DT)) {
        lo[0] = frag_lane_off(l32, 4 * s + half);
        lo[1] = frag_lane_off(l32, 4 * s + 2 + half);
      } else if constexpr (is_f8(C::DT)) {
        lo[0] = frag_lane_off(l32, 4 * s + 2 * half);
        lo[1] = frag_lane_off(l32, 4 * s + 2 * half + 1);
      } else {
        lo[0] = frag_lane_off(l32, 2 * s + half);
        lo[1] = 0;
      }
      f = read_frag<C::DT>(op + off[i], lo);
      // MXFP8: the scale of step s is byte 2s + half of the row's 4 bytes;
      // the matrix core reads byte 0 of the operand.  Step 0 reads the 4
      // bytes once, shifted to this lane's half; step 1 takes them from step
      // 0.s fragment (in step_fenced), so each iteration reads the scales
      // of a fragment with one LDS instruction instead of two.
      if constexpr (is_mx8(C::DT))
        f.s = (s & 1) ? 0 : (int32_t)(*(const uint32_t*)(op + sb + 128 * i) >> (8 * half));
      // MXFP4: step s covers K bytes 32s .. 32s+31 of the row, lane half h
      // the 16-byte block 2s + h of them (the scaled matrix core takes a
      // lane half's 32 values as one block, with that half's scale: checked
      // on the device with an all-ones operand and one lane's scale doubled),
      // whose scale is byte 2s + h of the row's 8
      if constexpr (C::DT == DT_MX4)
        f.s = (int32_t)(*(const uint32_t*)(op + sb + 256 * i + 4 * (s >> 1)) >>
                        (8 * (2 * (s & 1) + half)));
    }
    return f;
  }
};

template <typename C>
using ReaderA = FragReader<C, C::TRA, C::FM, C::BM, C::SCL_A>;
template <typename C>
using ReaderB = FragReader<C, C::TRB, C::FN, C::BN, C::SCL_B - C::BOFF>;

template <typename C>
__device__ __forceinline__ void read_step(Frag<C::DT> (&fa)[C::FM], Frag<C::DT> (&fb)[C::FN],
                                          const ReaderA<C>& ra, const ReaderB<C>& rb,
                                          const char* opA, const char* opB, int s) {
#pragma unroll
  for (int i = 0; i < C::FM; ++i) fa[i] = ra.read(opA, i, s);
#pragma unroll
  for (int j = 0; j < C::FN; ++j) fb[j] = rb.read(opB, j, s);
}

// Fragment registers are triple-buffered: the reads for step s+2 go to the
// set that step s-1 used, so they never overwrite registers that in-flight
// MFMAs of step s are still reading, and they are interleaved between the
// MFMAs of step s (one LDS read, then a couple of MFMAs).
template <typename C>
__device__ __forceinline__ void compute_stage(Acc<C>& acc, const char* stage, int tid) {
  constexpr int NM = C::FM * C::FN;              // MFMAs per step
  const int wave = uniform32(tid >> 6);
  const int lane = tid & 63;
  ReaderA<C> ra;
  ReaderB<C> rb;
  ra.init((wave / C::WGN) * C::WM, lane);
  rb.init((wave % C::WGN) * C::WN, lane);
  const char* opA = stage;
  const char* opB = stage + C::BOFF;
  if constexpr (!C::FRAG_LOOKAHEAD) {
    // one set of fragment registers: each step's reads, then its MFMAs
#pragma unroll
    for (int s = 0; s < C::STEPS; ++s) {
      Frag<C::DT> ga[C::FM], gb[C::FN];
      read_step<C>(ga, gb, ra, rb, opA, opB, s);
#pragma unroll
      for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j) mma<C::DT>(acc.a[i][j], ga[i], gb[j]);
      __builtin_amdgcn_sched_barrier(0);
    }
    return;
  }
  Frag<C::DT> fa[3][C::FM], fb[3][C::FN];
  read_step<C>(fa[0], fb[0], ra, rb, opA, opB, 0);
  if (C::STEPS > 1) read_step<C>(fa[1], fb[1], ra, rb, opA, opB, 1);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s = 0; s < C::STEPS; ++s) {
    const int cur = s % 3;
    if (s + 2 < C::STEPS) read_step<C>(fa[(s + 2) % 3], fb[(s + 2) % 3], ra, rb, opA, opB, s + 2);
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
      for (int j = 0; j < C::FN; ++j) mma<C::DT>(acc.a[i][j], fa[cur][i], fb[cur][j]);
    if (s + 2 < C::STEPS) {
      // interleave: each LDS read followed by its share of the MFMAs
      constexpr int PER = NM / C::NRD > 0 ? NM / C::NRD : 1;
#pragma unroll
      for (int r = 0; r < C::NRD; ++r) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one DS read
        __builtin_amdgcn_sched_group_barrier(0x008, PER, 0); // MFMAs
      }
      __builtin_amdgcn_sched_group_barrier(0x008, NM, 0);    // the rest
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Fast MAC loop over iterations [kb, ke), all of which satisfy the fast
// staging conditions.  Double-buffered: the global loads of iteration k+1
// are in flight while the matrix cores work on iteration k out of the other
// LDS stage.  Starts and ends with a workgroup barrier.
template <typename C>
__device__ __forceinline__ void mac_loop_fast(Acc<C>& acc, const OpTile& oa, const OpTile& ob,
                                              int kb, int ke, char* lds, int tid,
                                              int32_t* cover_row) {
  typename C::StageA sa;
  typename C::StageB sb;
  sa.issue(lds, oa, (int64_t)kb * C::KE, tid);
  sb.issue(lds + C::BOFF, ob, (int64_t)kb * C::KE, tid);
  sa.commit(lds, tid);
  sb.commit(lds + C::BOFF, tid);
  __syncthreads();
  for (int k = kb; k < ke; ++k) {
    const int cur = (k - kb) & 1;
    const bool more = k + 1 < ke;
    char* nxt = lds + (cur ^ 1) * C::STAGE;
    if (more) {
      sa.issue(nxt, oa, (int64_t)(k + 1) * C::KE, tid);
      sb.issue(nxt + C::BOFF, ob, (int64_t)(k + 1) * C::KE, tid);
    }
    if (cover_row != nullptr && tid == 0) atomicAdd(cover_row + k, 1);
    compute_stage<C>(acc, lds + cur * C::STAGE, tid);
    if (more) {
      sa.commit(nxt, tid);
      sb.commit(nxt + C::BOFF, tid);
    }
    __syncthreads();   // waits for this iteration's copies into nxt
  }
}

// Waits until at most `n` vector-memory operations of this wave are
// outstanding (n <= 63); other counters are not waited for.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Multi-stage MAC loop for LDS-direct copies of both operands.
//
// Iteration k works on LDS stage k mod NSTAGE in two halves of its
// matrix-core steps.  During the first half the fragments of the second
// half are read; then, in the middle of the iteration, each wave waits until
// its copies for iteration k+1 have landed and the workgroup barrier makes
// every wave's copies visible (the MFMAs issued before it keep the matrix
// cores busy through the wait); the copies of iteration k+NSTAGE-1 are issued
// into the stage of iteration k-1, which every wave has finished reading;
// during the second half the fragments of iteration k+1's first half are
// read.  So no LDS latency is exposed at iteration boundaries, and
// NSTAGE-2 iterations plus half of one cover the copy latency.
// One matrix-core step with the LDS reads of another step woven in: the
// t-th read is issued right before the t-th MFMA, and nothing is allowed to
// move across the pairs, so reads always trail far enough behind the MFMAs
// that consume earlier fragments.
template <typename C>
__device__ __forceinline__ void step_with_reads(Acc<C>& acc, const Frag<C::DT> (&fa)[C::FM],
                                                const Frag<C::DT> (&fb)[C::FN],
                                                Frag<C::DT> (&ra)[C::FM], Frag<C::DT> (&rb)[C::FN],
                                                const ReaderA<C>& rda, const ReaderB<C>& rdb,
                                                const char* opA, const char* opB, int rs) {
  constexpr int NM = C::FM * C::FN;
  constexpr int NT_ = C::NRD > NM ? C::NRD : NM;
  read_step<C>(ra, rb, rda, rdb, opA, opB, rs);
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) mma<C::DT>(acc.a[i][j], fa[i], fb[j]);
  // pattern for the scheduler: (one DS read, one MFMA) pairs, then the rest
#pragma unroll
  for (int t = 0; t < NT_; ++t) {
    if (t < C::NRD) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    if (t < NM) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
  }
  __builtin_amdgcn_sched_barrier(0);
}


// Fragment n of a step in the order the MFMAs of the next step consume
// them (output blocks i-major): A0, B0 .. B(FN-1), A1 .. A(FM-1).
template <typename C>
__device__ __forceinline__ void read_frag_n(Frag<C::DT> (&ra)[C::FM], Frag<C::DT> (&rb)[C::FN],
                                            const ReaderA<C>& rda, const ReaderB<C>& rdb,
                                            const char* opA, const char* opB, int rs, int n) {
  if (n == 0) ra[0] = rda.read(opA, 0, rs);
  else if (n <= C::FN) rb[n - 1] = rdb.read(opB, n - 1, rs);
  else ra[n - C::FN] = rda.read(opA, n - C::FN, rs);
}

// One matrix-core step of the ring loop with the fragments of another step
// read and, optionally, the copies of a later iteration issued: MFMA t is
// followed by its even share of the fragment reads and copies, and a fence
// keeps each group in place.
template <typename C, int CB, int CE>
__device__ __forceinline__ void step_fenced(
    Acc<C>& acc, const Frag<C::DT> (&fa)[C::FM], const Frag<C::DT> (&fb)[C::FN],
    Frag<C::DT> (&ra)[C::FM], Frag<C::DT> (&rb)[C::FN], const ReaderA<C>& rda,
    const ReaderB<C>& rdb, const char* opA, const char* opB, int rs,
    const typename C::StageA& sa, const typename C::StageB& sb, const ScaleStage<C>& ss,
    char* dst, int64_t k0, bool on, int tid) {
  // copies CB .. CE-1 of the iteration's NA + NB (+1 MXFP8 scale copy): A's
  // first, then B's, then the scales'
  constexpr int NM = C::FM * C::FN;
  constexpr int NRF = C::FM + C::FN;
  constexpr int NA = C::StageA::NI;
  constexpr int NCP = CE - CB;
  int kba = 0, kbb = 0;
  if constexpr (NCP > 0) {
    kba = sa.k_offset(k0);
    kbb = sb.k_offset(k0);
  }
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    mma<C::DT>(acc.a[t / C::FN][t % C::FN], fa[t / C::FN], fb[t % C::FN]);
#pragma unroll
    for (int n = t * NRF / NM; n < (t + 1) * NRF / NM; ++n) {
      read_frag_n<C>(ra, rb, rda, rdb, opA, opB, rs, n);
      // MXFP8, step 1 read during step 0 of the same iteration: its scale
      // is byte 2 of step 0's (bytes 2s + half of the row's 4)
      if constexpr (is_mx8(C::DT) || is_mx6(C::DT)) {
        if (rs & 1) {
          if (n < 1) ra[0].s = fa[0].s >> 16;
          else if (n <= C::FN) rb[n - 1].s = fb[n - 1].s >> 16;
          else ra[n - C::FN].s = fa[n - C::FN].s >> 16;
        }
      }
    }
#pragma unroll
    for (int c = CB + t * NCP / NM; c < CB + (t + 1) * NCP / NM; ++c) {
      if (c < NA) sa.issue_one(dst, kba, tid, on, c);
      else if (c < NA + C::StageB::NI) sb.issue_one(dst + C::BOFF, kbb, tid, on, c - NA);
      else ss.issue_one(dst, k0 / C::KE, tid, on, c - NA - C::StageB::NI);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int N>
__device__ __forceinline__ void wait_vmcnt_le(int ahead_iters) {
  // wait until at most `ahead_iters` iterations' copies (N each) are in
  // flight; ahead_iters is 0 .. 3
  static_assert(3 * N < 64, "vmcnt range");
  if (ahead_iters >= 3) wait_vmcnt<3 * N>();
  else if (ahead_iters == 2) wait_vmcnt<2 * N>();
  else if (ahead_iters == 1) wait_vmcnt<N>();
  else wait_vmcnt<0>();
}

// Waits until every LDS access (and scalar load) of this wave has completed.
__device__ __forceinline__ void wait_lgkmcnt0() {
  __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
}

template <typename C>
__device__ __forceinline__ void mac_loop_dma(Acc<C>& acc, const OpTile& oa, const OpTile& ob,
                                             int kb, int ke, char* lds, int tid,
                                             int32_t* cover_row) {
  constexpr int NS = C::NSTAGE;
  constexpr int ST = C::STEPS;
  constexpr int HALF = ST / 2;
  typename C::StageA sa;
  typename C::StageB sb;
  const int wave = uniform32(tid >> 6);
  const int lane = tid & 63;
  ReaderA<C> rda;
  ReaderB<C> rdb;
  rda.init((wave / C::WGN) * C::WM, lane);
  rdb.init((wave % C::WGN) * C::WN, lane);

#pragma unroll
  for (int j = 0; j < NS - 1; ++j) {
    if (kb + j < ke) {
      sa.issue(lds + j * C::STAGE, oa, (int64_t)(kb + j) * C::KE, tid);
      sb.issue(lds + j * C::STAGE + C::BOFF, ob, (int64_t)(kb + j) * C::KE, tid);
    }
  }
  // copies of iteration kb landed (later ones may still be in flight)
  wait_vmcnt_le<C::NLOADS>((int)imin(NS - 2, ke - 1 - kb));
  __builtin_amdgcn_s_barrier();

  Frag<C::DT> fa[ST][C::FM], fb[ST][C::FN];
#pragma unroll
  for (int s = 0; s < HALF; ++s)
    read_step<C>(fa[s], fb[s], rda, rdb, lds, lds + C::BOFF, s);

  int slot = 0;
  for (int k = kb; k < ke; ++k) {
    const char* cur = lds + slot * C::STAGE;
    const bool more = k + 1 < ke;
    const int nslot = more ? (slot == NS - 1 ? 0 : slot + 1) : slot;
    const char* nxt = lds + nslot * C::STAGE;   // last iteration: harmless re-read
    if (cover_row != nullptr && tid == 0) atomicAdd(cover_row + k, 1);
    // first half: MFMAs of steps [0, HALF), reads of steps [HALF, ST)
#pragma unroll
    for (int s = 0; s < HALF; ++s)
      step_with_reads<C>(acc, fa[s], fb[s], fa[s + HALF], fb[s + HALF], rda, rdb, cur,
                         cur + C::BOFF, s + HALF);
    // copies of k+1 landed in every wave; the stage of k-1 is free
    wait_vmcnt_le<C::NLOADS>((int)imin(NS - 3, imax(ke - 2 - k, 0)));
    __builtin_amdgcn_s_barrier();
    if (k + NS - 1 < ke) {
      const int fill = slot == 0 ? NS - 1 : slot - 1;
      char* dst = lds + fill * C::STAGE;
      sa.issue(dst, oa, (int64_t)(k + NS - 1) * C::KE, tid);
      sb.issue(dst + C::BOFF, ob, (int64_t)(k + NS - 1) * C::KE, tid);
    }
    __builtin_amdgcn_sched_barrier(0);
    // second half: MFMAs of steps [HALF, ST), reads of the next iteration's
    // steps [0, HALF)
#pragma unroll
    for (int s = HALF; s < ST; ++s)
      step_with_reads<C>(acc, fa[s], fb[s], fa[s - HALF], fb[s - HALF], rda, rdb, nxt,
                         nxt + C::BOFF, s - HALF);
    slot = nslot;
  }
  __syncthreads();   // the stages are reused by the next segment
}

// Multi-stage MAC loop whose stages are refilled as soon as they have been
// read (LDS-direct copies of both operands; any number of stages >= 2).
//
// Fragments are read LA matrix-core steps ahead of the MFMAs that use them
// (LA = 1: two fragment buffers; LA = 2, for transposing reads, which take
// twice the LDS instructions, and LA = 3, for 16-bit tiles below 256x256:
// four), the reads of a step spread evenly over the MFMAs of the step that
// issues them.  Once the reads of the
// iteration's last step are issued (before step ST-LA), nothing of stage k
// is read again: each wave waits for its own LDS reads, then for its copies
// of iteration k+1, and the workgroup barrier makes both facts hold for
// every wave.  After it, the copies of iteration k+NSTAGE go into stage k,
// spread over the MFMAs of the iteration's last LA steps, while the first
// fragments of iteration k+1 are read.  A copy therefore has NSTAGE-1 whole
// iterations to land, which lets a tile whose stage fills more than half of
// the LDS (256x256: 64 KiB) keep one copy in flight behind every iteration
// with two stages.  Every iteration in [kb, ke) must be whole (K elements
// k*KE .. k*KE+KE-1 all below K): the copies' per-lane offsets are formed
// once (prep) and only rows past M or N are masked.
template <typename C>
__device__ __forceinline__ void mac_loop_ring(Acc<C>& acc, const OpTile& oa, const OpTile& ob,
                                              const ScaleStage<C>& ss, int kb, int ke,
                                              char* lds, int tid, int32_t* cover_row) {
  constexpr int NS = C::NSTAGE;
  constexpr int ST = C::STEPS;
  constexpr int LA = C::RING_LA;
  constexpr int NBUF = LA == 1 ? 2 : 4;
  constexpr int NCP = C::StageA::NI + C::StageB::NI + ScaleStage<C>::NI;
  static_assert(NS >= 2 && NS <= 4 && ST % NBUF == 0 && LA <= ST, "ring loop shape");
  typename C::StageA sa;
  typename C::StageB sb;
  sa.prep(oa, tid);
  sb.prep(ob, tid);
  const int wave = uniform32(tid >> 6);
  const int lane = tid & 63;
  ReaderA<C> rda;
  ReaderB<C> rdb;
  rda.init((wave / C::WGN) * C::WM, lane);
  rdb.init((wave % C::WGN) * C::WN, lane);

#pragma unroll
  for (int j = 0; j < NS; ++j) {
    if (kb + j < ke) {
      sa.issue_pre(lds + j * C::STAGE, (int64_t)(kb + j) * C::KE, tid, true);
      sb.issue_pre(lds + j * C::STAGE + C::BOFF, (int64_t)(kb + j) * C::KE, tid, true);
      ss.issue(lds + j * C::STAGE, kb + j, tid, true);
    }
  }
  // copies of iteration kb landed in every wave (later ones may be in flight)
  wait_vmcnt_le<C::NLOADS>((int)imin(NS - 1, ke - 1 - kb));
  __builtin_amdgcn_s_barrier();

  Frag<C::DT> fa[NBUF][C::FM], fb[NBUF][C::FN];
#pragma unroll
  for (int s0 = 0; s0 < LA; ++s0)
#pragma unroll
    for (int n = 0; n < C::FM + C::FN; ++n)
      read_frag_n<C>(fa[s0], fb[s0], rda, rdb, lds, lds + C::BOFF, s0, n);

  int slot = 0;
  for (int k = kb; k < ke; ++k) {
    char* cur = lds + slot * C::STAGE;
    const bool more = k + 1 < ke;
    const int nslot = slot == NS - 1 ? 0 : slot + 1;
    // the last iteration's look-ahead re-reads its own (landed) stage
    const char* nxt = more ? lds + nslot * C::STAGE : cur;
    if (cover_row != nullptr && tid == 0) atomicAdd(cover_row + k, 1);
    // iteration k+NS refills stage k (past ke the copies read nothing and
    // zero the stage, which no later iteration of this loop reads)
    const int64_t kn0 = (int64_t)(k + NS) * C::KE;
    const bool refill = k + NS < ke;
#pragma unroll
    for (int s = 0; s < ST; ++s) {
      const int rs = s + LA < ST ? s + LA : s + LA - ST;     // step read ahead
      const char* src = s + LA < ST ? cur : nxt;
      if (s == ST - LA) {
        // stage k is read (this wave's reads completed), and the copies of
        // iteration k+1 landed (at most NS-2 later iterations in flight)
        wait_lgkmcnt0();
        wait_vmcnt_le<C::NLOADS>((int)imin(NS - 2, imax(ke - 2 - k, 0)));
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
      }
      if (s < ST - LA)
        step_fenced<C, 0, 0>(acc, fa[s % NBUF], fb[s % NBUF], fa[(s + LA) % NBUF],
                             fb[(s + LA) % NBUF], rda, rdb, src, src + C::BOFF, rs, sa, sb, ss, cur,
                             kn0, refill, tid);
      else if (LA == 3) {
        // the refill's copies spread over the three steps after the barrier
        if (s == ST - 3)
          step_fenced<C, 0, NCP / 3>(acc, fa[s % NBUF], fb[s % NBUF], fa[(s + LA) % NBUF],
                                     fb[(s + LA) % NBUF], rda, rdb, src, src + C::BOFF, rs, sa,
                                     sb, ss, cur, kn0, refill, tid);
        else if (s == ST - 2)
          step_fenced<C, NCP / 3, 2 * NCP / 3>(acc, fa[s % NBUF], fb[s % NBUF],
                                               fa[(s + LA) % NBUF], fb[(s + LA) % NBUF], rda,
                                               rdb, src, src + C::BOFF, rs, sa, sb, ss, cur, kn0,
                                               refill, tid);
        else
          step_fenced<C, 2 * NCP / 3, NCP>(acc, fa[s % NBUF], fb[s % NBUF], fa[(s + LA) % NBUF],
                                           fb[(s + LA) % NBUF], rda, rdb, src, src + C::BOFF, rs,
                                           sa, sb, ss, cur, kn0, refill, tid);
      } else if (LA == 1 || s == ST - 2)
        step_fenced<C, 0, (LA == 1 ? NCP : NCP / 2)>(
            acc, fa[s % NBUF], fb[s % NBUF], fa[(s + LA) % NBUF], fb[(s + LA) % NBUF], rda, rdb,
            src, src + C::BOFF, rs, sa, sb, ss, cur, kn0, refill, tid);
      else
        step_fenced<C, NCP / 2, NCP>(acc, fa[s % NBUF], fb[s % NBUF], fa[(s + LA) % NBUF],
                                     fb[(s + LA) % NBUF], rda, rdb, src, src + C::BOFF, rs, sa,
                                     sb, ss, cur, kn0, refill, tid);
    }
    slot = nslot;
  }
  __syncthreads();   // the stages are reused by the next segment
}

// One iteration through the element-wise path (edges the fast path cannot
// take).  Called after a barrier; ends with one.
template <typename C>
__device__ __forceinline__ void stage_slow(const OpTile& oa, const OpTile& ob,
                                                     int64_t k0, char* lds, int tid) {
  if (C::StageA::slow(oa, k0)) C::StageA::copy_slow(lds, oa, k0, tid);
  else {
    typename C::StageA sa;
    sa.issue(lds, oa, k0, tid);
    sa.commit(lds, tid);
  }
  if (C::StageB::slow(ob, k0)) C::StageB::copy_slow(lds + C::BOFF, ob, k0, tid);
  else {
    typename C::StageB sb;
    sb.issue(lds + C::BOFF, ob, k0, tid);
    sb.commit(lds + C::BOFF, tid);
  }
}

// MAC loop over iterations [kb, ke) of the tile whose first output element
// is (m0, n0): acc += A[m0:, k-slab] * B[k-slab, n0:] for each iteration.
template <typename C>
__device__ __forceinline__ void mac_loop(Acc<C>& acc, const ProbDesc& pd, int64_t m0,
                                         int64_t n0, int kb, int ke, char* lds, int tid,
                                         int32_t* cover_row) {
  constexpr int EB = C::EB;
  const OpTile oa{(const char*)pd.A, pd.lda * EB, m0, pd.M, pd.K, pd.aligned != 0};
  const OpTile ob{(const char*)pd.B, pd.ldb * EB, n0, pd.N, pd.K, pd.aligned != 0};
  // Fast iterations are a prefix [kb, kf): an unaligned problem or a tile
  // with a partial row chunk has none; a K that ends inside a chunk makes
  // only the last iteration slow.
  int kf = ke;
  if (C::StageA::slow(oa, (int64_t)kb * C::KE) || C::StageB::slow(ob, (int64_t)kb * C::KE))
    kf = kb;
  else if (ke > kb && (C::StageA::slow(oa, (int64_t)(ke - 1) * C::KE) ||
                       C::StageB::slow(ob, (int64_t)(ke - 1) * C::KE)))
    kf = ke - 1;
  // the ring loop takes whole iterations only: a last iteration that ends
  // past K goes to the masked per-iteration path below
  if constexpr (C::RING)
    if (kf > kb && !C::StageA::whole(oa, (int64_t)(kf - 1) * C::KE)) --kf;
  if constexpr (C::MX) {
    // MX launches are K-contiguous, 16-byte aligned and whole iterations
    // (K a multiple of 128 MXFP8 / 256 MXFP4 elements; checked on the
    // host): every iteration is whole and fast
    ScaleStage<C> ss;
    ss.prep(pd, m0, n0, tid);
    if (ke > kb) mac_loop_ring<C>(acc, oa, ob, ss, kb, ke, lds, tid, cover_row);
    return;
  }
  if (kf > kb) {
    if constexpr (C::RING) {
      const ScaleStage<C> none{};
      mac_loop_ring<C>(acc, oa, ob, none, kb, kf, lds, tid, cover_row);
    } else if constexpr (C::DMA && C::NSTAGE >= 3) {
      mac_loop_dma<C>(acc, oa, ob, kb, kf, lds, tid, cover_row);
    } else {
      mac_loop_fast<C>(acc, oa, ob, kb, kf, lds, tid, cover_row);
    }
  }
  for (int k = kf; k < ke; ++k) {
    stage_slow<C>(oa, ob, (int64_t)k * C::KE, lds, tid);
    __syncthreads();
    if (cover_row != nullptr && tid == 0) atomicAdd(cover_row + k, 1);
    compute_stage<C>(acc, lds, tid);
    __syncthreads();
  }
}

// Accumulator layout of a 32x32 block: register r of lane l holds
// row 8*(r/4) + 4*(l/32) + (r%4), column l%32.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Activations of the fused epilogue, in FP32, written for compact code (the
// epilogue is unrolled over every accumulator, so each instruction here is
// repeated per element): exp via the hardware exp2 (v_exp_f32) and
// reciprocals via v_rcp_f32, both accurate to about one ulp.
__device__ __forceinline__ float fast_exp(float x) {
  return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}

// erfc(z) for z >= 0 by the rational Chebyshev fit of Numerical Recipes in C
// (2nd ed., section 6.2, "erfcc"): fractional error below 1.2e-7 for every z.
__device__ __forceinline__ float erfc_nonneg(float z) {
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.5f, z, 1.f));
  float p = 0.17087277f;
  p = __builtin_fmaf(p, t, -0.82215223f);
  p = __builtin_fmaf(p, t, 1.48851587f);
  p = __builtin_fmaf(p, t, -1.13520398f);
  p = __builtin_fmaf(p, t, 0.27886807f);
  p = __builtin_fmaf(p, t, -0.18628806f);
  p = __builtin_fmaf(p, t, 0.09678418f);
  p = __builtin_fmaf(p, t, 0.37409196f);
  p = __builtin_fmaf(p, t, 1.00002368f);
  p = __builtin_fmaf(p, t, -1.26551223f);
  return t * fast_exp(__builtin_fmaf(-z, z, p));
}

// GELU(v) = v Phi(v) = (v/2) erfc(-v/sqrt 2): for v < 0 directly, for v >= 0
// as v - (v/2) erfc(v/sqrt 2), so no 1 + erf cancellation for either sign.
__device__ __forceinline__ float gelu(float v) {
  const float h = 0.5f * v * erfc_nonneg(__builtin_fabsf(v) * 0.70710678118654752f);
  return v < 0.f ? h : v - h;
}

__device__ __forceinline__ float silu(float v) {
  return v * __builtin_amdgcn_rcpf(1.f + fast_exp(-v));
}

template <typename C, int DTC, bool EX>
__device__ __forceinline__ void epilogue_t(const Acc<C>& acc, const ProbDesc& pd, int64_t m0,
                                           int64_t n0, int tid) {
  constexpr int ES = DTC == DT_F32 ? 4 : 2;           // output element size
  constexpr int NB = C::FM * C::FN;                   // 32x32 blocks per wave
  const int wave = uniform32(tid >> 6);
  int lane = tid & 63;
  // Keep the per-lane offsets below inside the epilogue (otherwise they are
  // hoisted out of the work loop and occupy registers during the MAC loop).
  asm volatile("" : "+v"(lane));
  const int wr = (wave / C::WGN) * C::WM + 4 * (lane >> 5);
  const int wc = (wave % C::WGN) * C::WN + (lane & 31);
  const float alpha = pd.alpha_s, beta = pd.beta;
  const int64_t rows_left = pd.M - m0, cols_left = pd.N - n0;
  const int32_t rl = (int32_t)imin(rows_left, C::BM), cl = (int32_t)imin(cols_left, C::BN);
  const int64_t tile_off = (m0 * pd.ldc + n0) * ES;
  const int64_t extent = ((rows_left - 1) * pd.ldc + cols_left) * ES;
  const __amdgpu_buffer_rsrc_t out = make_rsrc((const char*)pd.Cout + tile_off, extent);
  const bool use_cin = beta != 0.f;
  const __amdgpu_buffer_rsrc_t in =
      make_rsrc((const char*)(use_cin ? pd.Cin : pd.Cout) + tile_off, extent);
  const uint32_t ldc_b = (uint32_t)(pd.ldc * ES);
  const uint32_t lane_off = (uint32_t)wr * ldc_b + (uint32_t)(wc * ES);
  // byte offset of register r of block b (kOOB outside the matrix)
  auto elem_off = [&](int b, int r) -> int {
    const int i = b / C::FN, j = b % C::FN;
    const int dr = i * 32 + 8 * (r >> 2) + (r & 3);   // row offset from wr
    const bool ok = wr + dr < rl && wc + j * 32 < cl;
    return (int)(ok ? lane_off + ((uint32_t)dr * ldc_b + (uint32_t)(j * 32 * ES)) : kOOB);
  };
  auto load_cin = [&](int b, float (&dst)[16]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int off = elem_off(b, r);
      if constexpr (DTC == DT_F32)
        dst[r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(in, off, 0, 0));
      else if constexpr (DTC == DT_F16)
        dst[r] = (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(in, off, 0, 0));
      else
        dst[r] = __builtin_bit_cast(float, (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(in, off, 0, 0) << 16);
    }
  };
  // fused epilogue: the bias of this lane's column in each 32-column block
  float bias[C::FN];
  int act = SK_ACT_NONE;
  if constexpr (EX) {
    act = pd.act;
    const __amdgpu_buffer_rsrc_t br =
        make_rsrc((const char*)(pd.bias ? (const void*)pd.bias : pd.Cout) + n0 * 4,
                  pd.bias ? cols_left * 4 : 0);
#pragma unroll
    for (int j = 0; j < C::FN; ++j)   // columns past N read 0 (and are dropped)
      bias[j] = __builtin_bit_cast(
          float, __builtin_amdgcn_raw_buffer_load_b32(br, (wc + 32 * j) * 4, 0, 0));
  }
  // C_in of block b+1 is loaded while block b is finished, so only the first
  // block's load latency is exposed (plain epilogue; the fused one loads each
  // block's C_in just before it, which keeps its registers below the spill
  // point of the 256x256 kernels).
  float cin[2][16];
  if (use_cin && !EX) load_cin(0, cin[0]);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if constexpr (EX) {
      if (use_cin) load_cin(b, cin[b & 1]);
    } else {
      if (use_cin && b + 1 < NB) load_cin(b + 1, cin[(b + 1) & 1]);
    }
    __builtin_amdgcn_sched_barrier(0);
    const int i = b / C::FN, j = b % C::FN;
    float v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r)
      v[r] = use_cin ? __builtin_fmaf(alpha, acc.a[i][j][r], beta * cin[b & 1][r])
                     : alpha * acc.a[i][j][r];
    if constexpr (EX) {
      // one uniform branch per block (not per element) keeps each
      // activation's code together
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] += bias[j];
      if (act == SK_ACT_RELU) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = v[r] < 0.f ? 0.f : v[r];
      } else if (act == SK_ACT_GELU) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = gelu(v[r]);
      } else if (act == SK_ACT_SILU) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = silu(v[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int off = elem_off(b, r);
      if constexpr (DTC == DT_F32)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v[r]), out, off, 0, 0);
      else if constexpr (DTC == DT_F16)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (_Float16)v[r]), out, off, 0, 0);
      else
        __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16_rne(v[r]), out, off, 0, 0);
    }
    // one block at a time: keeps the scheduler from gathering all loads and
    // stores of the tile and the registers they would need
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Epilogue: out = alpha_s * acc + beta * Cin (one FP32 fma when beta != 0),
// then, when the problem asks for it, + bias[column] and the activation, all
// in FP32; rounded to nearest-even in the output type; out-of-range elements
// get an offset past the buffer and are dropped by the hardware.
template <typename C, bool EX>
__device__ __forceinline__ void epilogue_c(const Acc<C>& acc, const ProbDesc& pd, int dtype_c,
                                           int64_t m0, int64_t n0, int tid) {
  if (dtype_c == DT_F32) epilogue_t<C, DT_F32, EX>(acc, pd, m0, n0, tid);
  else if (dtype_c == DT_F16) epilogue_t<C, DT_F16, EX>(acc, pd, m0, n0, tid);
  else epilogue_t<C, DT_BF16, EX>(acc, pd, m0, n0, tid);
}

template <typename C>
__device__ __forceinline__ void epilogue(const Acc<C>& acc, const ProbDesc& pd, int dtype_c,
                                         int64_t m0, int64_t n0, int tid) {
  if (pd.bias != nullptr || pd.act != SK_ACT_NONE)
    epilogue_c<C, true>(acc, pd, dtype_c, m0, n0, tid);
  else
    epilogue_c<C, false>(acc, pd, dtype_c, m0, n0, tid);
}

// Partial tile <-> workspace slot.  Thread t owns the same accumulator
// registers in every workgroup, so the slot is laid out
// [block (i,j)][register quad][thread] x float4: each store or load
// instruction of a wave touches 1 KiB of contiguous memory.
//
// Partial tiles move at device scope (the sc1 cache-policy bit): such
// stores are acknowledged only once they are visible to every XCD, and such
// loads never return a stale line of the reader's own L2.  Publishing and
// consuming a partial therefore needs no cache-wide operation; an
// agent-scope fence would instead write back and invalidate the L2 of the
// workgroup's XCD, dropping the A/B panels that the other workgroups there
// are streaming.
constexpr int kCpolDevice = 16;   // sc1

template <typename C>
__device__ __forceinline__ void store_partial(const Acc<C>& acc, float* slot, int tid) {
  asm volatile("" : "+v"(tid));   // addresses are formed here, not hoisted
  const __amdgpu_buffer_rsrc_t rs = make_rsrc((const char*)slot, (int64_t)C::BM * C::BN * 4);
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v4f v = {acc.a[i][j][4 * q], acc.a[i][j][4 * q + 1], acc.a[i][j][4 * q + 2],
                 acc.a[i][j][4 * q + 3]};
        const int off = (((i * C::FN + j) * 4 + q) * C::NT + tid) * 16;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rs, off, 0,
                                               kCpolDevice);
        __builtin_amdgcn_sched_barrier(0);
      }
}

template <typename C>
__device__ __forceinline__ void add_partial(Acc<C>& acc, const float* slot, int tid) {
  constexpr int NB = C::FM * C::FN;
  asm volatile("" : "+v"(tid));   // addresses are formed here, not hoisted
  const __amdgpu_buffer_rsrc_t rs = make_rsrc((const char*)slot, (int64_t)C::BM * C::BN * 4);
  auto load_blk = [&](int b, u32x4 (&dst)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      dst[q] = __builtin_amdgcn_raw_buffer_load_b128(rs, ((b * 4 + q) * C::NT + tid) * 16, 0,
                                                     kCpolDevice);
  };
  // block b+1 is in flight while block b is added
  u32x4 buf[2][4];
  load_blk(0, buf[0]);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (b + 1 < NB) load_blk(b + 1, buf[(b + 1) & 1]);
    __builtin_amdgcn_sched_barrier(0);
    const int i = b / C::FN, j = b % C::FN;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const v4f v = __builtin_bit_cast(v4f, buf[b & 1][q]);
#pragma unroll
      for (int e = 0; e < 4; ++e) acc.a[i][j][4 * q + e] += v[e];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ---------------------------------------------------------------------------
// Tile lookup.
struct TileRef {
  int32_t p;          // problem
  int64_t t;          // global tile
  int64_t J;          // first global Stream-K iteration of the tile
  int32_t tr, tc;     // tile row / column inside the problem
};

__device__ __forceinline__ int32_t find_problem(const KParams& P, int64_t key, bool by_iter) {
  // largest p with start[p] <= key
  int32_t lo = 0, hi = P.nprobs - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    int64_t s = by_iter ? P.group[mid].iter_start : P.group[mid].tile_start;
    if (s <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ const ProbDesc& prob_of(const KParams& P, int32_t p) {
  return P.group ? P.group[p] : P.prob;
}

// Global Stream-K iteration -> tile containing it.
__device__ __forceinline__ TileRef tile_of_iter(const KParams& P, int64_t it) {
  TileRef r;
  r.p = P.group ? find_problem(P, it, true) : 0;
  const ProbDesc& pd = prob_of(P, r.p);
  int64_t u = (it - pd.iter_start) / pd.I;
  r.t = pd.tile_start + u;
  r.J = pd.iter_start + u * pd.I;
  tile_coords(u, pd.tm, pd.tn, P.group_m, &r.tr, &r.tc);
  return r;
}

// Global tile index -> tile.
__device__ __forceinline__ TileRef tile_of_index(const KParams& P, int64_t t) {
  TileRef r;
  r.p = P.group ? find_problem(P, t, false) : 0;
  const ProbDesc& pd = prob_of(P, r.p);
  int64_t u = t - pd.tile_start;
  r.t = t;
  r.J = 0;
  tile_coords(u, pd.tm, pd.tn, P.group_m, &r.tr, &r.tc);
  return r;
}

__device__ __forceinline__ void trace_segment(const KParams& P, int64_t x, const TileRef& tr,
                                              int kb, int ke, int role, int npeers) {
  if (P.trace == nullptr || threadIdx.x != 0) return;
  int64_t idx = atomicAdd((unsigned long long*)P.trace_count, 1ull);
  if (idx < P.trace_cap) {
    sk_segment s;
    s.wg = (int32_t)x;
    s.problem = prob_of(P, tr.p).user_index;
    s.tile = (int32_t)tr.t;
    s.tile_m = tr.tr;
    s.tile_n = tr.tc;
    s.k_begin = kb;
    s.k_end = ke;
    s.role = role;
    s.npeers = npeers;
    P.trace[idx] = s;
  }
}

// Fixup wait: one wavefront (lane 0 of wave 0) polls the token of peer
// workgroup y with device-scope loads, backing off with s_sleep, until it
// holds this launch's tag; the workgroup barrier then orders every wave's
// (device-scope) reads of y's partial slot after the poll that saw the tag.
// The poll is bounded: past spin_limit it raises the error word instead of
// hanging.
__device__ __forceinline__ void wait_token(const KParams& P, const uint32_t* token,
                                           uint32_t tag) {
  if (threadIdx.x == 0) {
    int64_t n = 0;
    while (__hip_atomic_load(token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tag) {
      __builtin_amdgcn_s_sleep(2);
      if (++n > P.spin_limit) {
        __hip_atomic_store(P.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}

// Publish a partial tile: each thread waits until its device-scope stores
// are acknowledged (visible on every XCD), the workgroup barrier collects
// all threads, then one thread writes the launch's tag into the
// workgroup's own token (one writer per token and launch: no atomics).
__device__ __forceinline__ void publish_token(uint32_t* token, uint32_t tag) {
  wait_vmcnt<0>();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(token, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tag of the running launch: the workspace's epoch word plus one, skipping 0
// (the value a freshly initialised token holds).
__device__ __forceinline__ uint32_t launch_tag(const uint32_t* epoch) {
  const uint32_t e = __hip_atomic_load(epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return e == 0xffffffffu ? 1u : e + 1u;
}

// End of a workgroup of a launch with split tiles: the last of the g
// workgroups to get here advances the epoch to this launch's tag and clears
// the counter.  Thread 0 waits for its own epoch load (and every other
// memory operation of its wave) before it counts itself, so the epoch only
// moves after every workgroup of the launch has read it.
__device__ __forceinline__ void end_of_launch(const KParams& P, uint32_t tag) {
  if (threadIdx.x == 0) {
    wait_vmcnt<0>();
    const uint32_t old = __hip_atomic_fetch_add(P.done, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old == (uint32_t)(P.g - 1)) {
      __hip_atomic_store(P.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(P.epoch, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// One work item of a workgroup: a Stream-K segment or a data-parallel tile.
struct Item {
  TileRef tr;
  int kb, ke, role, npeers;
};

template <typename C>
__global__ __launch_bounds__(C::NT, 1) void sk_gemm_kernel(KParams P) {
  __shared__ __attribute__((aligned(16))) char lds[C::NSTAGE * C::STAGE];
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;

  // Work of this workgroup: Stream-K iterations [it, e), then one
  // data-parallel tile per round of g tiles below T, taken at position x in
  // even rounds and g-1-x in odd ones (a tile list sorted longest first then
  // evens out).  The baseline grid runs exactly one data-parallel tile per
  // workgroup.
  int64_t x, it, e, dp_t, dp_step, dp_r = 0;
  if (P.dp_grid) {
    x = logical_id(b, P.T, P.xcd_remap, 0);
    it = e = 0;
    dp_t = x;
    dp_step = P.T;
  } else {
    x = logical_id(b, P.g, P.xcd_remap, P.reverse_ids);
    it = range_begin(x, P.q, P.rho);
    e = it + P.q + (x < P.rho ? 1 : 0);
    dp_t = P.S + x;
    dp_step = P.g;
  }
  // launch tag of the fixup tokens (only lane 0 of wave 0 polls and writes)
  const bool fixup = !P.dp_grid && P.S > 0;
  const uint32_t tag = fixup && tid == 0 ? launch_tag(P.epoch) : 0u;

  while (true) {
    Item w;
    ProbDesc pd;
    if (it < e) {
      // Stream-K segment: PARTIAL (first only), FULL*, FINISH (last only).
      w.tr = tile_of_iter(P, it);
      pd = prob_of(P, w.tr.p);
      w.kb = (int)(it - w.tr.J);
      w.ke = (int)(imin(e, w.tr.J + pd.I) - w.tr.J);
      w.npeers = 0;
      if (w.kb > 0) w.role = R_PARTIAL;
      else if (w.ke == pd.I) w.role = R_FULL;
      else {
        w.role = R_FINISH;
        w.npeers = (int)(iter_owner(w.tr.J + pd.I - 1, P.q, P.rho) - x);
      }
      it = w.tr.J + w.ke;
    } else if (dp_t < P.T) {
      w.tr = tile_of_index(P, dp_t);
      pd = prob_of(P, w.tr.p);
      w.kb = 0;
      w.ke = pd.I;
      w.role = R_DP;
      w.npeers = 0;
      if (P.dp_grid) {
        dp_t += dp_step;
      } else {
        ++dp_r;
        dp_t = P.S + dp_r * P.g + ((dp_r & 1) ? P.g - 1 - x : x);
      }
    } else {
      break;
    }
    trace_segment(P, x, w.tr, w.kb, w.ke, w.role, w.npeers);

    const int64_t m0 = (int64_t)w.tr.tr * C::BM, n0 = (int64_t)w.tr.tc * C::BN;
    Acc<C> acc;
    zero_acc(acc);
    int32_t* cover = P.cover ? P.cover + w.tr.t * P.cover_stride : nullptr;
    mac_loop<C>(acc, pd, m0, n0, w.kb, w.ke, lds, tid, cover);

    if (w.role == R_PARTIAL) {
      store_partial<C>(acc, P.slots + x * (int64_t)(C::BM * C::BN), tid);
      if (P.partial_delay > 0) {
        if (tid == 0)
          for (int d = 0; d < P.partial_delay; ++d) __builtin_amdgcn_s_sleep(1);
        __syncthreads();
      }
      publish_token(P.tokens + x, tag);
      continue;
    }
    if (w.role == R_FINISH) {
      // peers x+1 .. x+npeers in increasing id, each added once its token
      // carries this launch's tag
      for (int y = 1; y <= w.npeers; ++y) {
        wait_token(P, P.tokens + x + y, tag);
        add_partial<C>(acc, P.slots + (x + y) * (int64_t)(C::BM * C::BN), tid);
      }
    }
    epilogue<C>(acc, pd, P.dtype_c, m0, n0, tid);
  }
  if (fixup) end_of_launch(P, tag);
}

}  // namespace sk
