// Out-of-place matrix transpose for operand packing: gives an M- or
// N-major GEMM operand a K-contiguous copy, which the GEMM kernels read with
// plain 16-byte LDS reads instead of transposing ones (two instructions per
// 16-bit fragment, four per e4m3 fragment).
//
// One workgroup of 256 threads moves 64 x 64-element tiles through LDS:
// each thread reads 8 bytes along an input row and writes 8 bytes along an
// output row, so both sides of HBM see whole 64-byte row pieces per lane
// group.  The LDS tile's rows are padded by 4 bytes, an odd number of
// 4-byte banks, so the column reads of the write phase hit distinct banks.
// Edge tiles and operands whose rows are not 8-byte aligned go element by
// element.  Elements are copied bit for bit (1, 2 or 4 bytes).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "streamk.h"

namespace sk {
namespace {

constexpr int kTile = 64;
constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void transpose_kernel(const T* __restrict__ in,
                                                             int64_t rows, int64_t cols,
                                                             int64_t ld_in, T* __restrict__ out,
                                                             int64_t ld_out, int32_t vec_ok) {
  constexpr int V = 8 / sizeof(T);          // elements per 8-byte vector
  constexpr int LPR = kTile / V;            // threads per tile row
  constexpr int RPP = kThreads / LPR;       // tile rows per pass
  constexpr int PAD = 4 / sizeof(T);        // 4 bytes of padding per LDS row
  __shared__ T tile[kTile][kTile + PAD];

  const int tid = threadIdx.x;
  const int sub = tid / LPR;                // tile row (column) of this thread in a pass
  const int vo = (tid % LPR) * V;           // first of its V elements
  const int64_t tr = (rows + kTile - 1) / kTile, tc = (cols + kTile - 1) / kTile;
  for (int64_t t = blockIdx.x; t < tr * tc; t += gridDim.x) {
    const int64_t r0 = (t / tc) * kTile, c0 = (t % tc) * kTile;
    const bool full = vec_ok && r0 + kTile <= rows && c0 + kTile <= cols;
    // input rows r0 .. r0+63 into tile[r][.]
#pragma unroll
    for (int p = 0; p < kTile / RPP; ++p) {
      const int r = p * RPP + sub;
      const int64_t gr = r0 + r, gc = c0 + vo;
      if (full) {
        union { uint64_t u; T e[V]; } v;
        v.u = *(const uint64_t*)(in + gr * ld_in + gc);
#pragma unroll
        for (int e = 0; e < V; ++e) tile[r][vo + e] = v.e[e];
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e)
          tile[r][vo + e] = (gr < rows && gc + e < cols) ? in[gr * ld_in + gc + e] : T(0);
      }
    }
    __syncthreads();
    // output rows c0 .. c0+63 (input columns) from tile[.][c]
#pragma unroll
    for (int p = 0; p < kTile / RPP; ++p) {
      const int c = p * RPP + sub;
      const int64_t oc = c0 + c, orr = r0 + vo;
      if (full) {
        union { uint64_t u; T e[V]; } v;
#pragma unroll
        for (int e = 0; e < V; ++e) v.e[e] = tile[vo + e][c];
        *(uint64_t*)(out + oc * ld_out + orr) = v.u;
      } else if (oc < cols) {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (orr + e < rows) out[oc * ld_out + orr + e] = tile[vo + e][c];
      }
    }
    __syncthreads();   // the tile is refilled by the next iteration
  }
}

template <typename T>
sk_status launch_transpose(const void* in, int64_t rows, int64_t cols, int64_t ld_in, void* out,
                           int64_t ld_out, hipStream_t stream) {
  const bool vec_ok = ((uintptr_t)in % 8 == 0) && ((uintptr_t)out % 8 == 0) &&
                      (ld_in * (int64_t)sizeof(T)) % 8 == 0 &&
                      (ld_out * (int64_t)sizeof(T)) % 8 == 0;
  const int64_t tiles = ((rows + kTile - 1) / kTile) * ((cols + kTile - 1) / kTile);
  // enough workgroups to fill every CU several times over; larger matrices
  // loop over their tiles
  const unsigned grid = (unsigned)std::min<int64_t>(tiles, 8192);
  hipLaunchKernelGGL(transpose_kernel<T>, dim3(grid), dim3(kThreads), 0, stream, (const T*)in,
                     rows, cols, ld_in, (T*)out, ld_out, (int32_t)vec_ok);
  return hipGetLastError() == hipSuccess ? SK_OK : SK_ERR_HIP;
}

}  // namespace
}  // namespace sk

extern "C" sk_status sk_transpose(const void* in, int64_t rows, int64_t cols, int64_t ld_in,
                                  void* out, int64_t ld_out, int32_t elem_bytes,
                                  void* hip_stream) {
  if (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4) return SK_ERR_INVALID_ARG;
  if (rows < 0 || cols < 0) return SK_ERR_INVALID_ARG;
  if (ld_in < std::max<int64_t>(1, cols) || ld_out < std::max<int64_t>(1, rows))
    return SK_ERR_INVALID_ARG;
  if (rows == 0 || cols == 0) return SK_OK;
  if (in == nullptr || out == nullptr) return SK_ERR_INVALID_ARG;
  // byte extents below 2^60 (no overflow in the address arithmetic)
  constexpr int64_t kMaxElems = (int64_t)1 << 58;
  if (rows > kMaxElems / ld_in || cols > kMaxElems / ld_out) return SK_ERR_INVALID_ARG;
  // the two matrices' byte ranges must not overlap
  const uintptr_t a0 = (uintptr_t)in, a1 = a0 + (uintptr_t)(((rows - 1) * ld_in + cols) * elem_bytes);
  const uintptr_t b0 = (uintptr_t)out, b1 = b0 + (uintptr_t)(((cols - 1) * ld_out + rows) * elem_bytes);
  if (a0 < b1 && b0 < a1) return SK_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  switch (elem_bytes) {
    case 1: return sk::launch_transpose<uint8_t>(in, rows, cols, ld_in, out, ld_out, s);
    case 2: return sk::launch_transpose<uint16_t>(in, rows, cols, ld_in, out, ld_out, s);
    default: return sk::launch_transpose<uint32_t>(in, rows, cols, ld_in, out, ld_out, s);
  }
}
