// Kernel instantiations for one (input type, A layout, B layout) triple,
// selected by -DSK_DT / -DSK_LA / -DSK_LB at compile time.  The tile menu
// per input type is listed here.
#include "sk_kernel.hpp"
#include "sk_registry.hpp"

#ifndef SK_DT
#error "SK_DT must be defined"
#endif

#define SK_CAT_(a, b) a##b
#define SK_CAT(a, b) SK_CAT_(a, b)
#define SK_INST(BM, BN, WGM, NW)                                                      \
  static const bool SK_CAT(reg_, __LINE__) = sk::register_kernel(                     \
      {SK_DT, SK_LA, SK_LB, BM, BN, WGM, 64 * NW,                                     \
       (const void*)&sk::sk_gemm_kernel<sk::Cfg<SK_DT, SK_LA, SK_LB, BM, BN, WGM, NW>>});

#if SK_DT == 0
// f32: 128x128x32 (the 512^3 Stream-K configuration)
SK_INST(128, 128, 2, 4)
#else
// f16 / bf16 / e4m3: large tiles for compute-bound shapes, smaller ones for
// small or skinny problems.  256x256 runs 8 waves (two per SIMD, 128x64 wave
// tiles).  Where both operands are copied LDS-direct (every f16/bf16 layout,
// e4m3 with K-contiguous A and B), 256x128 and 128x128 also run 8 waves
// (64x64 and 32x64 wave tiles): two waves per SIMD hide LDS and load
// latency that one wave per SIMD leaves exposed.  e4m3 with an M- or
// N-major operand transposes bytes in registers while staging and runs out
// of registers at two waves per SIMD, so there 256x128 and 128x128 keep
// 4 waves (128x64 and 64x64 wave tiles).
SK_INST(256, 256, 2, 8)
#if SK_DT != 3 || (SK_LA == 0 && SK_LB == 1)
SK_INST(256, 128, 4, 8)
SK_INST(128, 128, 4, 8)
#else
SK_INST(256, 128, 2, 4)
SK_INST(128, 128, 2, 4)
#endif
#if SK_DT == 3
SK_INST(64, 128, 2, 4)
#endif
#endif
