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
#elif SK_DT >= 4 && SK_DT <= 8
// MXFP8 (e4m3, e5m2), MXFP4 (e2m1) and MXFP6 (e2m3, e3m2) with E8M0
// block scales: K-contiguous operands only
#if SK_LA == 0 && SK_LB == 1
SK_INST(256, 128, 4, 8)
SK_INST(128, 128, 4, 8)
#endif
#else
// f16 / bf16 / e4m3 / e5m2: large tiles for compute-bound shapes, smaller ones for
// small or skinny problems.  Both operands are copied LDS-direct in every
// layout (M/N-major ones read back with transposing LDS reads), and the
// three large tiles run 8 waves, two per SIMD, which hide LDS and load
// latency that one wave per SIMD leaves exposed: 128x64 wave tiles on
// 256x256, 64x64 on 256x128, 32x64 on 128x128.
SK_INST(256, 256, 2, 8)
SK_INST(256, 128, 4, 8)
SK_INST(128, 128, 4, 8)
#if SK_DT == 3 || SK_DT == 9
SK_INST(64, 128, 2, 4)
#endif
#endif
