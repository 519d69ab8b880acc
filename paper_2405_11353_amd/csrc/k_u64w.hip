// 64-bit coefficients, approximate Shoup quotient, wide lazy range: forward
// values in [0, 16q) for plans whose moduli are all below 2^60, so that the
// forward passes reduce on about half of their stages (Arith64<false, true>).
#define ARITH Arith64<false, true>
#ifndef COL_TILE
#define COL_TILE 16
#endif
#define WITH_LDS_PATH 1
#define LDS_MAX_LOG 14
#define LAUNCH_FN launch_u64w
#include "dispatch.inc"
