// 64-bit coefficients, exact Shoup quotient (lazy bound 2q): the four-step
// path only, kept as the measured alternative to the approximate quotient.
#define ARITH Arith64<true>
#ifndef COL_TILE
#define COL_TILE 16
#endif
#define WITH_LDS_PATH 0
#define LDS_MAX_LOG 14
#define LAUNCH_FN launch_u64x
#include "dispatch.inc"
