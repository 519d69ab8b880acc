// 64-bit coefficients, approximate Shoup quotient (lazy bound 4q, q < 2^61).
#define ARITH Arith64<false>
#ifndef COL_TILE
#define COL_TILE 16
#endif
#define WITH_LDS_PATH 1
#define LDS_MAX_LOG 14
#define LAUNCH_FN launch_u64
#include "dispatch.inc"
