// 64-bit coefficients, approximate Shoup quotient (lazy bound 4q, q < 2^61).
#define ARITH Arith64<false>
#define COL_TILE 16
#define WITH_LDS_PATH 1
#define LDS_MAX_LOG 14
#define LAUNCH_FN launch_u64
#include "dispatch.inc"
