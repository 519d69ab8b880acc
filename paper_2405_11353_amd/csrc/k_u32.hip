// 32-bit coefficients (q < 2^30), Shoup product at the paper's word size.
#define ARITH Arith32
#define COL_TILE 32
#define WITH_LDS_PATH 1
#define LDS_MAX_LOG 15
#define LAUNCH_FN launch_u32
#include "dispatch.inc"
