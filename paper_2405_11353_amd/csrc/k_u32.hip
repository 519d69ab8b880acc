// 32-bit coefficients (q < 2^30), Shoup product at the paper's word size.
#define ARITH Arith32
#ifndef COL_TILE
#define COL_TILE 32
#endif
#define WITH_LDS_PATH 1
#define LDS_MAX_LOG 15
#define LAUNCH_FN launch_u32
#include "dispatch.inc"
