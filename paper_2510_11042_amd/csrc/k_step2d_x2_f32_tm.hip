// k_step2d_x2_f32_tm.hip -- the 2-D two-step kernels, float, TM.
#define LBM_X2_T float
#define LBM_X2_POL TM
#include "k_step2d_x2.inc"
