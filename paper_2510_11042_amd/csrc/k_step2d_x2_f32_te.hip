// k_step2d_x2_f32_te.hip -- the 2-D two-step kernels, float, TE.
#define LBM_X2_T float
#define LBM_X2_POL TE
#include "k_step2d_x2.inc"
