// k_step2d_x2_f64_tm.hip -- the 2-D two-step kernels, double, TM.
#define LBM_X2_T double
#define LBM_X2_POL TM
#include "k_step2d_x2.inc"
