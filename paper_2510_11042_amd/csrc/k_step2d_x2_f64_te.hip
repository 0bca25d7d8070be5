// k_step2d_x2_f64_te.hip -- the 2-D two-step kernels, double, TE.
#define LBM_X2_T double
#define LBM_X2_POL TE
#include "k_step2d_x2.inc"
