// k_step3d.hip -- launcher of the 3-D two-step kernel (k_step3d_x2).
#include "launch.hpp"

namespace lbm {

template <typename T>
bool launch_step3d_x2(const StepArgs<T> &a, int tx, int ty, int zc, bool dft, hipStream_t s) {
    if (zc < 1 || zc + 2 > kX3MaxPlanes) return false;   // the chunk's vacuum flags live in LDS
    const int tiles = a.tiles_x * a.tiles_y;
    dim3 grid((unsigned)(tiles * ((a.nz + zc - 1) / zc)), 1, 1);
#define LBM_X3_DFT(TX, TY, LINE)                                                                          \
    if (dft) hipLaunchKernelGGL((k_step3d_x2<T, TX, TY, LINE, true>), grid, dim3(TX * TY), 0, s, a, zc); \
    else hipLaunchKernelGGL((k_step3d_x2<T, TX, TY, LINE, false>), grid, dim3(TX * TY), 0, s, a, zc);
#define LBM_X3(TX, TY)                           \
    if (tx == TX && ty == TY) {                  \
        if (a.line_tab) { LBM_X3_DFT(TX, TY, true) } \
        else { LBM_X3_DFT(TX, TY, false) }       \
        return true;                             \
    }
    if constexpr (sizeof(T) == 4) { LBM_X3_TILES_F32(LBM_X3) }
    else { LBM_X3_TILES_F64(LBM_X3) }
#undef LBM_X3
#undef LBM_X3_DFT
    return false;
}

template bool launch_step3d_x2<float>(const StepArgs<float> &, int, int, int, bool, hipStream_t);
template bool launch_step3d_x2<double>(const StepArgs<double> &, int, int, int, bool, hipStream_t);

}  // namespace lbm
