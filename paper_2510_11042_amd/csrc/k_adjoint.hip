// k_adjoint.hip -- launchers of the 2-D adjoint kernels.
#include "launch.hpp"

namespace lbm {

template <typename T>
void launch_adjoint1(const AdjArgs<T> &a, int pol, hipStream_t s) {
    dim3 block(64, 4, 1);
    dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4, 1);
    if (pol == TM) hipLaunchKernelGGL((k_adjoint2d<T, TM>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_adjoint2d<T, TE>), grid, block, 0, s, a);
}

template <typename T>
bool launch_adjoint_x2(const AdjArgs<T> &a, int pol, int tx, int ty, hipStream_t s) {
    dim3 grid((unsigned)(a.tiles_x * ((a.ny + ty - 1) / ty)), 1, 1);
#define LBM_ADJ2(TX, TY)                                                                                     \
    if (tx == TX && ty == TY) {                                                                              \
        if (pol == TM)                                                                                       \
            hipLaunchKernelGGL((k_adjoint2d_x2<T, TM, TX, TY>), grid, dim3(x2_threads<T, TX, TY>()), 0, s, a); \
        else                                                                                                 \
            hipLaunchKernelGGL((k_adjoint2d_x2<T, TE, TX, TY>), grid, dim3(x2_threads<T, TX, TY>()), 0, s, a); \
        return true;                                                                                         \
    }
    if constexpr (sizeof(T) == 4) { LBM_X2_TILES_F32(LBM_ADJ2) }
    else { LBM_X2_TILES_F64(LBM_ADJ2) }
#undef LBM_ADJ2
    return false;
}

template void launch_adjoint1<float>(const AdjArgs<float> &, int, hipStream_t);
template void launch_adjoint1<double>(const AdjArgs<double> &, int, hipStream_t);
template bool launch_adjoint_x2<float>(const AdjArgs<float> &, int, int, int, hipStream_t);
template bool launch_adjoint_x2<double>(const AdjArgs<double> &, int, int, int, hipStream_t);

}  // namespace lbm
