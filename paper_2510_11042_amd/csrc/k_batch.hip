// k_batch.hip -- launchers of the batched persistent kernels.
#include "launch.hpp"

namespace lbm {

template <typename T, int VX>
static void batch1_vx(const StepArgs<T> *d, int pol, int bx, int by, int grid, const int *tile_inst,
                      const int *tile_first, int ntiles, const int64_t *t_base, int64_t t_off, hipStream_t s) {
    dim3 block(bx, by, 1);
    if (pol == TM)
        hipLaunchKernelGGL((k_step2d_batch<T, TM, VX>), dim3(grid), block, 0, s, d, tile_inst, tile_first, ntiles,
                           t_base, t_off);
    else
        hipLaunchKernelGGL((k_step2d_batch<T, TE, VX>), dim3(grid), block, 0, s, d, tile_inst, tile_first, ntiles,
                           t_base, t_off);
}

template <typename T>
void launch_batch1(const StepArgs<T> *descs, int pol, int vx, int bx, int by, int grid, const int *tile_inst,
                   const int *tile_first, int ntiles, const int64_t *t_base, int64_t t_off, hipStream_t s) {
    if (vx == 1) batch1_vx<T, 1>(descs, pol, bx, by, grid, tile_inst, tile_first, ntiles, t_base, t_off, s);
    else if (vx == 2) batch1_vx<T, 2>(descs, pol, bx, by, grid, tile_inst, tile_first, ntiles, t_base, t_off, s);
    else if constexpr (sizeof(T) == 4)
        batch1_vx<T, 4>(descs, pol, bx, by, grid, tile_inst, tile_first, ntiles, t_base, t_off, s);
}

template <typename T, int POL>
static bool batch_x2_pol(const StepArgs<T> *d, int tx, int ty, bool two, bool dft, int grid, const int *tile_inst,
                         const int *tile_first, int ntiles, const int64_t *t_base, int64_t t_off, hipStream_t s) {
#define LBM_X2B(TX, TY)                                                                                          \
    if (tx == TX && ty == TY) {                                                                                   \
        if (two && dft)                                                                                           \
            hipLaunchKernelGGL((k_step2d_x2_batch<T, POL, TX, TY, true>), dim3(grid),                            \
                               dim3(x2_threads<T, TX, TY>()), 0, s, d, tile_inst, tile_first, ntiles, t_base,    \
                               t_off);                                                                           \
        else if (two)                                                                                             \
            hipLaunchKernelGGL((k_step2d_x2_batch<T, POL, TX, TY, false>), dim3(grid),                           \
                               dim3(x2_threads<T, TX, TY>()), 0, s, d, tile_inst, tile_first, ntiles, t_base,    \
                               t_off);                                                                           \
        else                                                                                                      \
            hipLaunchKernelGGL((k_step2d_tile_batch<T, POL, TX, TY>), dim3(grid),                                \
                               dim3(x2_threads<T, TX, TY>()), 0, s, d, tile_inst, tile_first, ntiles, t_base,    \
                               t_off);                                                                           \
        return true;                                                                                              \
    }
    if constexpr (sizeof(T) == 4) { LBM_X2_TILES_F32(LBM_X2B) }
    else { LBM_X2_TILES_F64(LBM_X2B) }
#undef LBM_X2B
    return false;
}

template <typename T>
bool launch_batch_x2(const StepArgs<T> *descs, int pol, int tx, int ty, bool two, bool dft, int grid,
                     const int *tile_inst, const int *tile_first, int ntiles, const int64_t *t_base, int64_t t_off,
                     hipStream_t s) {
    if (pol == TM)
        return batch_x2_pol<T, TM>(descs, tx, ty, two, dft, grid, tile_inst, tile_first, ntiles, t_base, t_off, s);
    return batch_x2_pol<T, TE>(descs, tx, ty, two, dft, grid, tile_inst, tile_first, ntiles, t_base, t_off, s);
}

template void launch_batch1<float>(const StepArgs<float> *, int, int, int, int, int, const int *, const int *, int,
                                   const int64_t *, int64_t, hipStream_t);
template void launch_batch1<double>(const StepArgs<double> *, int, int, int, int, int, const int *, const int *,
                                    int, const int64_t *, int64_t, hipStream_t);
template bool launch_batch_x2<float>(const StepArgs<float> *, int, int, int, bool, bool, int, const int *,
                                     const int *, int, const int64_t *, int64_t, hipStream_t);
template bool launch_batch_x2<double>(const StepArgs<double> *, int, int, int, bool, bool, int, const int *,
                                      const int *, int, const int64_t *, int64_t, hipStream_t);

}  // namespace lbm
