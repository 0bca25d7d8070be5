// k_step.hip -- launcher of the one-step kernels (k_step2d, k_step3d).
#include "launch.hpp"

namespace lbm {

template <typename T, int VX>
static void step1_vx(const StepArgs<T> &a, int pol, int bx, int by, hipStream_t s) {
    dim3 block(bx, by, 1);
    const int gx = (a.nx + VX - 1) / VX;
    dim3 grid((unsigned)((gx + bx - 1) / bx), (unsigned)((a.ny + by - 1) / by), (unsigned)a.nz);
    const bool rec = a.hist != nullptr;
    if (a.mu && a.line_tab) {
        if (pol == TM) hipLaunchKernelGGL((k_step2d<T, TM, VX, false, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step2d<T, TE, VX, false, true, true>), grid, block, 0, s, a);
    } else if (a.mu) {
        if (pol == TM) hipLaunchKernelGGL((k_step2d<T, TM, VX, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step2d<T, TE, VX, false, true>), grid, block, 0, s, a);
    } else if (a.line_tab && pol != D3) {
        if (pol == TM) hipLaunchKernelGGL((k_step2d<T, TM, VX, false, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step2d<T, TE, VX, false, false, true>), grid, block, 0, s, a);
    } else if (pol == TM) {
        if (rec) hipLaunchKernelGGL((k_step2d<T, TM, VX, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step2d<T, TM, VX>), grid, block, 0, s, a);
    } else if (pol == TE) {
        if (rec) hipLaunchKernelGGL((k_step2d<T, TE, VX, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step2d<T, TE, VX>), grid, block, 0, s, a);
    } else if (a.line_tab) {
        hipLaunchKernelGGL((k_step3d<T, VX, true>), grid, block, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_step3d<T, VX>), grid, block, 0, s, a);
    }
}

template <typename T>
void launch_step1(const StepArgs<T> &a, int pol, int vx, int bx, int by, hipStream_t s) {
    if (vx == 1) step1_vx<T, 1>(a, pol, bx, by, s);
    else if (vx == 2) step1_vx<T, 2>(a, pol, bx, by, s);
    else if constexpr (sizeof(T) == 4) step1_vx<T, 4>(a, pol, bx, by, s);
}

template void launch_step1<float>(const StepArgs<float> &, int, int, int, int, hipStream_t);
template void launch_step1<double>(const StepArgs<double> &, int, int, int, int, hipStream_t);

}  // namespace lbm
