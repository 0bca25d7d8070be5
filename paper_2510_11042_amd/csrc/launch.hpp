// launch.hpp -- host-side launchers of the step, batch and adjoint kernels.
//
// Each kernel family is instantiated and launched in translation units of
// its own (k_step.hip, k_step2d_x2_*.hip, k_step3d.hip, k_batch.hip,
// k_adjoint.hip), so the families compile in parallel; the runtime in
// lbm_em.hip calls them through these plain functions.  A launcher returns
// false when the requested tile is not one of the compiled shapes.
#pragma once

#include "kernels.hpp"

// Two-step tiles (2-D): TX x TY cells, TX a multiple of the 16-byte
// segment, one segment per thread and 256, 512 or 1024 threads.
#define LBM_X2_TILES_F32(M) M(64, 16) M(128, 8) M(128, 16) M(256, 8) M(256, 16) M(128, 32)
#define LBM_X2_TILES_F64(M) M(32, 16) M(64, 8) M(64, 16) M(128, 8) M(128, 16) M(64, 32)

// 3-D two-step tiles (one cell per thread; the LDS holds two planes of the
// tile's x/y movers: 136 KB for 64 x 16 FP32 and 32 x 16 FP64, 148 KB for
// 256 x 4 FP32 and 128 x 4 FP64; the 512-thread FP32 tiles take about 70 KB
// and run two blocks per compute unit).  Wide tiles spend fewer 128-byte
// lines on the ring columns.
#define LBM_X3_TILES_F32(M) M(64, 16) M(64, 8) M(32, 16) M(128, 8) M(256, 4) M(128, 4)
#define LBM_X3_TILES_F64(M) M(32, 16) M(32, 8) M(16, 16) M(64, 8) M(128, 4)

namespace lbm {

// One step, one-step kernels (k_step2d / k_step3d): every thread updates
// vx consecutive x cells, blocks of bx x by threads.  pol: TM, TE or D3.
template <typename T>
void launch_step1(const StepArgs<T> &a, int pol, int vx, int bx, int by, hipStream_t s);

// Two steps, 2-D (k_step2d_x2): a.tiles_x / a.tiles_y must be set.  One
// translation unit per precision and polarisation.  dft: the launch may
// meet the DFT window (selects the instantiation that accumulates it).
template <typename T, int POL>
bool launch_step2d_x2_pol(const StepArgs<T> &a, int tx, int ty, bool dft, hipStream_t s);
template <typename T>
inline bool launch_step2d_x2(const StepArgs<T> &a, int pol, int tx, int ty, bool dft, hipStream_t s) {
    return pol == TM ? launch_step2d_x2_pol<T, TM>(a, tx, ty, dft, s) : launch_step2d_x2_pol<T, TE>(a, tx, ty, dft, s);
}

// Two steps, 3-D z march (k_step3d_x2), z chunks of zc planes (1 <= zc <=
// kX3MaxPlanes - 2).  dft: the launch may fall into the DFT window (selects
// the instantiation that accumulates the contour DFT).  Returns false for an
// uncompiled tile or a chunk out of range.
template <typename T>
bool launch_step3d_x2(const StepArgs<T> &a, int tx, int ty, int zc, bool dft, hipStream_t s);

// Batched persistent launches over a flat (instance, tile) list.
template <typename T>
void launch_batch1(const StepArgs<T> *descs, int pol, int vx, int bx, int by, int grid, const int *tile_inst,
                   const int *tile_first, int ntiles, const int64_t *t_base, int64_t t_off, hipStream_t s);
template <typename T>
bool launch_batch_x2(const StepArgs<T> *descs, int pol, int tx, int ty, bool two, bool dft, int grid,
                     const int *tile_inst, const int *tile_first, int ntiles, const int64_t *t_base, int64_t t_off,
                     hipStream_t s);

// Adjoint: one reverse step, or two on the two-step tile.
template <typename T>
void launch_adjoint1(const AdjArgs<T> &a, int pol, hipStream_t s);
template <typename T>
bool launch_adjoint_x2(const AdjArgs<T> &a, int pol, int tx, int ty, hipStream_t s);

}  // namespace lbm
