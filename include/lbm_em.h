/*
 * lbm_em.h -- C ABI of the MI355X (gfx950) electromagnetic lattice Boltzmann
 * library: the hot path of "Lattice Boltzmann method for electromagnetic wave
 * scattering" (Khan, Thampi, Roy; arXiv 2510.11042).
 *
 * The problem the calls follow (paper sections 2 and 3):
 *   - Maxwell's equations on a D3Q7 lattice, vector distributions e_i, h_i,
 *     tau = 1/2 update  e_i(r + c_i, t+1) = 2 e_i^eq - e_i   (section 2.1,
 *     Eq. LBGK_equation) with the equilibria of Eq. EDF; c = 1/3 lattice units.
 *   - a per-cell relative permittivity eps_r(x) (mu_r = 1, section 3.1 end);
 *   - a linearly polarised plane wave of wavelength lambda (cells);
 *   - an open boundary (section 2.2) inside a graded absorbing layer;
 *   - steady-state time stepping, a one-period DFT of E and H on a closed
 *     contour and the near-to-far-field transform to the angular scattering
 *     intensity |S(theta)|^2 / |S(theta, phi)|^2 (sections 2.3, 2.4).
 *
 * Conventions for every call
 *   - Return value: LBM_EM_OK or a negative lbm_em_status; the library never
 *     aborts or throws across this boundary.  lbm_em_last_error() gives a
 *     message for the last failing call on the calling thread.
 *   - Arrays are indexed [z][y][x] with x fastest (nx*ny*nz elements).
 *   - A handle is not thread safe.  All device work of a handle is ordered
 *     on the stream given at creation; calls that return host data
 *     synchronise that stream before returning.
 *   - Ownership: the library owns all device state of a handle (allocated at
 *     create, freed at destroy).  Caller arrays are only read or written
 *     during the call (device pointers: until the work queued by the call
 *     has run on the handle's stream).
 */
#ifndef LBM_EM_H
#define LBM_EM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_EM_OK = 0,
    LBM_EM_EINVAL = -1,       /* bad argument (size, pointer, range)            */
    LBM_EM_ENOMEM = -2,       /* device allocation failed                         */
    LBM_EM_EDEVICE = -3,      /* no HIP device or a HIP runtime error             */
    LBM_EM_ESTATE = -4,       /* call not valid in the handle's current state     */
    LBM_EM_EUNSUPPORTED = -5  /* valid request the library does not implement     */
} lbm_em_status;

typedef struct lbm_em *lbm_em_handle;
typedef struct lbm_em_batch_s *lbm_em_batch;

/* Field layout of a handle.  2-D runs are D3Q7 on nz == 1 with z streaming the
 * identity; TM carries (E_z, H_x, H_y) -- E along the invariant axis, the
 * paper's TM incidence on cylinders (section 3.2) -- and TE (E_x, E_y, H_z). */
enum { LBM_EM_TM = 0, LBM_EM_TE = 1, LBM_EM_3D = 2 };
enum { LBM_EM_FP32 = 0, LBM_EM_FP64 = 1 };
enum { LBM_EM_HOST = 0, LBM_EM_DEVICE = 1 };

typedef struct {
    int32_t nx, ny, nz;     /* cells (>= 1); nz must be 1 for TM/TE, >= 3 for 3-D     */
    int32_t pol;            /* LBM_EM_TM, LBM_EM_TE or LBM_EM_3D                     */
    int32_t precision;      /* LBM_EM_FP32 (storage and arithmetic) or LBM_EM_FP64   */
    int32_t absorb[3];      /* absorbing-layer width W per axis, 0 = periodic axis;
                               2W <= n.  Layer strength sigma(d) = sigma_max (d/W)^2,
                               d = 1..W counted from the layer's inner edge          */
    double sigma_max;       /* e.g. 0.25                                              */
    void *stream;           /* hipStream_t to order all work on; NULL = null stream  */
} lbm_em_config;

/* Incident plane wave E = g(t) E0 ehat sin(omega t - k khat.(r - center)),
 * H = khat x E, omega = 2 pi/(3 lambda), k = 2 pi/lambda, g(t) =
 * sin^2(pi t/(2 t_r)) for t < t_r = ramp_periods * 3 lambda, 1 afterwards.
 * It is imposed in absorbing-layer cells whose eps_r (and mu_r) is exactly 1;
 * the layer relaxes every other layer cell towards zero field. */
typedef struct {
    double lambda;          /* free-space wavelength in cells; 3*lambda must be integral */
    double khat[3];         /* unit propagation direction (in-plane for TM/TE)           */
    double ehat[3];         /* unit E polarisation, perpendicular to khat;
                               TM: +-z, TE: in-plane                                       */
    double amplitude;       /* E0                                                          */
    double ramp_periods;    /* ramp length in periods                                      */
    double center[3];       /* phase reference point in cell coordinates                   */
} lbm_em_plane_wave;

/* Create a handle: allocates the distributions (reduced exact state: 11
 * scalars per cell in 2-D, 27 in 3-D, two buffers), eps_r (initialised to 1)
 * and zeroes the state (t = 0).  *out is set only on success.
 * Rows are padded to a multiple of 64 cells; one plane (padded nx * ny * nz
 * values) must stay below 4 GiB, as the kernels address a plane with 32-bit
 * byte offsets (FP32 up to 2^30 cells, e.g. 1024^3 or 32768^2).
 * Errors: EINVAL for bad sizes / pointers, EDEVICE without a HIP device,
 * ENOMEM when device memory runs out. */
lbm_em_status lbm_em_create(const lbm_em_config *cfg, lbm_em_handle *out);

/* Release all device memory of the handle (synchronises its stream).
 * ESTATE while the handle belongs to a batch (destroy the batch first). */
lbm_em_status lbm_em_destroy(lbm_em_handle h);

/* Set eps_r(x) (paper section 2.1: it enters the rest equilibrium and
 * E = D/eps_r).  eps: nx*ny*nz values, where = LBM_EM_HOST or LBM_EM_DEVICE,
 * dtype = LBM_EM_FP32 (float) or LBM_EM_FP64 (double).  Values are copied.
 * 2-D handles store no rest population (it is 6 (eps_r - 1) times the
 * stored z-pair), so a map changed between steps also rescales the rest
 * population at once; 3-D handles keep it.  Set maps before stepping (or
 * reset) for a run that matches the literal scheme.
 * Errors: EINVAL if a value is < 1 or not finite (checked on the host copy). */
lbm_em_status lbm_em_set_permittivity(lbm_em_handle h, const void *eps, int32_t where,
                                      int32_t dtype);

/* Set mu_r(x) of a 2-D (TM/TE) handle (section 2.1: it enters the rest
 * equilibrium h_0^eq = (mu_r - 1) H and H = B/mu_r).  Same layout and
 * validation as lbm_em_set_permittivity; the first call allocates one more
 * plane (mu_r = 1 until then), mu = NULL frees it (mu_r = 1 again).  One
 * and two steps per launch (every tile) support it; batches and the adjoint
 * are EUNSUPPORTED with it.  Like eps_r, it also sets the (unstored) rest
 * population h_0 = 6 (mu_r - 1) h_zpair.  Errors: EUNSUPPORTED for 3-D handles or after adjoint_setup,
 * ESTATE while the handle belongs to a batch, EINVAL as for eps. */
lbm_em_status lbm_em_set_permeability(lbm_em_handle h, const void *mu, int32_t where,
                                      int32_t dtype);

/* Perfect-conductor cells of a TM handle (section 3.2.1 scatters off PEC
 * cylinders with E along the axis; the paper takes the boundary rule from
 * the authors' earlier work, read here as: a flagged cell has zero electric
 * field, its H is recovered with mu_r = 1, and the absorbing layer imposes
 * no incident wave on it).  mask: nx*ny bytes [y][x], non-zero = conductor,
 * on the host or the device (where); copied.  NULL removes the conductor.
 * Cells leaving the mask return to mu_r = 1.  The mask shares the
 * permeability plane (a conductor is stored as mu = 0), so it has the
 * permeability map's limits: batches and the adjoint refuse the handle.
 * Errors: EUNSUPPORTED for TE and 3-D handles or after adjoint_setup
 * (staircase zero-E conductors are pinned for TM only), ESTATE while the
 * handle belongs to a batch, EINVAL for a bad `where`. */
lbm_em_status lbm_em_set_pec(lbm_em_handle h, const uint8_t *mask, int32_t where);

/* Set the incident plane wave (see lbm_em_plane_wave).  EINVAL if khat or
 * ehat is not a unit vector, not perpendicular, 3*lambda is not integral,
 * or the polarisation does not match the handle (TM: ehat = +-z; TE/TM:
 * khat_z = 0), or the ramp exceeds 1e7 steps; ESTATE while the handle
 * belongs to a batch.  The phase factors are tabulated once here (FP64, per
 * period step and per grid line), so the step kernels evaluate no sine. */
lbm_em_status lbm_em_set_source(lbm_em_handle h, const lbm_em_plane_wave *pw);

/* Record E and H phasors on the surface of the node box [lo, hi] (inclusive
 * cell coordinates; in 2-D lo[2] = hi[2] = 0) and at the probe node
 * ((lo+hi)/2) by a running DFT over the steps [window_start,
 * window_start + window_len):  X += (2/window_len) F(t) exp(-j omega t)
 * (section 2.4, "one period of the steady-state oscillation").  Clears the
 * accumulators.  EINVAL if the box is not strictly inside the grid, is
 * thinner than 3 nodes, or the window is empty; ESTATE before the source is
 * set or while the handle belongs to a batch. */
lbm_em_status lbm_em_set_ntff(lbm_em_handle h, const int32_t lo[3], const int32_t hi[3],
                              int64_t window_start, int64_t window_len);

/* Exact incident line (a total-field / scattered-field-like forcing, which
 * the paper names as future work in section 4) for a 2-D handle whose
 * source propagates along +-x or +-y, or a 3-D handle with incidence along
 * +-z (khat components within 1e-12 of axis-aligned): a one-cell-wide run
 * along that axis, with the same
 * layers on it and the same source, advances with the grid (one small
 * launch before each grid launch).  In background layer cells (eps_r =
 * mu_r = 1) the layer then damps only the scattered part,
 *     f' = f* + sigma (f_l* - f*) + sigma_a (f^eq_ref - f_l*),
 * f_l* being the line's post-collision populations at the cell's coordinate
 * along the axis and sigma_a the line's own layer strength there.  A
 * background-only grid reproduces the line at every row bit for bit, so the
 * line's phasors are the exact incident field: lbm_em_farfield(h, NULL, ...)
 * then subtracts and normalises by them and no companion run is needed.
 * enable = 0 removes the line.  Set it after the source and before stepping
 * (t = 0, or after a reset); a new source removes it.  Batches and the
 * adjoint refuse a handle with a line.
 * A line whose state fits 64 KB (2-D: 11 scalars per cell; 3-D: 27, FP32
 * nz <= 606, FP64 nz <= 303) is held in LDS for a whole 64-step graph
 * chunk; a longer one takes one or two steps through global memory before
 * each grid launch.
 * Errors: EUNSUPPORTED after adjoint_setup, ESTATE without a source, at
 * t > 0 or while batched, EINVAL for other directions. */
lbm_em_status lbm_em_set_incident_line(lbm_em_handle h, int32_t enable);

/* The incident line's phasors: out[(u*6 + c)*2 + {0,1}] = (re, im) of
 * component c in (Ex, Ey, Ez, Hx, Hy, Hz) at coordinate u along the line
 * (over the window of lbm_em_set_ntff); *n receives the line length (out
 * = NULL queries it).  ESTATE without a line.  Synchronises. */
lbm_em_status lbm_em_get_line_phasors(lbm_em_handle h, double *out, int32_t *n);

/* Advance n >= 0 time steps (asynchronous on the handle's stream): pull
 * streaming with the open boundary, moments, tau = 1/2 collision, absorbing
 * layer / source, contour DFT -- one fused kernel per step.  Steps are
 * replayed from a captured HIP graph in chunks. */
lbm_em_status lbm_em_step(lbm_em_handle h, int64_t n);

/* Advance `count` 2-D handles n steps together: one persistent launch per
 * step covers all instances (a flattened (instance, tile) work list that a
 * chip-sized grid strides over).  All handles must share polarisation,
 * precision, stream and device and be at the same time step; each keeps
 * its own grid size, permittivity, source and contour.  Results are
 * bit-identical to lbm_em_step on each handle.  Uses the launch settings of
 * hs[0]; with two steps per launch, the tile with the fewest padded cells
 * over the batched instances (hs[0]'s own tile when it is among the best).
 * An instance that fills the device by itself (two steps per launch, here
 * and on the handle, and at least one of its own two-step tiles per compute
 * unit) is advanced by the single-instance kernels instead, as a group of
 * its own: the persistent launch pays only for instances too small to fill
 * the chip.  Two or more such instances alternate over two side streams
 * that the batch forks from the handles' stream and joins back into it
 * within the call, so two independent kernels overlap; work queued on the
 * handles' stream afterwards sees every instance advanced.
 * EUNSUPPORTED for 3-D handles and handles with a permeability map.
 * (One-shot form of the batch calls below.) */
lbm_em_status lbm_em_step_many(const lbm_em_handle *hs, int32_t count, int64_t n);

/* A reusable batch: snapshots the handles' settings (source, contour, tile;
 * permittivity values may still change through set_permittivity) and
 * replays lbm_em_batch_step from captured HIP graphs.  Instances are packed
 * in order into groups whose state (two buffers + eps) fits a cache budget
 * (default 192 MiB, inside the 256 MB Infinity Cache); batch_step advances
 * each group the n steps in turn, one persistent launch per step per group.
 * The handles must not be destroyed, re-configured or stepped on their own
 * while the batch is used (ESTATE if their time steps diverge). */
lbm_em_status lbm_em_batch_create(const lbm_em_handle *hs, int32_t count, lbm_em_batch *out);
lbm_em_status lbm_em_batch_step(lbm_em_batch b, int64_t n);
/* Thread blocks of each persistent launch (default 32 per CU, capped at the
 * number of work items of the group). */
lbm_em_status lbm_em_batch_set_grid(lbm_em_batch b, int32_t grid);
/* Cache budget for grouping in bytes; 0 = all instances in one group. */
lbm_em_status lbm_em_batch_set_cache_budget(lbm_em_batch b, int64_t bytes);
/* Autotuner of the batch: times `launches` two-step launches of every
 * two-step tile over the instances the persistent kernel advances and keeps
 * the fastest tile (the padded-cell choice of batch_create is a heuristic:
 * wider tiles move whole 128-byte lines at the cost of padding).  Timed
 * launches read the current buffers and write the spare ones with the DFT
 * off, so no instance changes; results after tuning are bit-identical for
 * every tile.  *best_us (may be NULL): microseconds per step of all batched
 * instances with the chosen tile, 0 when nothing is timed (one step per
 * launch, or every instance advanced by its own kernels).  EINVAL for
 * launches < 1, ESTATE when the handles' time steps have diverged. */
lbm_em_status lbm_em_batch_autotune(lbm_em_batch b, int32_t launches, double *best_us);
/* Number of groups of the current plan (an instance advanced by its own
 * kernels counts as one group). */
lbm_em_status lbm_em_batch_groups(lbm_em_batch b, int32_t *groups);
/* The batch's launch shape: steps per launch (1 or 2) and the two-step tile
 * TX x TY of the persistent kernel (from batch_create or the autotuner). */
lbm_em_status lbm_em_batch_get_tile(lbm_em_batch b, int32_t *steps_per_launch, int32_t *tile_x, int32_t *tile_y);
lbm_em_status lbm_em_batch_destroy(lbm_em_batch b);

/* Launch shape of the step kernel: every thread updates vx consecutive
 * x-cells (vx in {1, 2, 4} for FP32, {1, 2} for FP64), thread blocks are
 * bx x by threads (64 <= bx*by <= 256, a multiple of the 64-wide wavefront).
 * The tile only changes speed, never results (each cell's update is
 * independent of the tiling).  EINVAL for other shapes. */
lbm_em_status lbm_em_set_tile(lbm_em_handle h, int32_t vx, int32_t bx, int32_t by);
lbm_em_status lbm_em_get_tile(lbm_em_handle h, int32_t *vx, int32_t *bx, int32_t *by);

/* Time steps per launch of lbm_em_step: 1 or 2 (the default).  Two steps
 * per launch read and write the state once per two steps and give bit-
 * identical results: in 2-D a TX x TY tile plus a one-cell ring through LDS
 * (FP32 tiles 64x16, 128x8, 128x16, 256x8, 256x16, 128x32; FP64 32x16,
 * 64x8, 64x16, 128x8, 128x16, 64x32), in 3-D a TX x TY column tile that
 * marches along z with a one-plane lag (FP32 64x16, 64x8, 32x16, 128x8,
 * 256x4, 128x4; FP64 32x16, 32x8, 16x16, 64x8, 128x4; 512-thread tiles run
 * two blocks per compute unit).  tile 0 x 0 keeps the current one; EINVAL
 * for other tiles.  get_fusion's tile outputs may be NULL. */
lbm_em_status lbm_em_set_fusion(lbm_em_handle h, int32_t steps_per_launch, int32_t tile_x, int32_t tile_y);
lbm_em_status lbm_em_get_fusion(lbm_em_handle h, int32_t *steps_per_launch, int32_t *tile_x, int32_t *tile_y);

/* Time every supported launch shape on this handle's grid -- one step per
 * launch with every tile, and two steps per launch with every two-step
 * tile -- `launches` launches each, reading the current state and
 * writing the spare buffer with the DFT off, so the simulation is not
 * advanced; keep the fastest per time step and verify that it reproduces
 * one-cell-per-thread single steps bit for bit (EDEVICE if not).
 * *best_us (may be NULL) receives the winner's time per step. */
lbm_em_status lbm_em_autotune(lbm_em_handle h, int32_t launches, double *best_us);

/* Restart from t = 0: zero the distributions and the DFT accumulators
 * (stream-ordered, no allocation).  Material maps, source and contour are
 * kept. */
lbm_em_status lbm_em_reset(lbm_em_handle h);

/* Current time step t (number of steps taken). */
lbm_em_status lbm_em_time(lbm_em_handle h, int64_t *t);

/* Fields at the current time t: E and H, each nx*ny*nz*3 values [cell][3]
 * in the handle's precision, on the host (synchronises) or device. */
lbm_em_status lbm_em_get_fields(lbm_em_handle h, void *E, void *H, int32_t where);

/* Raw DFT phasors: out[(node*6 + c)*2 + {0,1}] = (re, im) of component c in
 * (Ex, Ey, Ez, Hx, Hy, Hz) for the box-surface nodes in ascending linear
 * cell index, followed by the probe node.  *n_nodes receives the number of
 * surface nodes (the array must hold (n_nodes + 1) * 12 doubles; pass
 * out = NULL to query the count).  Synchronises. */
lbm_em_status lbm_em_get_phasors(lbm_em_handle h, double *out, int32_t *n_nodes);

/* Angular scattering intensity (sections 2.3-2.4).  Scattered phasors are
 * those of h minus those of `incident` (a companion handle with eps_r = 1 and
 * the same grid, source and contour), transformed with the background
 * (eps = mu = 1, unit impedance) far-field formulas, and normalised by the
 * incident probe amplitude |ehat . E_inc| (TM, 3-D) or |hhat . H_inc| (TE).
 * Angles: theta from khat; 2-D: in the plane, counter-clockwise about +z
 * (phi ignored); 3-D: phi about khat measured from ehat.  Host arrays of
 * n_angles; out_S2 receives |S|^2 (2-D: k r |E_s|^2/|E_i|^2, Eq. S2D; 3-D:
 * k^2 r^2 |E_s|^2/|E_i|^2, Eq. S3D).  incident = NULL: no subtraction and
 * normalisation by the source amplitude, or, on a handle with an incident
 * line, subtraction of and normalisation by the line's phasors.  ESTATE if
 * the DFT window has not
 * been completed or the incident probe amplitude is zero.  Synchronises. */
lbm_em_status lbm_em_farfield(lbm_em_handle h, lbm_em_handle incident, const double *theta_deg,
                              const double *phi_deg, int32_t n_angles, double *out_S2);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * |S|^2 as lbm_em_farfield (same arguments, same arithmetic), with every
 * device buffer of the call -- angles, far-field sums, |S|^2, the incident
 * amplitude and, on a handle with an incident line, the line's phasors on
 * the contour nodes -- in a static per-device array of the library
 * (LBM_EM_FARFIELD_STATIC_MAX_ANGLES angles, contours of up to
 * LBM_EM_FARFIELD_STATIC_MAX_NODES nodes: 3.4 MB, held by every device the
 * library runs on until the process ends).  The call allocates no device or
 * host memory and needs no workspace argument.  EINVAL beyond either
 * maximum; otherwise the statuses of lbm_em_farfield.  Calls that overlap
 * on one device share that array and race: issue them from one thread at a
 * time per device.  Synchronises. */
#define LBM_EM_FARFIELD_STATIC_MAX_ANGLES 4096
#define LBM_EM_FARFIELD_STATIC_MAX_NODES 32768
lbm_em_status lbm_em_farfield_static(lbm_em_handle h, lbm_em_handle incident, const double *theta_deg,
                                     const double *phi_deg, int32_t n_angles, double *out_S2);

/* ---------------------------------------------------------------------
 * Inverse design: gradient of a far-field objective with respect to eps_r
 * in a design rectangle, by the discrete adjoint of the step (2-D TM/TE).
 *
 *   J(eps) = sum_a weight[a] |S(theta_a)|^2
 *
 * with |S|^2 as lbm_em_farfield computes it against `incident` (2-D:
 * Eq. S2D of section 2.3 after the transform of section 2.4).  The design
 * rectangle [dlo, dhi] (inclusive, cells) must lie strictly inside the
 * contour box and outside the absorbing layer.
 * --------------------------------------------------------------------- */
/* Store the objective (angles in degrees from khat, weights; weight = NULL
 * means 1), the design rectangle and the checkpoint spacing (0: ceil(sqrt(n))
 * steps).  The incident handle must stay alive and completed. */
lbm_em_status lbm_em_adjoint_setup(lbm_em_handle h, lbm_em_handle incident, const double *theta_deg,
                                   const double *weight, int32_t n_angles, const int32_t dlo[2],
                                   const int32_t dhi[2], int32_t checkpoint_every);

/* Restart the handle at t = 0, run n steps keeping a full-state checkpoint
 * every K steps (K from adjoint_setup; memory ceil(n/K) states), evaluate J
 * into *J_out (host).  n must cover the DFT window.  Synchronises. */
lbm_em_status lbm_em_forward_checkpointed(lbm_em_handle h, int64_t n, double *J_out);

/* dJ/deps_r for the design rectangle, (dhi-dlo+1) row-major doubles [y][x],
 * on the host or device.  Segment by segment in reverse: restore the
 * checkpoint, recompute the segment (recording dE/deps of the design cells),
 * then run the adjoint step backwards over it.  Cost ~2 forward passes.
 * Afterwards the handle is back at t = 0 with zero fields.  Synchronises. */
lbm_em_status lbm_em_backward(lbm_em_handle h, double *grad_eps, int32_t where);

/* Measurement helper: bandwidth of a plain 16-byte-per-thread device copy
 * of `bytes` (multiple of 16), averaged over `reps` launches on the null
 * stream, counting bytes read + written.  Allocates and frees two buffers
 * of `bytes`.  The measured ceiling the step kernels are compared with. */
lbm_em_status lbm_em_copy_bandwidth(int64_t bytes, int32_t reps, double *gbs);

/* Measurement helper: bandwidth of the step kernels' access pattern without
 * their arithmetic -- every thread reads one cell of `planes_in` FP32 planes
 * and writes it to `planes_out` planes with streamed stores (1 <= planes_out
 * <= planes_in <= 32, 1 <= cells <= 2^31) -- averaged over `reps` launches
 * on the null stream, counting bytes read + written.  Allocates and frees
 * the planes (about 4 (planes_in + planes_out) cells bytes), laid out with
 * the state's plane stride.  24 planes in and out is the 3-D two-step
 * kernel's traffic for vacuum cells. */
lbm_em_status lbm_em_stream_bandwidth(int64_t cells, int32_t planes_in, int32_t planes_out, int32_t reps,
                                      double *gbs);

/* Message of the last failing call on this thread ("" if none). */
const char *lbm_em_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_EM_H */
