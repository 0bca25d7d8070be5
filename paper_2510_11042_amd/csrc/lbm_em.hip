// lbm_em.hip -- runtime and C ABI of the gfx950 electromagnetic LBM library.
//
// One handle = one scattering instance: reduced-state distributions in two
// ping-pong buffers (structure of arrays, rows padded to 64 elements), eps_r,
// plane-wave parameters, the contour DFT accumulators and a device step
// counter used when step(n) is replayed from a captured HIP graph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm_em.h"
#include "launch.hpp"

using namespace lbm;

namespace {

thread_local std::string g_last_error;

struct ApiError {
    lbm_em_status code;
    std::string msg;
};

[[noreturn]] void fail(lbm_em_status code, const std::string &msg) { throw ApiError{code, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(LBM_EM_ENOMEM, std::string(what) + ": out of device memory");
    fail(LBM_EM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
lbm_em_status guarded(F &&f) {
    try {
        f();
        g_last_error.clear();
        return LBM_EM_OK;
    } catch (const ApiError &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return LBM_EM_EDEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return LBM_EM_EDEVICE;
    }
}

constexpr int kGraphChunk = 64;   // steps per captured graph
static_assert(kGraphChunk == kLineSlots, "the incident line's table holds one graph chunk");

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

void hfree(void *p) {
    if (p) (void)hipFree(p);
}

}  // namespace

struct lbm_em {
    lbm_em_config cfg{};
    int dim = 2;
    int nplanes = 11;
    size_t elem = 4;
    int64_t sy = 0, sz = 0, plane = 0;  // element strides
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;                        // buf[cur] holds f*(t-1)
    void *eps = nullptr;
    void *mu = nullptr;                 // permeability map (2-D; 0 = conductor); NULL: mu_r = 1
    bool mu_user = false;               // mu holds a map set through set_permeability
    unsigned char *pec = nullptr;       // dense [y][x] conductor mask (TM); NULL: none
    // exact incident line (2-D, incidence along x or y)
    lbm_em *line = nullptr;             // the one-row (one-column) line run; NULL: off
    int line_axis = 0;
    void *line_tmp = nullptr;           // the line's middle state inside a two-step launch
    void *line_tab = nullptr;           // its post-collision populations, slots t & 1
    double *line_acc = nullptr;         // its phasors, line_n x 12
    int64_t t = 0;
    hipStream_t stream = nullptr;
    int vx = 1, bx = 128, by = 2;       // cells per thread along x, block shape
    int fuse = 1;                       // time steps per launch (1 or 2)
    int cus = 1;                        // compute units of the device
    int ftx = 64, fty = 16;             // output tile of the two-step kernel
    // source
    bool src_on = false;
    lbm_em_plane_wave pw{};
    double hhat[3] = {0, 0, 0};
    int period = 0;
    double *wtab = nullptr;             // phase tables of the source (StepArgs::wave_*, ramp)
    int64_t axes_off = 0;               // offset of the per-axis tables in doubles
    int batch_refs = 0;                 // batches that hold this handle
    // contour DFT
    bool dft_set = false;
    Box box{};
    int probe[3] = {0, 0, 0};
    int64_t nnodes = 0, win0 = 0, winlen = 0;
    double *acc = nullptr;
    // graph replay: [chunk may meet the DFT window][starting buffer parity]
    int64_t *t_dev = nullptr;
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    mutable bool graph_dft = true;      // set while capturing: the chunk may meet the DFT window
    int dev = 0;
    // 3-D vacuum planes (see vacuum_plane in kernels.hpp): per plane z the box
    // of cells whose eps_r differs from 1 (eps_box) and the box the kernels
    // use (run_box: also every cell that may still hold non-zero rest
    // populations since the last reset); vbox is the device copy of run_box
    std::vector<int4> eps_box, run_box;
    int4 *vbox = nullptr;
    mutable bool state_clean = true;    // both state buffers are zero (created or reset, never stepped)
    // inverse design (adjoint)
    bool adj_set = false;
    lbm_em *adj_inc = nullptr;
    std::vector<double> adj_theta, adj_w;           // radians from khat, weights
    int dlo[2] = {0, 0}, dhi[2] = {0, 0};
    int ck_every = 0, nck = 0, ck_k = 0;
    int64_t adj_T = 0;
    void *ck = nullptr;                              // nck checkpoints of the state
    size_t ck_bytes = 0;
    double *adj_P = nullptr;                         // far-field combinations at adj_theta
    double adj_kappa = 0.0;
};

// A batch: several 2-D handles advanced by one persistent launch per step.
// Instances are packed, in order, into groups whose state fits a cache
// budget (the 256 MB Infinity Cache by default); each group is advanced the
// requested number of steps before the next one, so a group's working set
// stays cache resident.  An instance that fills the device on its own (two
// steps per launch, at least one tile of its own two-step tile per compute
// unit) forms a group by itself that the single-instance kernels advance:
// the persistent kernel only pays where instances are too small to fill
// the chip.  Instances are independent and every kernel runs the same
// per-cell update, so neither choice changes any result.
struct BatchGroup {
    int first = 0, count = 0;              // instance range
    bool direct = false;                   // one instance, stepped by its own kernels
    void *descs[2] = {nullptr, nullptr};   // StepArgs per instance, for buffer parity 0 / 1
    int *tile_inst = nullptr, *tile_first = nullptr;
    int ntiles = 0, grid = 0;
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [meets a DFT window][parity]
};

struct lbm_em_batch_s {
    std::vector<lbm_em *> hs;
    std::vector<BatchGroup> groups;
    int pol = 0, precision = 0, vx = 1, bx = 128, by = 2;
    int fuse = 1, ftx = 64, fty = 16;   // two steps per launch with this tile
    int64_t *t_dev = nullptr;
    hipStream_t stream = nullptr;
    int dev = 0, cus = 1, grid_override = 0;
    int64_t budget = 0;
    // instances on their own kernels alternate over two side streams forked
    // from and joined back into `stream`: two independent step kernels
    // overlap each other's load, compute and store phases
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
};

namespace {

lbm_em *check_handle(lbm_em_handle h) {
    if (!h) fail(LBM_EM_EINVAL, "null handle");
    return h;
}

void select_device(const lbm_em *h) { hip_check(hipSetDevice(h->dev), "hipSetDevice"); }

void sync(const lbm_em *h) { hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize"); }

// Cells of the incident line: the grid's extent along the line's axis.
int64_t line_len(const lbm_em *h) {
    return h->line_axis == 0 ? h->cfg.nx : h->line_axis == 1 ? h->cfg.ny : h->cfg.nz;
}

template <typename T>
StepArgs<T> make_args(const lbm_em *h, const void *src, void *dst) {
    StepArgs<T> a{};
    a.nx = h->cfg.nx;
    a.ny = h->cfg.ny;
    a.nz = h->cfg.nz;
    a.sy = h->sy;
    a.sz = h->sz;
    a.plane = h->plane;
    for (int k = 0; k < 3; ++k) {
        a.W[k] = h->cfg.absorb[k];
        a.inv_w[k] = a.W[k] > 0 ? T(1) / (T)a.W[k] : T(0);
    }
    a.sigma_max = (T)h->cfg.sigma_max;
    a.src = (const T *)src;
    a.dst = (T *)dst;
    a.eps = (const T *)h->eps;
    a.mu = (const T *)h->mu;
    a.vbox = h->vbox;
    a.src_on = h->src_on ? 1 : 0;
    a.period = h->period > 0 ? h->period : 1;
    if (h->src_on) {
        a.amp = h->pw.amplitude;
        a.t_ramp = h->pw.ramp_periods * (double)h->period;
        for (int k = 0; k < 3; ++k) {
            a.ehat[k] = (T)h->pw.ehat[k];
            a.hhat[k] = (T)h->hhat[k];
        }
        // table layout: see lbm_em_set_source
        const double2 *w = (const double2 *)h->wtab;
        a.wave_t = w;
        a.ramp = (const double *)(w + h->period);
        using C2 = typename Cplx<T>::type;
        a.wave_x = (const C2 *)(h->wtab + h->axes_off);
        a.wave_y = a.wave_x + h->cfg.nx;
        a.wave_z = a.wave_y + h->cfg.ny;
    }
    a.dft_on = h->dft_set ? 1 : 0;
    a.box = h->box;
    for (int k = 0; k < 3; ++k) a.probe[k] = h->probe[k];
    a.nnodes = h->nnodes;
    a.win0 = h->win0;
    a.winlen = h->winlen;
    a.acc = h->acc;
    if (h->line) {
        a.line_tab = (const T *)h->line_tab;
        a.line_axis = h->line_axis;
        a.line_n = line_len(h);
    }
    return a;
}

template <typename T>
void launch_step_t(const lbm_em *h, const void *src, void *dst, const int64_t *t_base,
                   int64_t t_off, hipStream_t s, bool dft, void *hist, int64_t hist_t0) {
    h->state_clean = false;
    StepArgs<T> a = make_args<T>(h, src, dst);
    a.t_base = t_base;
    a.t_off = t_off;
    if (!dft) a.dft_on = 0;
    if (hist) {
        a.hist = (T *)hist;
        a.hist_t0 = hist_t0;
        for (int k = 0; k < 2; ++k) {
            a.dlo[k] = h->dlo[k];
            a.dhi[k] = h->dhi[k];
        }
    }
    if (hist && (a.mu || a.line_tab)) fail(LBM_EM_EUNSUPPORTED, "the adjoint needs mu_r = 1 and no incident line");
    if (a.mu && h->dim != 2) fail(LBM_EM_EUNSUPPORTED, "a permeability map needs a 2-D (TM/TE) handle");
    launch_step1<T>(a, h->cfg.pol, h->vx, h->bx, h->by, s);
}

// Largest line (in cells) whose state the LDS kernels hold: 64 KB of LDS,
// two cells per thread (2-D) or one (3-D).
bool line_in_lds(const lbm_em *h) {
    const int64_t n = line_len(h);
    return n <= (h->dim == 2 ? 2048 : 1024) && h->nplanes * n * (int64_t)h->elem <= 65536;
}

// The incident line's steps for the grid launches that follow: nsteps from
// step t_base + t_off, leaving the line at parity p ^ 1 (one grid launch
// follows) or p (a graph chunk, an even number of launches: flip = false).
// Lines that fit in LDS run all steps in one block with the state in LDS;
// longer ones take at most two steps per launch through global memory and
// the line's middle buffer.
template <typename T>
void launch_line_t(const lbm_em *h, int parity, const int64_t *t_base, int64_t t_off, hipStream_t s, int nsteps,
                   bool flip = true) {
    const lbm_em *l = h->line;
    if (line_in_lds(h)) {
        StepArgs<T> a = make_args<T>(l, l->buf[parity], nullptr);
        a.t_base = t_base;
        a.t_off = t_off;
        a.dft_on = h->dft_set ? 1 : 0;
        a.win0 = h->win0;
        a.winlen = h->winlen;
        a.line_rec = (T *)h->line_tab;
        a.line_acc = h->line_acc;
        a.line_axis = h->line_axis;
        a.line_n = line_len(h);
        T *dst = (T *)l->buf[flip ? parity ^ 1 : parity];
        const size_t lds = (size_t)h->nplanes * a.line_n * sizeof(T);
        if (h->cfg.pol == LBM_EM_TM) hipLaunchKernelGGL((k_line_lds<T, TM>), dim3(1), dim3(1024), lds, s, a, dst, nsteps);
        else if (h->cfg.pol == LBM_EM_TE) hipLaunchKernelGGL((k_line_lds<T, TE>), dim3(1), dim3(1024), lds, s, a, dst, nsteps);
        else hipLaunchKernelGGL((k_line3d_lds<T>), dim3(1), dim3(1024), lds, s, a, dst, nsteps);
        hip_check(hipGetLastError(), "k_line_lds");
        return;
    }
    if (nsteps > 2 || !flip) fail(LBM_EM_EINVAL, "internal: global-memory line steps are per grid launch");
    StepArgs<T> a0 = make_args<T>(l, l->buf[parity], nsteps == 2 ? h->line_tmp : l->buf[parity ^ 1]);
    StepArgs<T> a1 = make_args<T>(l, h->line_tmp, l->buf[parity ^ 1]);
    for (StepArgs<T> *a : {&a0, &a1}) {
        a->t_base = t_base;
        a->dft_on = h->dft_set ? 1 : 0;
        a->win0 = h->win0;
        a->winlen = h->winlen;
        a->line_rec = (T *)h->line_tab;
        a->line_acc = h->line_acc;
        a->line_axis = h->line_axis;
        a->line_n = line_len(h);
    }
    a0.t_off = t_off;
    a1.t_off = t_off + 1;
    if (h->cfg.pol == LBM_EM_TM) hipLaunchKernelGGL((k_line<T, TM>), dim3(1), dim3(1024), 0, s, a0, a1, nsteps);
    else if (h->cfg.pol == LBM_EM_TE) hipLaunchKernelGGL((k_line<T, TE>), dim3(1), dim3(1024), 0, s, a0, a1, nsteps);
    else hipLaunchKernelGGL((k_line3d<T>), dim3(1), dim3(1024), 0, s, a0, a1, nsteps);
    hip_check(hipGetLastError(), "k_line");
}

void launch_line(const lbm_em *h, int parity, const int64_t *t_base, int64_t t_off, hipStream_t s, int nsteps,
                 bool flip = true) {
    if (h->cfg.precision == LBM_EM_FP32) launch_line_t<float>(h, parity, t_base, t_off, s, nsteps, flip);
    else launch_line_t<double>(h, parity, t_base, t_off, s, nsteps, flip);
}

// One step.  dft = false (autotune timing, adjoint recompute): no DFT and
// no incident-line step (the line's table is left as it is).  line = false:
// the caller has already advanced the incident line over these steps.
void launch_step(const lbm_em *h, int parity, const int64_t *t_base, int64_t t_off, hipStream_t s,
                 bool dft = true, void *hist = nullptr, int64_t hist_t0 = 0, bool line = true) {
    if (h->line && dft && line) launch_line(h, parity, t_base, t_off, s, 1);
    const void *src = h->buf[parity];
    void *dst = h->buf[parity ^ 1];
    if (h->cfg.precision == LBM_EM_FP32) launch_step_t<float>(h, src, dst, t_base, t_off, s, dft, hist, hist_t0);
    else launch_step_t<double>(h, src, dst, t_base, t_off, s, dft, hist, hist_t0);
}

// Two steps in one launch: reads src, writes f*(t+1) to dst.

// Stride between population planes, in elements: the plane's cells rounded
// up to an odd multiple of 4 KiB.  At strides that are multiples of large
// powers of two (a 512^3 FP32 plane is 2^29 bytes) the 24-54 concurrent
// plane streams of a launch meet the memory channels in step: 24 planes in
// and 24 out at 512^3 (lbm_em_stream_bandwidth) stream at 5.35 TB/s with
// the bare stride and at 5.80 TB/s with this one (384^3, whose plane
// already has an odd factor, is unaffected).
int64_t plane_stride(int64_t cells, int64_t elem) {
    const int64_t unit = 4096 / elem;
    int64_t p = (cells + unit - 1) / unit;
    if (p % 2 == 0) ++p;
    return p * unit;
}

// z chunk of the 3-D two-step kernel: each block marches zc planes plus two
// extra ones (at most kX3MaxPlanes in all); pick the chunk count that
// minimises rounds x (zc + 2).
int x3_chunk(int nz, int tiles, int slots) {
    int best_zc = std::min(nz, kX3MaxPlanes - 2);
    int64_t best = INT64_MAX;
    for (int n = 1; n <= nz; ++n) {
        const int zc = (nz + n - 1) / n;
        if (zc + 2 > kX3MaxPlanes) continue;
        const int64_t blocks = (int64_t)tiles * ((nz + zc - 1) / zc);
        const int64_t rounds = (blocks + slots - 1) / slots;
        const int64_t cost = rounds * (zc + 2);
        if (cost < best) {
            best = cost;
            best_zc = zc;
        }
    }
    return best_zc;
}

// Whether a two-step launch may meet the DFT window: steps t_off and
// t_off + 1, or a captured chunk flagged so.  Only such launches take the
// kernel instantiation that carries the contour accumulation.
template <typename T>
bool launch_meets_window(const lbm_em *h, const StepArgs<T> &a) {
    return a.dft_on && (a.t_base ? h->graph_dft : (a.t_off + 2 > h->win0 && a.t_off < h->win0 + h->winlen));
}

template <typename T>
void launch_step2_3d(const lbm_em *h, StepArgs<T> a, hipStream_t s) {
    const int tx = h->ftx, ty = h->fty;
    a.tiles_x = (a.nx + tx - 1) / tx;
    a.tiles_y = (a.ny + ty - 1) / ty;
    const int tiles = a.tiles_x * a.tiles_y;
    const int zc = x3_chunk(a.nz, tiles, h->cus * std::max(1, 1024 / (tx * ty)));
    if (!launch_step3d_x2<T>(a, tx, ty, zc, launch_meets_window(h, a), s))
        fail(LBM_EM_EINVAL, "unsupported 3-D two-step tile or z chunk");
}

template <typename T>
void launch_step2_2d(const lbm_em *h, StepArgs<T> a, hipStream_t s) {
    const int tx = h->ftx, ty = h->fty;
    a.tiles_x = (a.nx + tx - 1) / tx;
    a.tiles_y = (a.ny + ty - 1) / ty;
    if (!launch_step2d_x2<T>(a, h->cfg.pol, tx, ty, launch_meets_window(h, a), s))
        fail(LBM_EM_EINVAL, "unsupported two-step tile");
}

template <typename T>
void launch_step2_t(const lbm_em *h, const void *src, void *dst, const int64_t *t_base, int64_t t_off,
                    hipStream_t s, bool dft, void *hist = nullptr, int64_t hist_t0 = 0) {
    h->state_clean = false;
    StepArgs<T> a = make_args<T>(h, src, dst);
    a.t_base = t_base;
    a.t_off = t_off;
    if (!dft) a.dft_on = 0;
    if (hist) {
        a.hist = (T *)hist;
        a.hist_t0 = hist_t0;
        for (int k = 0; k < 2; ++k) {
            a.dlo[k] = h->dlo[k];
            a.dhi[k] = h->dhi[k];
        }
    }
    if (h->cfg.pol == LBM_EM_TM || h->cfg.pol == LBM_EM_TE) launch_step2_2d<T>(h, a, s);
    else launch_step2_3d<T>(h, a, s);
}

void launch_step2(const lbm_em *h, int parity, const int64_t *t_base, int64_t t_off, hipStream_t s,
                  bool dft = true, void *hist = nullptr, int64_t hist_t0 = 0, bool line = true) {
    if ((h->mu || h->line) && hist) fail(LBM_EM_EUNSUPPORTED, "the adjoint needs mu_r = 1 and no incident line");
    if (h->line && dft && line) launch_line(h, parity, t_base, t_off, s, 2);
    const void *src = h->buf[parity];
    void *dst = h->buf[parity ^ 1];
    if (h->cfg.precision == LBM_EM_FP32) launch_step2_t<float>(h, src, dst, t_base, t_off, s, dft, hist, hist_t0);
    else launch_step2_t<double>(h, src, dst, t_base, t_off, s, dft, hist, hist_t0);
}

bool fused_tile_ok(int dim, int precision, int tx, int ty) {
#define LBM_X2_OK(TX, TY) if (tx == TX && ty == TY) return true;
    if (dim == 3) {
        if (precision == LBM_EM_FP32) { LBM_X3_TILES_F32(LBM_X2_OK) }
        else { LBM_X3_TILES_F64(LBM_X2_OK) }
    } else if (precision == LBM_EM_FP32) { LBM_X2_TILES_F32(LBM_X2_OK) }
    else { LBM_X2_TILES_F64(LBM_X2_OK) }
#undef LBM_X2_OK
    return false;
}

bool tile_ok(const lbm_em *h, int vx, int bx, int by) {
    const bool vx_ok = vx == 1 || vx == 2 || (vx == 4 && h->cfg.precision == LBM_EM_FP32);
    const int th = bx * by;
    return vx_ok && bx >= 1 && by >= 1 && th >= 64 && th <= 256 && th % 64 == 0;
}

void drop_graphs(lbm_em *h) {
    for (auto &gw : h->graph)
        for (auto &g : gw)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

// Capture kGraphChunk steps (starting from buffer parity p) plus the device
// step-counter advance into one executable graph.  win: the chunks it will
// replay may meet the DFT window (selects the two-step kernels'
// instantiation with the contour accumulation).
hipGraphExec_t build_graph(lbm_em *h, int p, bool win) {
    hipStream_t cs = nullptr;
    hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        hip_check(e, "hipStreamBeginCapture");
    }
    int par = p;
    h->graph_dft = win;
    // an incident line held in LDS takes the whole chunk in one launch up front
    const bool line_chunk = h->line && line_in_lds(h);
    if (line_chunk) launch_line(h, p, h->t_dev, 0, cs, kGraphChunk, false);
    if (h->fuse == 2) {
        for (int k = 0; k < kGraphChunk; k += 2) {
            launch_step2(h, par, h->t_dev, k, cs, true, nullptr, 0, !line_chunk);
            par ^= 1;
        }
    } else {
        for (int k = 0; k < kGraphChunk; ++k) {
            launch_step(h, par, h->t_dev, k, cs, true, nullptr, 0, !line_chunk);
            par ^= 1;
        }
    }
    hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, cs, h->t_dev, (int64_t)kGraphChunk);
    h->graph_dft = true;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    hip_check(e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "hipGraphInstantiate");
    return ge;
}

// `on`: the stream to order the work on (default: the handle's own).
void do_steps(lbm_em *h, int64_t n, hipStream_t on = nullptr) {
    select_device(h);
    hipStream_t st = on ? on : h->stream;
    int64_t chunks = n / kGraphChunk;
    if (chunks > 0) {
        hipLaunchKernelGGL(k_set_time, dim3(1), dim3(64), 0, st, h->t_dev, h->t);
        hip_check(hipGetLastError(), "k_set_time");
        for (int64_t c = 0; c < chunks; ++c) {
            // chunks outside the DFT window replay the graph whose kernels
            // carry no contour accumulation
            const int64_t tc = h->t + c * kGraphChunk;
            const int win = h->dft_set && tc < h->win0 + h->winlen && tc + kGraphChunk > h->win0;
            if (!h->graph[win][h->cur]) h->graph[win][h->cur] = build_graph(h, h->cur, win);
            hip_check(hipGraphLaunch(h->graph[win][h->cur], st), "hipGraphLaunch");
            // a chunk flips the buffers an even number of times (32 fused
            // or 64 single launches): the parity is unchanged
        }
        h->t += chunks * kGraphChunk;
    }
    int64_t rest = n - chunks * kGraphChunk;
    if (h->fuse == 2) {
        for (; rest >= 2; rest -= 2) {
            launch_step2(h, h->cur, nullptr, h->t, st);
            hip_check(hipGetLastError(), "fused step kernel launch");
            h->cur ^= 1;
            h->t += 2;
        }
    }
    for (int64_t k = 0; k < rest; ++k) {
        launch_step(h, h->cur, nullptr, h->t, st);
        hip_check(hipGetLastError(), "step kernel launch");
        h->cur ^= 1;
        h->t += 1;
    }
}

int64_t handle_bytes(const lbm_em *h) { return (int64_t)h->plane * (2 * h->nplanes + 1) * (int64_t)h->elem; }

// dft = false: descriptors for timing launches (no DFT accumulation).
template <typename T>
void fill_group(lbm_em_batch_s *b, BatchGroup &g, bool dft) {
    std::vector<int> first;
    for (int par = 0; par < 2; ++par) {
        std::vector<StepArgs<T>> d(g.count);
        for (int i = 0; i < g.count; ++i) {
            const lbm_em *h = b->hs[g.first + i];
            d[i] = make_args<T>(h, h->buf[par], h->buf[par ^ 1]);
            if (!dft) d[i].dft_on = 0;
            if (b->fuse == 2) {
                d[i].tiles_x = (h->cfg.nx + b->ftx - 1) / b->ftx;
                d[i].tiles_y = (h->cfg.ny + b->fty - 1) / b->fty;
            } else {
                d[i].tiles_x = ((h->cfg.nx + b->vx - 1) / b->vx + b->bx - 1) / b->bx;
                d[i].tiles_y = (h->cfg.ny + b->by - 1) / b->by;
            }
        }
        if (par == 0) {
            int acc = 0;
            for (auto &x : d) {
                first.push_back(acc);
                acc += x.tiles_x * x.tiles_y;
            }
            g.ntiles = acc;
        }
        hip_check(hipMalloc(&g.descs[par], d.size() * sizeof(StepArgs<T>)), "hipMalloc batch");
        hip_check(hipMemcpyAsync(g.descs[par], d.data(), d.size() * sizeof(StepArgs<T>), hipMemcpyHostToDevice,
                                 b->stream), "H2D batch");
    }
    std::vector<int> inst(g.ntiles);
    for (int i = 0; i < g.count; ++i) {
        const int end = i + 1 < g.count ? first[i + 1] : g.ntiles;
        for (int w = first[i]; w < end; ++w) inst[w] = i;
    }
    hip_check(hipMalloc(&g.tile_inst, inst.size() * sizeof(int)), "hipMalloc batch");
    hip_check(hipMalloc(&g.tile_first, first.size() * sizeof(int)), "hipMalloc batch");
    hip_check(hipMemcpyAsync(g.tile_inst, inst.data(), inst.size() * sizeof(int), hipMemcpyHostToDevice, b->stream),
              "H2D batch");
    hip_check(hipMemcpyAsync(g.tile_first, first.data(), first.size() * sizeof(int), hipMemcpyHostToDevice,
                             b->stream), "H2D batch");
    g.grid = std::min(g.ntiles, b->grid_override > 0 ? b->grid_override : b->cus * 32);
}

// One launch of the batch.  With fused tiles (b->fuse == 2) `steps` is 2
// (two-step kernel) or 1 (a single step on the same tiles).  dft: the launch
// may meet the DFT window of an instance of the group.
template <typename T>
void launch_batch_t(const lbm_em_batch_s *b, const BatchGroup &g, int par, const int64_t *t_base, int64_t t_off,
                    hipStream_t s, int steps, bool dft) {
    const StepArgs<T> *d = (const StepArgs<T> *)g.descs[par];
    if (b->fuse == 2) {
        if (!launch_batch_x2<T>(d, b->pol, b->ftx, b->fty, steps != 1, dft, g.grid, g.tile_inst, g.tile_first,
                                g.ntiles, t_base, t_off, s))
            fail(LBM_EM_EINVAL, "unsupported two-step tile");
    } else {
        launch_batch1<T>(d, b->pol, b->vx, b->bx, b->by, g.grid, g.tile_inst, g.tile_first, g.ntiles, t_base, t_off,
                         s);
    }
}

void launch_batch(const lbm_em_batch_s *b, const BatchGroup &g, int par, const int64_t *t_base, int64_t t_off,
                  hipStream_t s, int steps = 0, bool dft = true) {
    if (b->precision == LBM_EM_FP32) launch_batch_t<float>(b, g, par, t_base, t_off, s, steps, dft);
    else launch_batch_t<double>(b, g, par, t_base, t_off, s, steps, dft);
}

// Whether steps [t0, t0 + len) meet the DFT window of an instance of group g.
bool group_meets_window(const lbm_em_batch_s *b, const BatchGroup &g, int64_t t0, int64_t len) {
    for (int i = 0; i < g.count; ++i) {
        const lbm_em *h = b->hs[g.first + i];
        if (h->dft_set && t0 < h->win0 + h->winlen && t0 + len > h->win0) return true;
    }
    return false;
}

void free_groups(lbm_em_batch_s *b) {
    for (auto &g : b->groups) {
        for (auto &gw : g.graph)
            for (auto &ge : gw)
                if (ge) (void)hipGraphExecDestroy(ge);
        hfree(g.descs[0]);
        hfree(g.descs[1]);
        hfree(g.tile_inst);
        hfree(g.tile_first);
    }
    b->groups.clear();
}

void free_batch(lbm_em_batch_s *b) {
    if (!b) return;
    (void)hipSetDevice(b->dev);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    free_groups(b);
    hfree(b->t_dev);
    for (int k = 0; k < 2; ++k) {
        if (b->side[k]) (void)hipStreamSynchronize(b->side[k]);
        if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (lbm_em *h : b->hs) --h->batch_refs;
    delete b;
}

// (Re)build the groups for the current cache budget and grid setting.
// The instance fills the device by itself: two steps per launch (like the
// batch) with at least one of its own two-step tiles per compute unit.
bool batch_direct(const lbm_em_batch_s *b, const lbm_em *h) {
    if (b->fuse != 2 || h->fuse != 2) return false;
    const int64_t tiles = (int64_t)((h->cfg.nx + h->ftx - 1) / h->ftx) * ((h->cfg.ny + h->fty - 1) / h->fty);
    return tiles >= b->cus;
}

void plan_batch(lbm_em_batch_s *b, bool dft = true) {
    if (b->stream) hip_check(hipStreamSynchronize(b->stream), "sync");
    free_groups(b);
    const int n = (int)b->hs.size();
    int i = 0;
    while (i < n) {
        BatchGroup g;
        g.first = i;
        if (batch_direct(b, b->hs[i])) {
            g.count = 1;
            g.direct = true;
            b->groups.push_back(g);
            ++i;
            continue;
        }
        int64_t bytes = 0;
        do {
            bytes += handle_bytes(b->hs[i]);
            ++i;
        } while (i < n && !batch_direct(b, b->hs[i]) &&
                 (b->budget <= 0 || bytes + handle_bytes(b->hs[i]) <= b->budget));
        g.count = i - g.first;
        b->groups.push_back(g);
        if (b->precision == LBM_EM_FP32) fill_group<float>(b, b->groups.back(), dft);
        else fill_group<double>(b, b->groups.back(), dft);
    }
    hip_check(hipStreamSynchronize(b->stream), "sync");
}

lbm_em_batch_s *make_batch(const lbm_em_handle *hs, int32_t count) {
    if (!hs || count < 1) fail(LBM_EM_EINVAL, "need at least one handle");
    lbm_em *h0 = check_handle(hs[0]);
    for (int i = 0; i < count; ++i) {
        lbm_em *h = check_handle(hs[i]);
        if (h->dim != 2) fail(LBM_EM_EUNSUPPORTED, "batched stepping supports 2-D (TM/TE) handles");
        if (h->mu) fail(LBM_EM_EUNSUPPORTED, "batched stepping needs mu_r = 1");
        if (h->line) fail(LBM_EM_EUNSUPPORTED, "batched stepping does not run incident lines");
        if (h->cfg.pol != h0->cfg.pol || h->cfg.precision != h0->cfg.precision)
            fail(LBM_EM_EINVAL, "batched handles must share polarisation and precision");
        if (h->stream != h0->stream || h->dev != h0->dev) fail(LBM_EM_EINVAL, "batched handles must share stream and device");
        if (h->t != h0->t || h->cur != h0->cur) fail(LBM_EM_ESTATE, "batched handles must be at the same time step");
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) fail(LBM_EM_EINVAL, "a handle appears twice in the batch");
    }
    select_device(h0);
    lbm_em_batch_s *b = new lbm_em_batch_s();
    try {
        b->dev = h0->dev;
        b->stream = h0->stream;
        b->pol = h0->cfg.pol;
        b->precision = h0->cfg.precision;
        b->vx = h0->vx;
        b->bx = h0->bx;
        b->by = h0->by;
        b->fuse = h0->fuse;
        b->ftx = h0->ftx;
        b->fty = h0->fty;
        hip_check(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->dev), "attribute");
        b->cus = std::max(1, b->cus);
        if (b->fuse == 2) {
            // Two-step tile of the batch: the fewest padded cells over the
            // instances (small, uneven grids waste much of a large tile);
            // the handles' own tile when it is among the best, else the
            // largest of them.
            auto padded = [&](int tx, int ty) {
                int64_t p = 0;
                for (int i = 0; i < count; ++i) {
                    const lbm_em *h = hs[i];
                    if (batch_direct(b, h)) continue;   // advanced by its own kernels
                    p += (int64_t)((h->cfg.nx + tx - 1) / tx) * tx * (int64_t)((h->cfg.ny + ty - 1) / ty) * ty;
                }
                return p;
            };
            int64_t best = padded(b->ftx, b->fty);
            int btx = b->ftx, bty = b->fty;
#define LBM_X2_PICK(TX, TY)                                                                        \
    {                                                                                              \
        const int64_t p = padded(TX, TY);                                                          \
        if (p < best || (p == best && (btx != b->ftx || bty != b->fty) && TX * TY > btx * bty)) { \
            best = p;                                                                              \
            btx = TX;                                                                              \
            bty = TY;                                                                              \
        }                                                                                          \
    }
            if (b->precision == LBM_EM_FP32) { LBM_X2_TILES_F32(LBM_X2_PICK) }
            else { LBM_X2_TILES_F64(LBM_X2_PICK) }
#undef LBM_X2_PICK
            b->ftx = btx;
            b->fty = bty;
        }
        b->budget = (int64_t)192 << 20;
        for (int i = 0; i < count; ++i) {
            b->hs.push_back(hs[i]);
            ++hs[i]->batch_refs;
        }
        hip_check(hipMalloc(&b->t_dev, 64), "hipMalloc batch");
        plan_batch(b);
    } catch (...) {
        free_batch(b);
        throw;
    }
    return b;
}

// win: the chunks it replays may meet a DFT window of the group.
hipGraphExec_t build_batch_graph(lbm_em_batch_s *b, const BatchGroup &grp, int p, bool win) {
    hipStream_t cs = nullptr;
    hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        hip_check(e, "hipStreamBeginCapture");
    }
    int par = p;
    for (int k = 0; k < kGraphChunk; k += b->fuse) {
        launch_batch(b, grp, par, b->t_dev, k, cs, 0, win);
        par ^= 1;
    }
    hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, cs, b->t_dev, (int64_t)kGraphChunk);
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    hip_check(e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "hipGraphInstantiate");
    return ge;
}

void batch_steps(lbm_em_batch_s *b, int64_t n, bool use_graph) {
    lbm_em *h0 = b->hs[0];
    for (auto *h : b->hs)
        if (h->t != h0->t || h->cur != h0->cur)
            fail(LBM_EM_ESTATE, "batched handles were stepped separately since the batch was made");
    (void)hipSetDevice(b->dev);
    // a handle's launch shape may have changed since the plan was made
    bool stale = false;
    for (const auto &g : b->groups)
        for (int i = 0; i < g.count; ++i) stale = stale || batch_direct(b, b->hs[g.first + i]) != g.direct;
    if (stale) plan_batch(b);
    const int64_t t_start = h0->t;
    const int cur_start = h0->cur;
    int64_t t = t_start;
    int cur = cur_start;
    int ndirect = 0;
    for (const auto &g : b->groups) ndirect += g.direct ? 1 : 0;
    const bool two = ndirect >= 2 && n > 0;
    if (two) {
        for (int k = 0; k < 2; ++k) {
            if (!b->side[k]) hip_check(hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking), "hipStreamCreate");
            if (!b->join[k]) hip_check(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming), "hipEventCreate");
        }
        if (!b->fork) hip_check(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "hipEventCreate");
        hip_check(hipEventRecord(b->fork, b->stream), "hipEventRecord");
        for (int k = 0; k < 2; ++k) hip_check(hipStreamWaitEvent(b->side[k], b->fork, 0), "hipStreamWaitEvent");
    }
    int jd = 0;
    for (auto &g : b->groups) {
        t = t_start;
        cur = cur_start;
        if (g.direct) {
            do_steps(b->hs[g.first], n, two ? b->side[jd++ & 1] : nullptr);
            continue;
        }
        int64_t chunks = use_graph ? n / kGraphChunk : 0;
        if (chunks > 0) {
            hipLaunchKernelGGL(k_set_time, dim3(1), dim3(64), 0, b->stream, b->t_dev, t);
            hip_check(hipGetLastError(), "k_set_time");
            for (int64_t c = 0; c < chunks; ++c) {
                // chunks outside every DFT window of the group replay the
                // graph whose kernels carry no contour accumulation
                const int win = group_meets_window(b, g, t + c * kGraphChunk, kGraphChunk);
                if (!g.graph[win][cur]) g.graph[win][cur] = build_batch_graph(b, g, cur, win);
                hip_check(hipGraphLaunch(g.graph[win][cur], b->stream), "hipGraphLaunch");
            }
            t += chunks * kGraphChunk;
        }
        int64_t rest = n - chunks * kGraphChunk;
        while (rest > 0) {
            const int adv = (b->fuse == 2 && rest >= 2) ? 2 : 1;   // a trailing odd step runs alone
            launch_batch(b, g, cur, nullptr, t, b->stream, adv, group_meets_window(b, g, t, adv));
            hip_check(hipGetLastError(), "batch kernel launch");
            cur ^= 1;
            t += adv;
            rest -= adv;
        }
    }
    if (two)
        for (int k = 0; k < 2; ++k) {
            hip_check(hipEventRecord(b->join[k], b->side[k]), "hipEventRecord");
            hip_check(hipStreamWaitEvent(b->stream, b->join[k], 0), "hipStreamWaitEvent");
        }
    // the buffer parity after n steps: graph chunks flip it an even number
    // of times and every other launch once, in the batched and in the
    // single-instance path alike
    t = t_start + n;
    const int64_t rest = use_graph ? n % kGraphChunk : n;
    cur = cur_start ^ (int)((b->fuse == 2 ? rest / 2 + rest % 2 : rest) & 1);
    for (auto *h : b->hs) {
        if (h->t != t || h->cur != cur) {
            if (h->t != t_start) fail(LBM_EM_ESTATE, "batched instance left at an unexpected step");
            h->t = t;
            h->cur = cur;
        }
    }
}

// The incident line's phasors laid out like the contour accumulators (one
// row of 12 per box node, then the probe), in a new device buffer.
double *line_incident(lbm_em *h) {
    const int64_t n = line_len(h);
    std::vector<double> L((size_t)n * 12), out((size_t)(h->nnodes + 1) * 12);
    hip_check(hipMemcpyAsync(L.data(), h->line_acc, L.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream), "D2H");
    sync(h);
    const Box &b = h->box;
    for (int z = b.lo[2]; z <= b.hi[2]; ++z)
        for (int y = b.lo[1]; y <= b.hi[1]; ++y)
            for (int x = b.lo[0]; x <= b.hi[0]; ++x) {
                if (!on_box(b, h->dim, x, y, z)) continue;
                const int64_t node = box_node_index(b, h->dim, x, y, z);
                const int u = h->line_axis == 0 ? x : h->line_axis == 1 ? y : z;
                std::memcpy(&out[(size_t)node * 12], &L[(size_t)u * 12], 12 * sizeof(double));
            }
    const int up = h->probe[h->line_axis];
    std::memcpy(&out[(size_t)h->nnodes * 12], &L[(size_t)up * 12], 12 * sizeof(double));
    double *d = nullptr;
    hip_check(hipMalloc(&d, out.size() * sizeof(double)), "hipMalloc");
    hip_check(hipMemcpyAsync(d, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, h->stream), "H2D");
    sync(h);
    return d;
}

// Far-field combinations P (4 doubles per angle, device) for angles given
// in radians; returns the incident amplitude used for normalisation.
double farfield_P(lbm_em *h, const double *acc_inc, const double *theta_rad, const double *phi_rad, int n,
                  double *d_P) {
    std::vector<double> ang(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        ang[i] = theta_rad[i];
        ang[n + i] = phi_rad ? phi_rad[i] : 0.0;
    }
    double *d_ang = nullptr;
    hip_check(hipMalloc(&d_ang, ang.size() * sizeof(double)), "hipMalloc");
    hip_check(hipMemcpyAsync(d_ang, ang.data(), ang.size() * sizeof(double), hipMemcpyHostToDevice, h->stream), "H2D");
    NtffArgs a{};
    a.acc = h->acc;
    a.acc_inc = acc_inc;
    a.box = h->box;
    a.dim = h->dim;
    a.pol = h->cfg.pol;
    a.k = 2.0 * M_PI / h->pw.lambda;
    const auto &c = h->cfg;
    a.center[0] = (c.nx - 1) / 2.0;
    a.center[1] = (c.ny - 1) / 2.0;
    a.center[2] = h->dim == 3 ? (c.nz - 1) / 2.0 : 0.0;
    for (int k = 0; k < 3; ++k) {
        a.khat[k] = h->pw.khat[k];
        a.ehat[k] = h->pw.ehat[k];
        a.bhat[k] = h->hhat[k];
    }
    a.theta = d_ang;
    a.phi = d_ang + n;
    a.out = d_P;
    hipLaunchKernelGGL(k_ntff, dim3(n), dim3(256), 0, h->stream, a);
    hip_check(hipGetLastError(), "k_ntff");
    double amp = h->pw.amplitude;
    if (acc_inc) {
        double pr[12];
        hip_check(hipMemcpyAsync(pr, acc_inc + h->nnodes * 12, sizeof pr, hipMemcpyDeviceToHost, h->stream), "D2H");
        sync(h);
        const double *v = h->cfg.pol == LBM_EM_TE ? pr + 6 : pr;
        const double *u = h->cfg.pol == LBM_EM_TE ? h->hhat : h->pw.ehat;
        double re = 0, im = 0;
        for (int k = 0; k < 3; ++k) {
            re += u[k] * v[2 * k];
            im += u[k] * v[2 * k + 1];
        }
        amp = std::sqrt(re * re + im * im);
    }
    sync(h);
    hfree(d_ang);
    return amp;
}

void check_incident(const lbm_em *h, const lbm_em *inc) {
    if (inc->cfg.nx != h->cfg.nx || inc->cfg.ny != h->cfg.ny || inc->cfg.nz != h->cfg.nz ||
        inc->cfg.pol != h->cfg.pol || !inc->dft_set)
        fail(LBM_EM_EINVAL, "incident handle must match grid, polarisation and contour");
    for (int a = 0; a < 3; ++a)
        if (inc->box.lo[a] != h->box.lo[a] || inc->box.hi[a] != h->box.hi[a])
            fail(LBM_EM_EINVAL, "incident handle has a different contour");
    if (inc->t < inc->win0 + inc->winlen) fail(LBM_EM_ESTATE, "incident DFT window not completed");
}

void upload_vbox(lbm_em *h) {
    if (!h->vbox) return;
    hip_check(hipMemcpyAsync(h->vbox, h->run_box.data(), h->run_box.size() * sizeof(int4), hipMemcpyHostToDevice,
                             h->stream), "vacuum boxes H2D");
    sync(h);
}

void reset_state(lbm_em *h) {
    const size_t bytes = (size_t)h->plane * h->nplanes * h->elem;
    hip_check(hipMemsetAsync(h->buf[0], 0, bytes, h->stream), "hipMemset state");
    hip_check(hipMemsetAsync(h->buf[1], 0, bytes, h->stream), "hipMemset state");
    // zero state: only cells with eps_r != 1 can acquire rest populations
    h->state_clean = true;
    if (h->vbox) {
        h->run_box = h->eps_box;
        upload_vbox(h);
    }
    if (h->acc)
        hip_check(hipMemsetAsync(h->acc, 0, (size_t)(h->nnodes + 1) * 12 * sizeof(double), h->stream), "hipMemset dft");
    h->t = 0;
    h->cur = 0;
    if (h->line) {
        reset_state(h->line);
        const int64_t n = line_len(h);
        hip_check(hipMemsetAsync(h->line_acc, 0, (size_t)n * 12 * sizeof(double), h->stream), "hipMemset line dft");
    }
}

template <typename T>
// One adjoint step at t, or (hist_prev given) the two steps t and t - 1.
void launch_adjoint(const lbm_em *h, const void *src, void *dst, int64_t t, const void *hist, double *grad,
                    const double *G, const void *hist_prev = nullptr) {
    AdjArgs<T> a{};
    a.nx = h->cfg.nx;
    a.ny = h->cfg.ny;
    a.sy = h->sy;
    a.plane = h->plane;
    for (int k = 0; k < 2; ++k) {
        a.W[k] = h->cfg.absorb[k];
        a.inv_w[k] = a.W[k] > 0 ? T(1) / (T)a.W[k] : T(0);
    }
    a.sigma_max = (T)h->cfg.sigma_max;
    a.src = (const T *)src;
    a.dst = (T *)dst;
    a.eps = (const T *)h->eps;
    a.t = t;
    a.box = h->box;
    a.win0 = h->win0;
    a.winlen = h->winlen;
    a.period = h->period;
    a.G = G;
    a.hist = (const T *)hist;
    a.grad = grad;
    for (int k = 0; k < 2; ++k) {
        a.dlo[k] = h->dlo[k];
        a.dhi[k] = h->dhi[k];
    }
    if (!hist_prev) {
        launch_adjoint1<T>(a, h->cfg.pol, h->stream);
        return;
    }
    // two steps (t, t - 1) on the handle's two-step tile
    a.hist_prev = (const T *)hist_prev;
    a.tiles_x = (a.nx + h->ftx - 1) / h->ftx;
    if (!launch_adjoint_x2<T>(a, h->cfg.pol, h->ftx, h->fty, h->stream)) fail(LBM_EM_EINVAL, "unsupported two-step tile");
}

void free_handle(lbm_em *h);

// Remove the incident line (its run, table and phasors).
void drop_line(lbm_em *h) {
    if (!h->line) return;
    free_handle(h->line);
    h->line = nullptr;
    hfree(h->line_tmp);
    hfree(h->line_tab);
    hfree(h->line_acc);
    h->line_tmp = h->line_tab = nullptr;
    h->line_acc = nullptr;
}

void free_handle(lbm_em *h) {
    if (!h) return;
    (void)hipSetDevice(h->dev);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    drop_graphs(h);
    hfree(h->buf[0]);
    hfree(h->buf[1]);
    hfree(h->eps);
    hfree(h->mu);
    hfree(h->pec);
    drop_line(h);
    hfree(h->acc);
    hfree(h->t_dev);
    hfree(h->ck);
    hfree(h->adj_P);
    hfree(h->wtab);
    hfree(h->vbox);
    delete h;
}

// Material map upload shared by eps_r and mu_r: validate (finite, >= 1) on
// a host copy, then convert into the padded plane `dst` of the handle.
// boxes (3-D eps_r): per plane, the box of the cells whose value is not 1.
void load_material(lbm_em *h, const void *src, int32_t where, int32_t dtype, void *dst, const char *name,
                   std::vector<int4> *boxes = nullptr) {
    if (dtype != LBM_EM_FP32 && dtype != LBM_EM_FP64) fail(LBM_EM_EINVAL, "dtype must be FP32 or FP64");
    if (where != LBM_EM_HOST && where != LBM_EM_DEVICE) fail(LBM_EM_EINVAL, "where must be HOST or DEVICE");
    select_device(h);
    const auto &c = h->cfg;
    const size_t cells = (size_t)c.nx * c.ny * c.nz;
    const size_t isz = dtype == LBM_EM_FP32 ? 4 : 8;
    std::vector<char> host(cells * isz);
    if (where == LBM_EM_HOST) std::memcpy(host.data(), src, host.size());
    else {
        hip_check(hipMemcpyAsync(host.data(), src, host.size(), hipMemcpyDeviceToHost, h->stream), "material D2H");
        sync(h);
    }
    for (size_t i = 0; i < cells; ++i) {
        double v = dtype == LBM_EM_FP32 ? ((const float *)host.data())[i] : ((const double *)host.data())[i];
        if (!std::isfinite(v) || v < 1.0) fail(LBM_EM_EINVAL, std::string(name) + " must be finite and >= 1");
    }
    if (boxes) {
        boxes->assign(c.nz, make_int4(c.nx, -1, c.ny, -1));   // empty: x_lo > x_hi
        for (size_t i = 0; i < cells; ++i) {
            const double v = dtype == LBM_EM_FP32 ? ((const float *)host.data())[i] : ((const double *)host.data())[i];
            if (v == 1.0) continue;
            const int x = (int)(i % c.nx), y = (int)(i / c.nx % c.ny), z = (int)(i / ((size_t)c.nx * c.ny));
            int4 &b = (*boxes)[z];
            b.x = std::min(b.x, x);
            b.y = std::max(b.y, x);
            b.z = std::min(b.z, y);
            b.w = std::max(b.w, y);
        }
    }
    void *d_in = nullptr;
    hip_check(hipMalloc(&d_in, host.size()), "hipMalloc");
    try {
        hip_check(hipMemcpyAsync(d_in, host.data(), host.size(), hipMemcpyHostToDevice, h->stream), "material H2D");
        dim3 grid((c.nx + 255) / 256, c.ny, c.nz);
        if (dtype == LBM_EM_FP32 && h->elem == 4)
            hipLaunchKernelGGL((k_load_eps<float, float>), grid, dim3(256), 0, h->stream, (const float *)d_in,
                               (float *)dst, c.nx, c.ny, c.nz, h->sy, h->sz);
        else if (dtype == LBM_EM_FP32)
            hipLaunchKernelGGL((k_load_eps<float, double>), grid, dim3(256), 0, h->stream, (const float *)d_in,
                               (double *)dst, c.nx, c.ny, c.nz, h->sy, h->sz);
        else if (h->elem == 4)
            hipLaunchKernelGGL((k_load_eps<double, float>), grid, dim3(256), 0, h->stream, (const double *)d_in,
                               (float *)dst, c.nx, c.ny, c.nz, h->sy, h->sz);
        else
            hipLaunchKernelGGL((k_load_eps<double, double>), grid, dim3(256), 0, h->stream, (const double *)d_in,
                               (double *)dst, c.nx, c.ny, c.nz, h->sy, h->sz);
        hip_check(hipGetLastError(), "k_load_eps");
        sync(h);
    } catch (...) {
        sync(h);
        hfree(d_in);
        throw;
    }
    hfree(d_in);
}

// Write v into the mu plane at the cells of the handle's conductor mask.
void mask_fill(lbm_em *h, double v) {
    if (!h->pec || !h->mu) return;
    const auto &c = h->cfg;
    dim3 grid((c.nx + 255) / 256, c.ny, c.nz);
    if (h->elem == 4)
        hipLaunchKernelGGL((k_mask_fill<float>), grid, dim3(256), 0, h->stream, h->pec, (float *)h->mu, (float)v,
                           c.nx, c.ny, h->sy, h->sz);
    else
        hipLaunchKernelGGL((k_mask_fill<double>), grid, dim3(256), 0, h->stream, h->pec, (double *)h->mu, v, c.nx,
                           c.ny, h->sy, h->sz);
    hip_check(hipGetLastError(), "k_mask_fill");
}

// Set every element of a padded material plane to 1.
void fill_ones(lbm_em *h, void *dst) {
    const int64_t ne = h->plane;
    const unsigned blocks = (unsigned)((ne + 255) / 256);
    if (h->elem == 4) hipLaunchKernelGGL((k_fill<float>), dim3(blocks), dim3(256), 0, h->stream, (float *)dst, ne, 1.0f);
    else hipLaunchKernelGGL((k_fill<double>), dim3(blocks), dim3(256), 0, h->stream, (double *)dst, ne, 1.0);
    hip_check(hipGetLastError(), "material init");
}

void check_unit(const double v[3], const char *name) {
    double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!std::isfinite(n) || std::fabs(n - 1.0) > 1e-9)
        fail(LBM_EM_EINVAL, std::string(name) + " must be a unit vector");
}


}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free far field (lbm_em_farfield_static).  Its device buffers --
// the angles, the far-field combinations P, |S|^2, the incident amplitude
// and the incident line's phasors on the contour nodes -- live in one
// file-scope device array, one copy per device, so a call allocates nothing.
// Host code addresses the array only through the pointer that
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr int kFfMaxAngles = LBM_EM_FARFIELD_STATIC_MAX_ANGLES;
constexpr int kFfMaxNodes = LBM_EM_FARFIELD_STATIC_MAX_NODES;
constexpr size_t kFfAng = 0;                                   // theta [max], phi [max] (radians)
constexpr size_t kFfP = kFfAng + 2 * (size_t)kFfMaxAngles;     // 4 per angle
constexpr size_t kFfS2 = kFfP + 4 * (size_t)kFfMaxAngles;      // 1 per angle
constexpr size_t kFfAmp = kFfS2 + (size_t)kFfMaxAngles;        // 1 (padded to 32)
constexpr size_t kFfLine = kFfAmp + 32;                        // (nodes + 1) x 12
constexpr size_t kFfDoubles = kFfLine + ((size_t)kFfMaxNodes + 1) * 12;

__device__ __align__(256) double lbm_ff_scratch[kFfDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_ff_mutex;
double *g_ff_ptr[kMaxDevices] = {};

// Device address of this device's copy of lbm_ff_scratch (the current
// device must be dev), looked up once per device.
double *ff_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(LBM_EM_EDEVICE, "device index out of range for the far-field scratch");
    std::lock_guard<std::mutex> lock(g_ff_mutex);
    if (!g_ff_ptr[dev]) {
        void *p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(lbm_ff_scratch)), "hipGetSymbolAddress(far-field scratch)");
        if (!p) fail(LBM_EM_EDEVICE, "far-field scratch has no device address");
        g_ff_ptr[dev] = (double *)p;
    }
    return g_ff_ptr[dev];
}

// degrees -> radians in place (theta at ang[0..n), phi at ang[max..max+n);
// without phi the second half is set to zero)
__global__ void k_ff_angles(double *ang, int n, int has_phi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ang[i] = ang[i] * M_PI / 180.0;
    ang[kFfMaxAngles + i] = has_phi ? ang[kFfMaxAngles + i] * M_PI / 180.0 : 0.0;
}

// the incident line's phasors at every contour node (and the probe, last)
__global__ void k_ff_line_nodes(const double *line_acc, double *out, Box b, int dim, int axis, int probe_u,
                                int64_t nnodes) {
    const int64_t nbx = b.hi[0] - b.lo[0] + 1, nby = b.hi[1] - b.lo[1] + 1, nbz = b.hi[2] - b.lo[2] + 1;
    const int64_t cells = nbx * nby * nbz;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c <= cells; c += (int64_t)gridDim.x * blockDim.x) {
        if (c == cells) {
            for (int k = 0; k < 12; ++k) out[nnodes * 12 + k] = line_acc[(int64_t)probe_u * 12 + k];
            continue;
        }
        const int x = b.lo[0] + (int)(c % nbx), y = b.lo[1] + (int)((c / nbx) % nby), z = b.lo[2] + (int)(c / (nbx * nby));
        if (!on_box(b, dim, x, y, z)) continue;
        const int64_t node = box_node_index(b, dim, x, y, z);
        const int u = axis == 0 ? x : axis == 1 ? y : z;
        for (int k = 0; k < 12; ++k) out[node * 12 + k] = line_acc[(int64_t)u * 12 + k];
    }
}

// |S|^2 = kappa |P|^2 / amp^2, amp = |u . v| of the incident probe phasor v
// (the source amplitude without an incident field)
__global__ void k_ff_finish(const double *P, const double *probe, double u0, double u1, double u2, double amplitude,
                            double kappa, int n, double *S2, double *amp_out) {
    double amp = amplitude;
    if (probe) {
        const double u[3] = {u0, u1, u2};
        double re = 0, im = 0;
        for (int k = 0; k < 3; ++k) {
            re += u[k] * probe[2 * k];
            im += u[k] * probe[2 * k + 1];
        }
        amp = sqrt(re * re + im * im);
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *amp_out = amp;
    if (i >= n) return;
    const double *q = P + 4 * (size_t)i;
    const double p = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    S2[i] = kappa * p / (amp * amp);
}

}  // namespace

namespace {

// Multi-plane streaming (measured ceiling of the step kernels' access
// pattern): every thread reads cell c of nin planes and writes cell c of
// nout planes (streamed stores, as the 3-D two-step kernel), plane stride P.
__global__ void __launch_bounds__(256) k_stream_planes(const float *__restrict__ in, float *__restrict__ out,
                                                               int64_t P, int64_t n, int nin, int nout) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    float v[32];
    // every load is issued before any of them is used
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = i < nin ? in[i * P + c] : 0.f;
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < 32; ++i) acc += v[i];
#pragma unroll
    for (int i = 0; i < 32; ++i)
        if (i < nout) __builtin_nontemporal_store(fmaf(v[i], 0.5f, acc), out + i * P + c);
}

}  // namespace

extern "C" {

const char *lbm_em_last_error(void) { return g_last_error.c_str(); }

lbm_em_status lbm_em_create(const lbm_em_config *cfg, lbm_em_handle *out) {
    return guarded([&] {
        if (!cfg || !out) fail(LBM_EM_EINVAL, "null config or output pointer");
        const lbm_em_config &c = *cfg;
        if (c.nx < 1 || c.ny < 1 || c.nz < 1) fail(LBM_EM_EINVAL, "grid sizes must be >= 1");
        if ((int64_t)c.nx * c.ny * c.nz > (int64_t)1 << 31)
            fail(LBM_EM_EINVAL, "more than 2^31 cells");
        {   // kernels address a population plane with 32-bit byte offsets
            const int64_t esz = c.precision == LBM_EM_FP64 ? 8 : 4;
            if (round_up(c.nx, 64) * c.ny * c.nz * esz >= (int64_t)1 << 32)
                fail(LBM_EM_EINVAL, "grid too large: one population plane (x padded to 64) must stay below 4 GiB");
        }
        if (c.pol != LBM_EM_TM && c.pol != LBM_EM_TE && c.pol != LBM_EM_3D)
            fail(LBM_EM_EINVAL, "pol must be LBM_EM_TM, LBM_EM_TE or LBM_EM_3D");
        if (c.pol != LBM_EM_3D && c.nz != 1) fail(LBM_EM_EINVAL, "TM/TE runs need nz == 1");
        if (c.pol == LBM_EM_3D && c.nz < 3) fail(LBM_EM_EINVAL, "3-D runs need nz >= 3");
        if (c.precision != LBM_EM_FP32 && c.precision != LBM_EM_FP64)
            fail(LBM_EM_EINVAL, "precision must be LBM_EM_FP32 or LBM_EM_FP64");
        const int n[3] = {c.nx, c.ny, c.nz};
        for (int a = 0; a < 3; ++a) {
            if (c.absorb[a] < 0 || 2 * c.absorb[a] > n[a] || (c.absorb[a] > 0 && n[a] < 2))
                fail(LBM_EM_EINVAL, "absorbing width must satisfy 0 <= 2W <= n (and n >= 2 when W > 0)");
            if (c.pol != LBM_EM_3D && a == 2 && c.absorb[a] != 0)
                fail(LBM_EM_EINVAL, "2-D runs are periodic in z (absorb[2] = 0)");
        }
        if (!(c.sigma_max >= 0.0 && c.sigma_max <= 1.0)) fail(LBM_EM_EINVAL, "sigma_max must be in [0, 1]");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(LBM_EM_EDEVICE, "no HIP device");

        lbm_em *h = new lbm_em();
        try {
            h->cfg = c;
            hip_check(hipGetDevice(&h->dev), "hipGetDevice");
            h->dim = c.pol == LBM_EM_3D ? 3 : 2;
            h->nplanes = c.pol == LBM_EM_3D ? 27 : 11;
            h->elem = c.precision == LBM_EM_FP32 ? 4 : 8;
            hip_check(hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->dev), "attribute");
            h->cus = std::max(1, h->cus);
            if (h->dim == 2) {
                h->fuse = 2;
                // 1024-thread tiles: the smallest re-read halo (autotune may
                // pick another)
                h->ftx = c.precision == LBM_EM_FP32 ? 256 : 128;
                h->fty = 16;
            } else {
                h->fuse = 2;      // z march, one-plane lag (k_step3d_x2)
                // wide tiles: fewer 128-byte lines spent on the ring columns
                h->ftx = 128;
                h->fty = c.precision == LBM_EM_FP32 ? 8 : 4;
            }
            h->sy = round_up(c.nx, 64);
            h->sz = h->sy * c.ny;
            h->plane = plane_stride(h->sz * c.nz, h->elem);
            h->stream = (hipStream_t)c.stream;
            const size_t bytes = (size_t)h->plane * h->nplanes * h->elem;
            hip_check(hipMalloc(&h->buf[0], bytes), "hipMalloc state");
            hip_check(hipMalloc(&h->buf[1], bytes), "hipMalloc state");
            hip_check(hipMalloc(&h->eps, (size_t)h->plane * h->elem), "hipMalloc eps");
            hip_check(hipMalloc(&h->t_dev, 64), "hipMalloc counter");
            hip_check(hipMemsetAsync(h->buf[0], 0, bytes, h->stream), "hipMemset");
            hip_check(hipMemsetAsync(h->buf[1], 0, bytes, h->stream), "hipMemset");
            fill_ones(h, h->eps);   // eps_r = 1 everywhere (padding included)
            if (h->dim == 3) {
                h->eps_box.assign(c.nz, make_int4(c.nx, -1, c.ny, -1));
                h->run_box = h->eps_box;
                hip_check(hipMalloc(&h->vbox, (size_t)c.nz * sizeof(int4)), "hipMalloc vacuum boxes");
                upload_vbox(h);
            }
            hip_check(hipStreamSynchronize(h->stream), "sync");
        } catch (...) {
            free_handle(h);
            throw;
        }
        *out = h;
    });
}

lbm_em_status lbm_em_destroy(lbm_em_handle h) {
    return guarded([&] {
        check_handle(h);
        if (h->batch_refs) fail(LBM_EM_ESTATE, "handle is part of a batch; destroy the batch first");
        free_handle(h);
    });
}

lbm_em_status lbm_em_set_permittivity(lbm_em_handle hh, const void *eps, int32_t where, int32_t dtype) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!eps) fail(LBM_EM_EINVAL, "null eps");
        std::vector<int4> boxes;
        load_material(h, eps, where, dtype, h->eps, "eps_r", h->vbox ? &boxes : nullptr);
        if (h->vbox) {
            // after steps, cells that were not vacuum may keep rest populations
            std::vector<int4> run = boxes;
            if (!h->state_clean)
                for (size_t z = 0; z < run.size(); ++z) {
                    const int4 o = h->run_box[z];
                    int4 &b = run[z];
                    if (o.x > o.y) continue;
                    if (b.x > b.y) { b = o; continue; }
                    b = make_int4(std::min(b.x, o.x), std::max(b.y, o.y), std::min(b.z, o.z), std::max(b.w, o.w));
                }
            h->eps_box = std::move(boxes);
            h->run_box = std::move(run);
            upload_vbox(h);
        }
    });
}

lbm_em_status lbm_em_set_permeability(lbm_em_handle hh, const void *mu, int32_t where, int32_t dtype) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (h->dim != 2) fail(LBM_EM_EUNSUPPORTED, "a permeability map needs a 2-D (TM/TE) handle");
        if (h->batch_refs) fail(LBM_EM_ESTATE, "handle is part of a batch; destroy the batch first");
        if (h->adj_set) fail(LBM_EM_EUNSUPPORTED, "the adjoint needs mu_r = 1");
        select_device(h);
        if (!mu) {   // back to mu_r = 1 (conductor cells stay)
            sync(h);
            if (h->pec) {
                fill_ones(h, h->mu);
                mask_fill(h, 0.0);
                sync(h);
            } else {
                hfree(h->mu);
                h->mu = nullptr;
            }
            h->mu_user = false;
            drop_graphs(h);
            return;
        }
        void *dst = h->mu;
        if (!dst) {
            hip_check(hipMalloc(&dst, (size_t)h->plane * h->elem), "hipMalloc mu");
            fill_ones(h, dst);
        }
        try {
            load_material(h, mu, where, dtype, dst, "mu_r");
        } catch (...) {
            if (dst != h->mu) hfree(dst);
            throw;
        }
        h->mu = dst;
        h->mu_user = true;
        mask_fill(h, 0.0);
        sync(h);
        drop_graphs(h);
    });
}

lbm_em_status lbm_em_set_pec(lbm_em_handle hh, const uint8_t *mask, int32_t where) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (h->cfg.pol != LBM_EM_TM)
            fail(LBM_EM_EUNSUPPORTED, "perfect-conductor cells are supported for TM handles (E along the axis)");
        if (h->batch_refs) fail(LBM_EM_ESTATE, "handle is part of a batch; destroy the batch first");
        if (h->adj_set) fail(LBM_EM_EUNSUPPORTED, "the adjoint does not cover perfect conductors");
        if (where != LBM_EM_HOST && where != LBM_EM_DEVICE) fail(LBM_EM_EINVAL, "where must be HOST or DEVICE");
        select_device(h);
        const size_t cells = (size_t)h->cfg.nx * h->cfg.ny * h->cfg.nz;
        // release the previous mask: its cells return to mu_r = 1
        mask_fill(h, 1.0);
        sync(h);
        hfree(h->pec);
        h->pec = nullptr;
        if (!mask) {
            if (!h->mu_user) {
                hfree(h->mu);
                h->mu = nullptr;
            }
            drop_graphs(h);
            return;
        }
        unsigned char *d = nullptr;
        hip_check(hipMalloc(&d, cells), "hipMalloc pec");
        try {
            hip_check(hipMemcpyAsync(d, mask, cells, where == LBM_EM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                     h->stream), "pec copy");
            if (!h->mu) {
                void *m = nullptr;
                hip_check(hipMalloc(&m, (size_t)h->plane * h->elem), "hipMalloc mu");
                h->mu = m;
                fill_ones(h, h->mu);
            }
        } catch (...) {
            sync(h);
            hfree(d);
            throw;
        }
        h->pec = d;
        mask_fill(h, 0.0);
        sync(h);
        drop_graphs(h);
    });
}

lbm_em_status lbm_em_set_incident_line(lbm_em_handle hh, int32_t enable) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (h->batch_refs) fail(LBM_EM_ESTATE, "handle is part of a batch; destroy the batch first");
        if (h->adj_set) fail(LBM_EM_EUNSUPPORTED, "the adjoint uses the companion run, not an incident line");
        select_device(h);
        sync(h);
        drop_line(h);
        drop_graphs(h);
        if (!enable) return;
        if (!h->src_on) fail(LBM_EM_ESTATE, "set the source first");
        if (h->t != 0) fail(LBM_EM_ESTATE, "set the incident line before stepping (or after a reset)");
        const double *k = h->pw.khat;
        int axis = -1;
        for (int ax = 0; ax < 3; ++ax)
            if (std::fabs(std::fabs(k[ax]) - 1.0) <= 1e-12 && std::fabs(k[(ax + 1) % 3]) <= 1e-12 &&
                std::fabs(k[(ax + 2) % 3]) <= 1e-12)
                axis = ax;
        if (h->dim == 2 && axis != 0 && axis != 1)
            fail(LBM_EM_EINVAL, "the incident line needs incidence along +-x or +-y");
        if (h->dim == 3 && axis != 2) fail(LBM_EM_EINVAL, "a 3-D incident line needs incidence along +-z");
        h->line_axis = axis;
        lbm_em_config lc = h->cfg;
        const int n3[3] = {h->cfg.nx, h->cfg.ny, h->cfg.nz};
        lc.nx = axis == 0 ? n3[0] : 1;
        lc.ny = axis == 1 ? n3[1] : 1;
        lc.nz = axis == 2 ? n3[2] : 1;
        for (int ax = 0; ax < 3; ++ax) lc.absorb[ax] = ax == axis ? h->cfg.absorb[ax] : 0;
        lc.stream = (void *)h->stream;
        lbm_em *l = nullptr;
        lbm_em_status st = lbm_em_create(&lc, &l);
        if (st != LBM_EM_OK) fail(st, std::string("incident line: ") + g_last_error);
        h->line = l;
        h->line_axis = axis;
        st = lbm_em_set_source(l, &h->pw);
        if (st != LBM_EM_OK) {
            const std::string msg = g_last_error;
            drop_line(h);
            fail(st, "incident line: " + msg);
        }
        try {
            const int64_t n = line_len(h);
            const size_t tab = (size_t)kLineSlots * h->nplanes * n * h->elem;
            hip_check(hipMalloc(&h->line_tmp, (size_t)l->plane * l->nplanes * l->elem), "hipMalloc line");
            hip_check(hipMalloc(&h->line_tab, tab), "hipMalloc line");
            hip_check(hipMalloc(&h->line_acc, (size_t)n * 12 * sizeof(double)), "hipMalloc line");
            hip_check(hipMemsetAsync(h->line_tab, 0, tab, h->stream), "hipMemset line");
            hip_check(hipMemsetAsync(h->line_acc, 0, (size_t)n * 12 * sizeof(double), h->stream), "hipMemset line");
            sync(h);
        } catch (...) {
            drop_line(h);
            throw;
        }
    });
}

lbm_em_status lbm_em_get_line_phasors(lbm_em_handle hh, double *out, int32_t *n) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!n) fail(LBM_EM_EINVAL, "null count");
        if (!h->line) fail(LBM_EM_ESTATE, "no incident line");
        *n = line_len(h);
        if (!out) return;
        select_device(h);
        hip_check(hipMemcpyAsync(out, h->line_acc, (size_t)*n * 12 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                  "D2H");
        sync(h);
    });
}

lbm_em_status lbm_em_set_source(lbm_em_handle hh, const lbm_em_plane_wave *pw) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!pw) fail(LBM_EM_EINVAL, "null plane wave");
        check_unit(pw->khat, "khat");
        check_unit(pw->ehat, "ehat");
        double kd = pw->khat[0] * pw->ehat[0] + pw->khat[1] * pw->ehat[1] + pw->khat[2] * pw->ehat[2];
        if (std::fabs(kd) > 1e-9) fail(LBM_EM_EINVAL, "ehat must be perpendicular to khat");
        if (!(pw->lambda > 2.0) || !std::isfinite(pw->lambda)) fail(LBM_EM_EINVAL, "lambda must be > 2 cells");
        double T = 3.0 * pw->lambda;
        if (std::fabs(T - std::round(T)) > 1e-9) fail(LBM_EM_EINVAL, "3*lambda must be an integer");
        if (!(pw->ramp_periods >= 0.0) || !std::isfinite(pw->amplitude)) fail(LBM_EM_EINVAL, "bad ramp / amplitude");
        if (h->cfg.pol != LBM_EM_3D) {
            if (std::fabs(pw->khat[2]) > 1e-12) fail(LBM_EM_EINVAL, "2-D runs need khat in the xy plane");
            if (h->cfg.pol == LBM_EM_TM && std::fabs(std::fabs(pw->ehat[2]) - 1.0) > 1e-12)
                fail(LBM_EM_EINVAL, "TM needs ehat = +-z");
            if (h->cfg.pol == LBM_EM_TE && std::fabs(pw->ehat[2]) > 1e-12)
                fail(LBM_EM_EINVAL, "TE needs ehat in the xy plane");
        }
        const double t_ramp = pw->ramp_periods * T;
        if (t_ramp > 1e7) fail(LBM_EM_EINVAL, "ramp longer than 1e7 steps");
        if (h->batch_refs) fail(LBM_EM_ESTATE, "handle is part of a batch; destroy the batch first");
        select_device(h);
        sync(h);
        drop_line(h);       // a new source ends the incident line (set it again)
        // Tables, in one allocation: (cos, sin)(2 pi k / T) for k < T (FP64);
        // the ramp g(t) = sin^2(pi t / (2 t_ramp)) for t < t_ramp (FP64);
        // (cos, sin)(2 pi u_a) per column, row and slab, u_a = khat_a (a -
        // center_a) / lambda reduced to [0, 1) before the sine, computed in
        // FP64 and stored in the run's precision.
        const int period = (int)std::lround(T);
        const int nramp = (int)std::ceil(t_ramp);
        const int n[3] = {h->cfg.nx, h->cfg.ny, h->cfg.nz};
        std::vector<double> head, axes;
        auto unit = [](std::vector<double> &v, double u) {
            u -= std::floor(u);
            v.push_back(std::cos(2.0 * M_PI * u));
            v.push_back(std::sin(2.0 * M_PI * u));
        };
        for (int k = 0; k < period; ++k) unit(head, (double)k / (double)period);
        for (int i = 0; i < nramp; ++i) {
            const double sr = std::sin(M_PI * (double)i / (2.0 * t_ramp));
            head.push_back(sr * sr);
        }
        if (head.size() % 2) head.push_back(0.0);     // 16-byte aligned axis tables
        for (int ax = 0; ax < 3; ++ax)
            for (int i = 0; i < n[ax]; ++i) unit(axes, pw->khat[ax] * ((double)i - pw->center[ax]) / pw->lambda);
        std::vector<char> bytes(head.size() * 8 + axes.size() * h->elem);
        std::memcpy(bytes.data(), head.data(), head.size() * 8);
        char *ap = bytes.data() + head.size() * 8;
        for (size_t i = 0; i < axes.size(); ++i) {
            if (h->elem == 8) std::memcpy(ap + 8 * i, &axes[i], 8);
            else {
                const float v = (float)axes[i];
                std::memcpy(ap + 4 * i, &v, 4);
            }
        }
        double *dtab = nullptr;
        hip_check(hipMalloc(&dtab, bytes.size()), "hipMalloc source tables");
        hipError_t e = hipMemcpyAsync(dtab, bytes.data(), bytes.size(), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            hfree(dtab);
            hip_check(e, "H2D source tables");
        }
        sync(h);            // no launch in flight still reads the old tables
        hfree(h->wtab);
        h->wtab = dtab;
        h->pw = *pw;
        const double *k = pw->khat, *ev = pw->ehat;
        h->hhat[0] = k[1] * ev[2] - k[2] * ev[1];
        h->hhat[1] = k[2] * ev[0] - k[0] * ev[2];
        h->hhat[2] = k[0] * ev[1] - k[1] * ev[0];
        h->period = period;
        h->axes_off = (int64_t)head.size();
        h->src_on = true;
        drop_graphs(h);
    });
}

lbm_em_status lbm_em_set_ntff(lbm_em_handle hh, const int32_t lo[3], const int32_t hi[3],
                              int64_t window_start, int64_t window_len) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!lo || !hi) fail(LBM_EM_EINVAL, "null box");
        if (!h->src_on) fail(LBM_EM_ESTATE, "set the source before the contour (the DFT frequency is the source's)");
        if (h->batch_refs) fail(LBM_EM_ESTATE, "handle is part of a batch; destroy the batch first");
        const int n[3] = {h->cfg.nx, h->cfg.ny, h->cfg.nz};
        for (int a = 0; a < h->dim; ++a)
            if (lo[a] < 1 || hi[a] > n[a] - 2 || hi[a] - lo[a] < 2)
                fail(LBM_EM_EINVAL, "contour box must lie strictly inside the grid and span >= 3 nodes");
        if (h->dim == 2 && (lo[2] != 0 || hi[2] != 0)) fail(LBM_EM_EINVAL, "2-D box needs lo[2] = hi[2] = 0");
        if (window_start < 0 || window_len < 1) fail(LBM_EM_EINVAL, "empty DFT window");
        select_device(h);
        for (int a = 0; a < 3; ++a) {
            h->box.lo[a] = lo[a];
            h->box.hi[a] = hi[a];
            h->probe[a] = (lo[a] + hi[a]) / 2;
        }
        h->nnodes = box_nodes(h->box, h->dim);
        h->win0 = window_start;
        h->winlen = window_len;
        hfree(h->acc);
        h->acc = nullptr;
        const size_t bytes = (size_t)(h->nnodes + 1) * 12 * sizeof(double);
        hip_check(hipMalloc(&h->acc, bytes), "hipMalloc dft");
        hip_check(hipMemsetAsync(h->acc, 0, bytes, h->stream), "hipMemset dft");
        if (h->line) {
            const int64_t n = line_len(h);
            hip_check(hipMemsetAsync(h->line_acc, 0, (size_t)n * 12 * sizeof(double), h->stream), "hipMemset line dft");
        }
        h->dft_set = true;
        drop_graphs(h);
    });
}

lbm_em_status lbm_em_step(lbm_em_handle hh, int64_t n) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (n < 0) fail(LBM_EM_EINVAL, "n must be >= 0");
        do_steps(h, n);
    });
}

lbm_em_status lbm_em_step_many(const lbm_em_handle *hs, int32_t count, int64_t n) {
    return guarded([&] {
        if (n < 0) fail(LBM_EM_EINVAL, "n must be >= 0");
        lbm_em_batch_s *b = make_batch(hs, count);
        try {
            batch_steps(b, n, false);
        } catch (...) {
            free_batch(b);
            throw;
        }
        free_batch(b);
    });
}

lbm_em_status lbm_em_batch_create(const lbm_em_handle *hs, int32_t count, lbm_em_batch *out) {
    return guarded([&] {
        if (!out) fail(LBM_EM_EINVAL, "null output");
        *out = make_batch(hs, count);
    });
}

lbm_em_status lbm_em_batch_step(lbm_em_batch b, int64_t n) {
    return guarded([&] {
        if (!b) fail(LBM_EM_EINVAL, "null batch");
        if (n < 0) fail(LBM_EM_EINVAL, "n must be >= 0");
        batch_steps(b, n, true);
    });
}

lbm_em_status lbm_em_batch_set_grid(lbm_em_batch b, int32_t grid) {
    return guarded([&] {
        if (!b) fail(LBM_EM_EINVAL, "null batch");
        if (grid < 1) fail(LBM_EM_EINVAL, "grid must be >= 1");
        b->grid_override = grid;
        plan_batch(b);
    });
}

lbm_em_status lbm_em_batch_set_cache_budget(lbm_em_batch b, int64_t bytes) {
    return guarded([&] {
        if (!b) fail(LBM_EM_EINVAL, "null batch");
        if (bytes < 0) fail(LBM_EM_EINVAL, "budget must be >= 0");
        b->budget = bytes;
        plan_batch(b);
    });
}

lbm_em_status lbm_em_batch_autotune(lbm_em_batch b, int32_t launches, double *best_us) {
    return guarded([&] {
        if (!b) fail(LBM_EM_EINVAL, "null batch");
        if (launches < 1) fail(LBM_EM_EINVAL, "launches must be >= 1");
        lbm_em *h0 = b->hs[0];
        for (auto *h : b->hs)
            if (h->t != h0->t || h->cur != h0->cur)
                fail(LBM_EM_ESTATE, "batched handles were stepped separately since the batch was made");
        (void)hipSetDevice(b->dev);
        std::vector<std::pair<int, int>> cands;
        if (b->fuse == 2) {
#define LBM_X2_BCAND(TX, TY) cands.push_back({TX, TY});
            if (b->precision == LBM_EM_FP32) { LBM_X2_TILES_F32(LBM_X2_BCAND) }
            else { LBM_X2_TILES_F64(LBM_X2_BCAND) }
#undef LBM_X2_BCAND
        }
        bool timed = false;
        for (const auto &g : b->groups) timed = timed || !g.direct;
        const int keep_tx = b->ftx, keep_ty = b->fty;
        double best = 0.0;
        if (!cands.empty() && timed) {
            hipEvent_t e0, e1;
            hip_check(hipEventCreate(&e0), "hipEventCreate");
            hip_check(hipEventCreate(&e1), "hipEventCreate");
            int btx = keep_tx, bty = keep_ty;
            best = 1e30;
            try {
                for (const auto &c : cands) {
                    b->ftx = c.first;
                    b->fty = c.second;
                    plan_batch(b, false);
                    // timed launches read the current buffers and write the
                    // spare ones with the DFT off: no state changes
                    auto run = [&](int reps) {
                        for (const auto &g : b->groups)
                            if (!g.direct)
                                for (int i = 0; i < reps; ++i)
                                    launch_batch(b, g, h0->cur, nullptr, h0->t, b->stream, 2, false);
                    };
                    run(1);
                    hip_check(hipEventRecord(e0, b->stream), "hipEventRecord");
                    run(launches);
                    hip_check(hipEventRecord(e1, b->stream), "hipEventRecord");
                    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
                    float ms = 0.f;
                    hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                    const double us = 1e3 * (double)ms / launches / 2;   // per step, all batched instances
                    if (us < best) {
                        best = us;
                        btx = c.first;
                        bty = c.second;
                    }
                }
            } catch (...) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                b->ftx = keep_tx;
                b->fty = keep_ty;
                plan_batch(b);
                throw;
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            b->ftx = btx;
            b->fty = bty;
        }
        plan_batch(b);
        if (best_us) *best_us = best;
    });
}

lbm_em_status lbm_em_batch_groups(lbm_em_batch b, int32_t *groups) {
    return guarded([&] {
        if (!b || !groups) fail(LBM_EM_EINVAL, "null argument");
        *groups = (int32_t)b->groups.size();
    });
}

lbm_em_status lbm_em_batch_get_tile(lbm_em_batch b, int32_t *steps_per_launch, int32_t *tile_x, int32_t *tile_y) {
    return guarded([&] {
        if (!b || !steps_per_launch || !tile_x || !tile_y) fail(LBM_EM_EINVAL, "null argument");
        *steps_per_launch = b->fuse;
        *tile_x = b->ftx;
        *tile_y = b->fty;
    });
}

lbm_em_status lbm_em_batch_destroy(lbm_em_batch b) {
    return guarded([&] {
        if (!b) fail(LBM_EM_EINVAL, "null batch");
        free_batch(b);
    });
}

lbm_em_status lbm_em_set_tile(lbm_em_handle hh, int32_t vx, int32_t bx, int32_t by) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!tile_ok(h, vx, bx, by))
            fail(LBM_EM_EINVAL, "tile: vx in {1,2} (FP64) or {1,2,4} (FP32), 64 <= bx*by <= 256, bx*by % 64 == 0");
        h->vx = vx;
        h->bx = bx;
        h->by = by;
        drop_graphs(h);
    });
}

lbm_em_status lbm_em_set_fusion(lbm_em_handle hh, int32_t steps_per_launch, int32_t tile_x, int32_t tile_y) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (steps_per_launch != 1 && steps_per_launch != 2) fail(LBM_EM_EINVAL, "steps_per_launch must be 1 or 2");
        if (steps_per_launch == 2 && (tile_x || tile_y)) {
            if (!fused_tile_ok(h->dim, h->cfg.precision, tile_x, tile_y))
                fail(LBM_EM_EINVAL,
                     h->dim == 3 ? (h->cfg.precision == LBM_EM_FP32 ? "3-D FP32 two-step tile must be 64x16, 64x8, 32x16, 128x8, 256x4 or 128x4"
                                                                    : "3-D FP64 two-step tile must be 32x16, 32x8, 16x16, 64x8 or 128x4")
                     : h->cfg.precision == LBM_EM_FP32
                         ? "FP32 two-step tile must be 64x16, 128x8, 128x16, 256x8, 256x16 or 128x32"
                         : "FP64 two-step tile must be 32x16, 64x8, 64x16, 128x8, 128x16 or 64x32");
            h->ftx = tile_x;
            h->fty = tile_y;
        }
        h->fuse = steps_per_launch;
        drop_graphs(h);
    });
}

lbm_em_status lbm_em_get_fusion(lbm_em_handle hh, int32_t *steps_per_launch, int32_t *tile_x, int32_t *tile_y) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!steps_per_launch) fail(LBM_EM_EINVAL, "null output");
        *steps_per_launch = h->fuse;
        if (tile_x) *tile_x = h->ftx;
        if (tile_y) *tile_y = h->fty;
    });
}

lbm_em_status lbm_em_get_tile(lbm_em_handle hh, int32_t *vx, int32_t *bx, int32_t *by) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!vx || !bx || !by) fail(LBM_EM_EINVAL, "null output");
        *vx = h->vx;
        *bx = h->bx;
        *by = h->by;
    });
}

lbm_em_status lbm_em_autotune(lbm_em_handle hh, int32_t launches, double *best_us) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (launches < 1) fail(LBM_EM_EINVAL, "launches must be >= 1");
        select_device(h);
        struct Cand { int fuse, a, b, c; };   // fuse 1: (vx, bx, by); fuse 2: (tx, ty)
        std::vector<Cand> cands;
        static const int shapes[][2] = {{64, 4}, {128, 2}, {256, 1}, {32, 8}, {64, 2}, {128, 1}, {64, 1}, {16, 16}};
        for (int vx : {1, 2, 4})
            for (auto &sh : shapes)
                if (tile_ok(h, vx, sh[0], sh[1])) cands.push_back({1, vx, sh[0], sh[1]});
#define LBM_X2_CAND(TX, TY) cands.push_back({2, TX, TY, 0});
        if (h->dim == 2) {
            if (h->cfg.precision == LBM_EM_FP32) { LBM_X2_TILES_F32(LBM_X2_CAND) }
            else { LBM_X2_TILES_F64(LBM_X2_CAND) }
        } else {
            if (h->cfg.precision == LBM_EM_FP32) { LBM_X3_TILES_F32(LBM_X2_CAND) }
            else { LBM_X3_TILES_F64(LBM_X2_CAND) }
        }
#undef LBM_X2_CAND
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        hip_check(hipEventCreate(&e1), "hipEventCreate");
        const lbm_em keep = *h;
        auto apply = [&](const Cand &c) {
            h->fuse = c.fuse;
            if (c.fuse == 1) { h->vx = c.a; h->bx = c.b; h->by = c.c; }
            else { h->ftx = c.a; h->fty = c.b; }
        };
        // Timed launches read the current buffer and write the spare one with
        // the DFT off: the simulation state is not changed.
        auto launch = [&]() {
            if (h->fuse == 2) launch_step2(h, h->cur, nullptr, h->t, h->stream, false);
            else launch_step(h, h->cur, nullptr, h->t, h->stream, false);
        };
        Cand best = cands[0];
        double best_per_step = 1e30;
        for (const Cand &c : cands) {
            apply(c);
            launch();
            hip_check(hipEventRecord(e0, h->stream), "hipEventRecord");
            for (int i = 0; i < launches; ++i) launch();
            hip_check(hipEventRecord(e1, h->stream), "hipEventRecord");
            hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            const double per_step = (double)ms / launches / c.fuse;
            if (per_step < best_per_step) {
                best_per_step = per_step;
                best = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        // The winner must reproduce one-cell-per-thread single steps bit for
        // bit (after one launch: one step, or two for the fused kernel).
        const size_t n = (size_t)h->plane * h->nplanes;
        void *ref = nullptr;
        int *flag = nullptr;
        try {
            hip_check(hipMalloc(&ref, n * h->elem), "hipMalloc");
            hip_check(hipMalloc(&flag, sizeof(int)), "hipMalloc");
            hip_check(hipMemsetAsync(flag, 0, sizeof(int), h->stream), "hipMemset");
            h->fuse = 1; h->vx = 1; h->bx = 64; h->by = 4;
            if (best.fuse == 1) {
                launch_step(h, h->cur, nullptr, h->t, h->stream, false);
                hip_check(hipMemcpyAsync(ref, h->buf[h->cur ^ 1], n * h->elem, hipMemcpyDeviceToDevice, h->stream), "copy");
            } else if (h->elem == 4) {
                launch_step_t<float>(h, h->buf[h->cur], h->buf[h->cur ^ 1], nullptr, h->t, h->stream, false, nullptr, 0);
                launch_step_t<float>(h, h->buf[h->cur ^ 1], ref, nullptr, h->t + 1, h->stream, false, nullptr, 0);
            } else {
                launch_step_t<double>(h, h->buf[h->cur], h->buf[h->cur ^ 1], nullptr, h->t, h->stream, false, nullptr, 0);
                launch_step_t<double>(h, h->buf[h->cur ^ 1], ref, nullptr, h->t + 1, h->stream, false, nullptr, 0);
            }
            apply(best);
            launch();
            const unsigned blocks = (unsigned)((n + 255) / 256);
            if (h->elem == 4)
                hipLaunchKernelGGL((k_compare<float>), dim3(blocks), dim3(256), 0, h->stream, (const float *)ref,
                                   (const float *)h->buf[h->cur ^ 1], (int64_t)n, h->plane, h->sz * h->cfg.nz, flag);
            else
                hipLaunchKernelGGL((k_compare<double>), dim3(blocks), dim3(256), 0, h->stream, (const double *)ref,
                                   (const double *)h->buf[h->cur ^ 1], (int64_t)n, h->plane, h->sz * h->cfg.nz, flag);
            int differs = 0;
            hip_check(hipMemcpyAsync(&differs, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream), "D2H");
            sync(h);
            hfree(ref);
            hfree(flag);
            ref = nullptr;
            flag = nullptr;
            if (differs) fail(LBM_EM_EDEVICE, "autotune: tuned kernel differs from the reference kernel");
        } catch (...) {
            hfree(ref);
            hfree(flag);
            h->fuse = keep.fuse; h->vx = keep.vx; h->bx = keep.bx; h->by = keep.by;
            h->ftx = keep.ftx; h->fty = keep.fty;
            throw;
        }
        // the shape family that did not win keeps its previous setting
        if (best.fuse == 2) { h->vx = keep.vx; h->bx = keep.bx; h->by = keep.by; }
        else { h->ftx = keep.ftx; h->fty = keep.fty; }
        drop_graphs(h);
        if (best_us) *best_us = 1e3 * best_per_step;
    });
}

lbm_em_status lbm_em_reset(lbm_em_handle hh) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        select_device(h);
        reset_state(h);
    });
}

lbm_em_status lbm_em_time(lbm_em_handle hh, int64_t *t) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!t) fail(LBM_EM_EINVAL, "null output");
        *t = h->t;
    });
}

lbm_em_status lbm_em_get_fields(lbm_em_handle hh, void *E, void *H, int32_t where) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!E || !H) fail(LBM_EM_EINVAL, "null output");
        if (where != LBM_EM_HOST && where != LBM_EM_DEVICE) fail(LBM_EM_EINVAL, "where must be HOST or DEVICE");
        select_device(h);
        const auto &c = h->cfg;
        const size_t bytes = (size_t)c.nx * c.ny * c.nz * 3 * h->elem;
        void *dE = E, *dH = H;
        if (where == LBM_EM_HOST) {
            hip_check(hipMalloc(&dE, bytes), "hipMalloc");
            hip_check(hipMalloc(&dH, bytes), "hipMalloc");
        }
        dim3 block(h->bx, h->by, 1);
        dim3 grid((c.nx + h->bx - 1) / h->bx, (c.ny + h->by - 1) / h->by, c.nz);
        if (h->elem == 4) {
            auto a = make_args<float>(h, h->buf[h->cur], nullptr);
            if (c.pol == LBM_EM_TM) hipLaunchKernelGGL((k_fields<float, TM>), grid, block, 0, h->stream, a, (float *)dE, (float *)dH);
            else if (c.pol == LBM_EM_TE) hipLaunchKernelGGL((k_fields<float, TE>), grid, block, 0, h->stream, a, (float *)dE, (float *)dH);
            else hipLaunchKernelGGL((k_fields<float, D3>), grid, block, 0, h->stream, a, (float *)dE, (float *)dH);
        } else {
            auto a = make_args<double>(h, h->buf[h->cur], nullptr);
            if (c.pol == LBM_EM_TM) hipLaunchKernelGGL((k_fields<double, TM>), grid, block, 0, h->stream, a, (double *)dE, (double *)dH);
            else if (c.pol == LBM_EM_TE) hipLaunchKernelGGL((k_fields<double, TE>), grid, block, 0, h->stream, a, (double *)dE, (double *)dH);
            else hipLaunchKernelGGL((k_fields<double, D3>), grid, block, 0, h->stream, a, (double *)dE, (double *)dH);
        }
        hip_check(hipGetLastError(), "k_fields");
        if (where == LBM_EM_HOST) {
            hip_check(hipMemcpyAsync(E, dE, bytes, hipMemcpyDeviceToHost, h->stream), "D2H");
            hip_check(hipMemcpyAsync(H, dH, bytes, hipMemcpyDeviceToHost, h->stream), "D2H");
            sync(h);
            hfree(dE);
            hfree(dH);
        }
    });
}

lbm_em_status lbm_em_get_phasors(lbm_em_handle hh, double *out, int32_t *n_nodes) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!n_nodes) fail(LBM_EM_EINVAL, "null n_nodes");
        if (!h->dft_set) fail(LBM_EM_ESTATE, "no contour set");
        *n_nodes = (int32_t)h->nnodes;
        if (!out) return;
        select_device(h);
        std::vector<double> raw((size_t)(h->nnodes + 1) * 12);
        hip_check(hipMemcpyAsync(raw.data(), h->acc, raw.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 h->stream), "D2H");
        sync(h);
        // surface nodes in ascending linear index (z, y, x)
        const Box &b = h->box;
        int64_t k = 0;
        for (int z = b.lo[2]; z <= b.hi[2]; ++z)
            for (int y = b.lo[1]; y <= b.hi[1]; ++y)
                for (int x = b.lo[0]; x <= b.hi[0]; ++x) {
                    if (!on_box(b, h->dim, x, y, z)) continue;
                    int64_t node = box_node_index(b, h->dim, x, y, z);
                    std::memcpy(out + k * 12, raw.data() + node * 12, 12 * sizeof(double));
                    ++k;
                }
        std::memcpy(out + k * 12, raw.data() + h->nnodes * 12, 12 * sizeof(double));
    });
}

lbm_em_status lbm_em_farfield(lbm_em_handle hh, lbm_em_handle inc, const double *theta_deg,
                              const double *phi_deg, int32_t n_angles, double *out_S2) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!theta_deg || !out_S2 || n_angles < 1) fail(LBM_EM_EINVAL, "bad angle / output arrays");
        if (h->dim == 3 && !phi_deg) fail(LBM_EM_EINVAL, "3-D needs phi");
        if (!h->dft_set) fail(LBM_EM_ESTATE, "no contour set");
        if (h->t < h->win0 + h->winlen) fail(LBM_EM_ESTATE, "DFT window not completed");
        if (inc) check_incident(h, inc);
        select_device(h);
        if (inc) sync(inc);
        std::vector<double> th(n_angles), ph(n_angles);
        for (int i = 0; i < n_angles; ++i) {
            th[i] = theta_deg[i] * M_PI / 180.0;
            ph[i] = phi_deg ? phi_deg[i] * M_PI / 180.0 : 0.0;
        }
        double *d_out = nullptr, *d_line = nullptr;
        hip_check(hipMalloc(&d_out, (size_t)n_angles * 4 * sizeof(double)), "hipMalloc");
        const double *acc_inc = inc ? inc->acc : nullptr;
        if (!inc && h->line) {
            // the incident line's phasors at every contour node and the probe
            try {
                d_line = line_incident(h);
            } catch (...) {
                hfree(d_out);
                throw;
            }
            acc_inc = d_line;
        }
        const double amp = farfield_P(h, acc_inc, th.data(), ph.data(), n_angles, d_out);
        hfree(d_line);
        if (!(amp > 0.0)) {
            hfree(d_out);
            fail(LBM_EM_ESTATE, "incident amplitude at the probe node is zero (the wave has not arrived)");
        }
        std::vector<double> P((size_t)n_angles * 4);
        hip_check(hipMemcpyAsync(P.data(), d_out, P.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream), "D2H");
        sync(h);
        hfree(d_out);
        const double k = 2.0 * M_PI / h->pw.lambda;
        const double kappa = h->dim == 2 ? k * k / (8.0 * M_PI) : k * k * k * k / (16.0 * M_PI * M_PI);
        for (int i = 0; i < n_angles; ++i) {
            double p = P[4 * i] * P[4 * i] + P[4 * i + 1] * P[4 * i + 1] + P[4 * i + 2] * P[4 * i + 2] +
                       P[4 * i + 3] * P[4 * i + 3];
            out_S2[i] = kappa * p / (amp * amp);
        }
    });
}

lbm_em_status lbm_em_farfield_static(lbm_em_handle hh, lbm_em_handle inc, const double *theta_deg,
                                     const double *phi_deg, int32_t n_angles, double *out_S2) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!theta_deg || !out_S2 || n_angles < 1) fail(LBM_EM_EINVAL, "bad angle / output arrays");
        if (n_angles > kFfMaxAngles) fail(LBM_EM_EINVAL, "n_angles exceeds LBM_EM_FARFIELD_STATIC_MAX_ANGLES");
        if (h->dim == 3 && !phi_deg) fail(LBM_EM_EINVAL, "3-D needs phi");
        if (!h->dft_set) fail(LBM_EM_ESTATE, "no contour set");
        if (h->t < h->win0 + h->winlen) fail(LBM_EM_ESTATE, "DFT window not completed");
        if (inc) check_incident(h, inc);
        const bool use_line = !inc && h->line;
        if (use_line && h->nnodes > kFfMaxNodes) fail(LBM_EM_EINVAL, "contour exceeds LBM_EM_FARFIELD_STATIC_MAX_NODES");
        select_device(h);
        if (inc) sync(inc);
        double *sc = ff_scratch(h->dev);
        hipStream_t st = h->stream;
        double *ang = sc + kFfAng, *P = sc + kFfP, *S2 = sc + kFfS2, *amp_d = sc + kFfAmp, *line = sc + kFfLine;
        hip_check(hipMemcpyAsync(ang, theta_deg, (size_t)n_angles * sizeof(double), hipMemcpyHostToDevice, st), "H2D angles");
        if (phi_deg)
            hip_check(hipMemcpyAsync(ang + kFfMaxAngles, phi_deg, (size_t)n_angles * sizeof(double),
                                     hipMemcpyHostToDevice, st), "H2D angles");
        const unsigned ab = (unsigned)((n_angles + 255) / 256);
        hipLaunchKernelGGL(k_ff_angles, dim3(ab), dim3(256), 0, st, ang, n_angles, phi_deg ? 1 : 0);
        hip_check(hipGetLastError(), "k_ff_angles");
        const double *acc_inc = inc ? inc->acc : nullptr;
        if (use_line) {
            const Box &b = h->box;
            const int64_t cells = (int64_t)(b.hi[0] - b.lo[0] + 1) * (b.hi[1] - b.lo[1] + 1) * (b.hi[2] - b.lo[2] + 1);
            const unsigned lb = (unsigned)std::min<int64_t>((cells + 256) / 256, 1024);
            hipLaunchKernelGGL(k_ff_line_nodes, dim3(lb), dim3(256), 0, st, h->line_acc, line, b, h->dim, h->line_axis,
                               h->probe[h->line_axis], h->nnodes);
            hip_check(hipGetLastError(), "k_ff_line_nodes");
            acc_inc = line;
        }
        NtffArgs a{};
        a.acc = h->acc;
        a.acc_inc = acc_inc;
        a.box = h->box;
        a.dim = h->dim;
        a.pol = h->cfg.pol;
        a.k = 2.0 * M_PI / h->pw.lambda;
        const auto &c = h->cfg;
        a.center[0] = (c.nx - 1) / 2.0;
        a.center[1] = (c.ny - 1) / 2.0;
        a.center[2] = h->dim == 3 ? (c.nz - 1) / 2.0 : 0.0;
        for (int k = 0; k < 3; ++k) {
            a.khat[k] = h->pw.khat[k];
            a.ehat[k] = h->pw.ehat[k];
            a.bhat[k] = h->hhat[k];
        }
        a.theta = ang;
        a.phi = ang + kFfMaxAngles;
        a.out = P;
        hipLaunchKernelGGL(k_ntff, dim3(n_angles), dim3(256), 0, st, a);
        hip_check(hipGetLastError(), "k_ntff");
        const double k = a.k;
        const double kappa = h->dim == 2 ? k * k / (8.0 * M_PI) : k * k * k * k / (16.0 * M_PI * M_PI);
        const double *u = h->cfg.pol == LBM_EM_TE ? h->hhat : h->pw.ehat;
        const double *probe = acc_inc ? acc_inc + h->nnodes * 12 + (h->cfg.pol == LBM_EM_TE ? 6 : 0) : nullptr;
        hipLaunchKernelGGL(k_ff_finish, dim3(ab), dim3(256), 0, st, P, probe, u[0], u[1], u[2], h->pw.amplitude,
                           kappa, n_angles, S2, amp_d);
        hip_check(hipGetLastError(), "k_ff_finish");
        double amp = 0.0;
        hip_check(hipMemcpyAsync(&amp, amp_d, sizeof amp, hipMemcpyDeviceToHost, st), "D2H amplitude");
        sync(h);
        if (!(amp > 0.0)) fail(LBM_EM_ESTATE, "incident amplitude at the probe node is zero (the wave has not arrived)");
        hip_check(hipMemcpyAsync(out_S2, S2, (size_t)n_angles * sizeof(double), hipMemcpyDeviceToHost, st), "D2H S2");
        sync(h);
    });
}

lbm_em_status lbm_em_adjoint_setup(lbm_em_handle hh, lbm_em_handle inc, const double *theta_deg,
                                   const double *weight, int32_t n_angles, const int32_t dlo[2],
                                   const int32_t dhi[2], int32_t checkpoint_every) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (h->dim != 2) fail(LBM_EM_EUNSUPPORTED, "the adjoint supports 2-D (TM/TE) handles");
        if (h->mu) fail(LBM_EM_EUNSUPPORTED, "the adjoint needs mu_r = 1");
        if (h->line) fail(LBM_EM_EUNSUPPORTED, "the adjoint uses the companion run, not an incident line");
        if (!inc) fail(LBM_EM_EINVAL, "the objective needs the incident (eps = 1) companion handle");
        if (!theta_deg || n_angles < 1) fail(LBM_EM_EINVAL, "need at least one angle");
        if (!dlo || !dhi) fail(LBM_EM_EINVAL, "null design rectangle");
        if (!h->dft_set || !h->src_on) fail(LBM_EM_ESTATE, "set the source and contour first");
        if (checkpoint_every < 0) fail(LBM_EM_EINVAL, "checkpoint_every must be >= 0");
        const int n[2] = {h->cfg.nx, h->cfg.ny};
        for (int a = 0; a < 2; ++a) {
            if (dlo[a] > dhi[a] || dlo[a] < 0 || dhi[a] >= n[a]) fail(LBM_EM_EINVAL, "design rectangle outside the grid");
            if (dlo[a] <= h->box.lo[a] || dhi[a] >= h->box.hi[a])
                fail(LBM_EM_EINVAL, "design rectangle must lie strictly inside the contour box");
            const int W = h->cfg.absorb[a];
            if (W && (dlo[a] < W || dhi[a] >= n[a] - W)) fail(LBM_EM_EINVAL, "design rectangle overlaps the layer");
        }
        h->adj_inc = check_handle(inc);
        if (h->adj_inc->mu) fail(LBM_EM_EUNSUPPORTED, "the adjoint needs mu_r = 1");
        h->adj_theta.assign(n_angles, 0.0);
        h->adj_w.assign(n_angles, 1.0);
        for (int i = 0; i < n_angles; ++i) {
            h->adj_theta[i] = theta_deg[i] * M_PI / 180.0;
            if (weight) h->adj_w[i] = weight[i];
        }
        for (int a = 0; a < 2; ++a) {
            h->dlo[a] = dlo[a];
            h->dhi[a] = dhi[a];
        }
        h->ck_every = checkpoint_every;
        h->adj_T = 0;
        h->adj_set = true;
    });
}

lbm_em_status lbm_em_forward_checkpointed(lbm_em_handle hh, int64_t n, double *J_out) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!h->adj_set) fail(LBM_EM_ESTATE, "call lbm_em_adjoint_setup first");
        if (!J_out) fail(LBM_EM_EINVAL, "null J_out");
        if (n < h->win0 + h->winlen) fail(LBM_EM_EINVAL, "n must cover the DFT window");
        check_incident(h, h->adj_inc);
        select_device(h);
        reset_state(h);
        const int K = h->ck_every > 0 ? h->ck_every : (int)std::ceil(std::sqrt((double)n));
        const int nck = (int)((n + K - 1) / K);
        const size_t sb = (size_t)h->plane * h->nplanes * h->elem;
        if (h->ck_bytes < sb * nck) {
            hfree(h->ck);
            h->ck = nullptr;
            h->ck_bytes = 0;
            hip_check(hipMalloc(&h->ck, sb * nck), "hipMalloc checkpoints");
            h->ck_bytes = sb * nck;
        }
        h->nck = nck;
        h->ck_k = K;
        for (int k = 0; k < nck; ++k) {
            hip_check(hipMemcpyAsync((char *)h->ck + sb * k, h->buf[h->cur], sb, hipMemcpyDeviceToDevice, h->stream),
                      "checkpoint");
            do_steps(h, std::min<int64_t>(K, n - (int64_t)k * K));
        }
        const int na = (int)h->adj_theta.size();
        hfree(h->adj_P);
        h->adj_P = nullptr;
        hip_check(hipMalloc(&h->adj_P, (size_t)na * 4 * sizeof(double)), "hipMalloc");
        const double amp = farfield_P(h, h->adj_inc->acc, h->adj_theta.data(), nullptr, na, h->adj_P);
        if (!(amp > 0.0)) fail(LBM_EM_ESTATE, "incident amplitude at the probe node is zero (the wave has not arrived)");
        std::vector<double> P((size_t)na * 4);
        hip_check(hipMemcpyAsync(P.data(), h->adj_P, P.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream), "D2H");
        sync(h);
        const double k = 2.0 * M_PI / h->pw.lambda;
        h->adj_kappa = k * k / (8.0 * M_PI) / (amp * amp);
        double J = 0.0;
        for (int i = 0; i < na; ++i)
            J += h->adj_w[i] * h->adj_kappa * (P[4 * i] * P[4 * i] + P[4 * i + 1] * P[4 * i + 1]);
        h->adj_T = n;
        *J_out = J;
    });
}

lbm_em_status lbm_em_backward(lbm_em_handle hh, double *grad_eps, int32_t where) {
    return guarded([&] {
        lbm_em *h = check_handle(hh);
        if (!h->adj_set || h->adj_T == 0 || h->t != h->adj_T)
            fail(LBM_EM_ESTATE, "call lbm_em_forward_checkpointed (and nothing else) first");
        if (!grad_eps) fail(LBM_EM_EINVAL, "null gradient output");
        if (where != LBM_EM_HOST && where != LBM_EM_DEVICE) fail(LBM_EM_EINVAL, "where must be HOST or DEVICE");
        select_device(h);
        const int64_t T = h->adj_T;
        const int K = h->ck_k, nck = h->nck;
        const int ncomp = h->cfg.pol == LBM_EM_TM ? 1 : 2;
        const int64_t dcells = (int64_t)(h->dhi[0] - h->dlo[0] + 1) * (h->dhi[1] - h->dlo[1] + 1);
        const size_t sb = (size_t)h->plane * h->nplanes * h->elem;
        void *abuf[2] = {nullptr, nullptr};
        void *hist = nullptr;
        double *grad = nullptr, *G = nullptr;
        try {
            hip_check(hipMalloc(&abuf[0], sb), "hipMalloc adjoint");
            hip_check(hipMalloc(&abuf[1], sb), "hipMalloc adjoint");
            hip_check(hipMalloc(&hist, (size_t)K * dcells * ncomp * h->elem), "hipMalloc history");
            hip_check(hipMalloc(&grad, dcells * sizeof(double)), "hipMalloc gradient");
            hip_check(hipMalloc(&G, (size_t)h->nnodes * 12 * sizeof(double)), "hipMalloc weights");
            hip_check(hipMemsetAsync(abuf[0], 0, sb, h->stream), "hipMemset");
            hip_check(hipMemsetAsync(abuf[1], 0, sb, h->stream), "hipMemset");
            hip_check(hipMemsetAsync(grad, 0, dcells * sizeof(double), h->stream), "hipMemset");
            // adjoint source weights from the forward far field
            const int na = (int)h->adj_theta.size();
            double *d_tw = nullptr;
            std::vector<double> tw(2 * (size_t)na);
            for (int i = 0; i < na; ++i) {
                tw[i] = h->adj_theta[i];
                tw[na + i] = h->adj_w[i];
            }
            hip_check(hipMalloc(&d_tw, tw.size() * sizeof(double)), "hipMalloc");
            hip_check(hipMemcpyAsync(d_tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice, h->stream), "H2D");
            AdjWeightArgs wa{};
            wa.box = h->box;
            wa.pol = h->cfg.pol;
            wa.k = 2.0 * M_PI / h->pw.lambda;
            wa.kappa = h->adj_kappa;
            wa.center[0] = (h->cfg.nx - 1) / 2.0;
            wa.center[1] = (h->cfg.ny - 1) / 2.0;
            for (int k = 0; k < 3; ++k) wa.khat[k] = h->pw.khat[k];
            wa.theta = d_tw;
            wa.w = d_tw + na;
            wa.P = h->adj_P;
            wa.n_angles = na;
            wa.nnodes = h->nnodes;
            wa.G = G;
            hipLaunchKernelGGL(k_adjoint_weights2d, dim3((unsigned)((h->nnodes + 255) / 256)), dim3(256), 0, h->stream, wa);
            hip_check(hipGetLastError(), "k_adjoint_weights2d");
            int ap = 0;
            for (int k = nck - 1; k >= 0; --k) {
                const int64_t t0 = (int64_t)k * K, t1 = std::min<int64_t>(t0 + K, T);
                // recompute the segment from its checkpoint, recording dE/deps
                hip_check(hipMemcpyAsync(h->buf[0], (char *)h->ck + sb * k, sb, hipMemcpyDeviceToDevice, h->stream),
                          "restore");
                // (two steps per launch where the handle uses them, then a
                // single trailing step)
                int cur = 0;
                int64_t t = t0;
                if (h->fuse == 2)
                    for (; t + 2 <= t1; t += 2) {
                        launch_step2(h, cur, nullptr, t, h->stream, false, hist, t0);
                        hip_check(hipGetLastError(), "recompute");
                        cur ^= 1;
                    }
                for (; t < t1; ++t) {
                    launch_step(h, cur, nullptr, t, h->stream, false, hist, t0);
                    hip_check(hipGetLastError(), "recompute");
                    cur ^= 1;
                }
                // reverse sweep over the segment (two steps per launch where
                // the handle uses them)
                auto hs = [&](int64_t tt) { return (const char *)hist + (size_t)(tt - t0) * dcells * ncomp * h->elem; };
                for (int64_t t = t1 - 1; t >= t0;) {
                    const bool two = h->fuse == 2 && t - 1 >= t0;
                    const void *hp = two ? hs(t - 1) : nullptr;
                    if (h->elem == 4) launch_adjoint<float>(h, abuf[ap], abuf[ap ^ 1], t, hs(t), grad, G, hp);
                    else launch_adjoint<double>(h, abuf[ap], abuf[ap ^ 1], t, hs(t), grad, G, hp);
                    hip_check(hipGetLastError(), "adjoint step");
                    ap ^= 1;
                    t -= two ? 2 : 1;
                }
            }
            hip_check(hipMemcpyAsync(grad_eps, grad, dcells * sizeof(double),
                                     where == LBM_EM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, h->stream),
                      "gradient copy");
            sync(h);
            hfree(d_tw);
        } catch (...) {
            hfree(abuf[0]); hfree(abuf[1]); hfree(hist); hfree(grad); hfree(G);
            throw;
        }
        hfree(abuf[0]); hfree(abuf[1]); hfree(hist); hfree(grad); hfree(G);
        // the recompute used the state buffers: start over
        reset_state(h);
        h->adj_T = 0;
    });
}

lbm_em_status lbm_em_copy_bandwidth(int64_t bytes, int32_t reps, double *gbs) {
    return guarded([&] {
        if (bytes < 16 || bytes % 16 != 0 || reps < 1 || !gbs) fail(LBM_EM_EINVAL, "bytes must be a positive multiple of 16");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(LBM_EM_EDEVICE, "no HIP device");
        void *a = nullptr, *b = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        try {
            hip_check(hipMalloc(&a, bytes), "hipMalloc");
            hip_check(hipMalloc(&b, bytes), "hipMalloc");
            hip_check(hipMemset(a, 0, bytes), "hipMemset");
            const int64_t n = bytes / 16;
            const unsigned blocks = (unsigned)((n + 255) / 256);
            hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(256), 0, nullptr, (const float4 *)a, (float4 *)b, n);
            hip_check(hipEventCreate(&e0), "hipEventCreate");
            hip_check(hipEventCreate(&e1), "hipEventCreate");
            hip_check(hipEventRecord(e0, nullptr), "hipEventRecord");
            for (int r = 0; r < reps; ++r)
                hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(256), 0, nullptr, (const float4 *)a, (float4 *)b, n);
            hip_check(hipEventRecord(e1, nullptr), "hipEventRecord");
            hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
        } catch (...) {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            hfree(a);
            hfree(b);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        hfree(a);
        hfree(b);
    });
}

lbm_em_status lbm_em_stream_bandwidth(int64_t cells, int32_t planes_in, int32_t planes_out, int32_t reps,
                                      double *gbs) {
    return guarded([&] {
        if (cells < 1 || cells > ((int64_t)1 << 31) || planes_in < 1 || planes_in > 32 || planes_out < 1 ||
            planes_out > planes_in || reps < 1 || !gbs)
            fail(LBM_EM_EINVAL, "need 1 <= cells <= 2^31, 1 <= planes_out <= planes_in <= 32, reps >= 1");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(LBM_EM_EDEVICE, "no HIP device");
        const int64_t P = plane_stride(cells, 4);   // the state's plane layout
        void *a = nullptr, *b = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        try {
            hip_check(hipMalloc(&a, (size_t)P * planes_in * sizeof(float)), "hipMalloc");
            hip_check(hipMalloc(&b, (size_t)P * planes_out * sizeof(float)), "hipMalloc");
            hip_check(hipMemset(a, 0, (size_t)P * planes_in * sizeof(float)), "hipMemset");
            const unsigned blocks = (unsigned)((cells + 255) / 256);
            auto launch = [&] {
                hipLaunchKernelGGL(k_stream_planes, dim3(blocks), dim3(256), 0, nullptr, (const float *)a, (float *)b,
                                   P, cells, planes_in, planes_out);
            };
            launch();
            hip_check(hipEventCreate(&e0), "hipEventCreate");
            hip_check(hipEventCreate(&e1), "hipEventCreate");
            hip_check(hipEventRecord(e0, nullptr), "hipEventRecord");
            for (int r = 0; r < reps; ++r) launch();
            hip_check(hipEventRecord(e1, nullptr), "hipEventRecord");
            hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            *gbs = (double)(planes_in + planes_out) * 4.0 * (double)cells * reps / (ms * 1e-3) / 1e9;
        } catch (...) {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            hfree(a);
            hfree(b);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        hfree(a);
        hfree(b);
    });
}

}  // extern "C"


