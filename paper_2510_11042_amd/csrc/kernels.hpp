// kernels.hpp -- gfx950 kernels of the electromagnetic lattice Boltzmann hot path.
//
// Scheme (paper section 2.1, Eq. LBGK_equation and Eq. EDF): D3Q7 velocities
// c_0 = 0, +-x, +-y, +-z; vector distributions e_i, h_i; tau = 1/2 update
//   f_i(r + c_i, t+1) = 2 f_i^eq(r,t) - f_i(r,t),
//   e_i^eq = (E - c_i x H)/6, h_i^eq = (H + c_i x E)/6 (i != 0),
//   e_0^eq = (eps_r - 1) E, h_0^eq = (mu_r - 1) H,
// and fields from the zeroth moments, E = sum_i e_i / eps_r, H = sum_i h_i / mu_r.
// mu_r = 1 except in the 2-D one-step kernel's permeability variant (MU).
//
// Exact reduced state.  For every moving direction the combination
// e_i_perp + c_i x h_i has zero equilibrium, so collision only flips its sign,
// streaming carries it along, and the absorbing layer relaxes it towards
// zero: from a zero (or equilibrium) start it stays zero and
// h_i = eta_i c_i + c_i x e_i with eta_i = h_i . c_i.  h_0 stays zero for
// mu_r = 1.  That leaves 27 scalars per cell in 3-D (e_i and eta_i for six
// directions, e_0).  In 2-D (nz = 1, z streaming the identity) the +z and -z
// populations never move and have equal equilibria, so they stay equal and
// merge into one "z-pair", and the rest population is slaved to it,
// e_0 = 6 (eps_r - 1) e_zpair (the difference flips sign every step and
// starts at zero; the layer relaxes both towards equilibria in the same
// ratio).  By the same argument h_0 = 6 (mu_r - 1) h_zpair, so a 2-D
// permeability map needs no extra state.  A 2-D polarisation then needs 11
// scalars per cell:
//   TM (E_z, H_x, H_y): planes 0..3  e_z of +x,-x,+y,-y
//                       planes 4..7  h_x of +-x, h_y of +-y   (eta)
//                       planes 8..10 z-pair e_z, h_x, h_y
//   TE (E_x, E_y, H_z): planes 0..3  e_x of +x,-x,+y,-y
//                       planes 4..7  e_y of +x,-x,+y,-y
//                       planes 8..10 z-pair e_x, e_y, h_z
//   3-D:                planes 4d..4d+2 e of direction d (+x,-x,+y,-y,+z,-z),
//                       plane 4d+3 eta_d, planes 24..26 e_0.
// Fields computed from this state equal those of the literal 42-scalar scheme.
//
// Storage: structure of arrays, one plane per scalar, x fastest, each buffer
// holding the post-collision state f*(t-1); a step PULLS f_i(r,t) =
// f*_i(r - c_i, t-1).  On an absorbing axis the pull is clamped at the faces,
// which is exactly the paper's open boundary (section 2.2, f_i^L = f_i^{L-dx}
// for incoming populations): the incoming population of the boundary node
// takes the post-collision value of the node itself, the one the first
// interior node received by streaming.  Periodic axes wrap.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <stdint.h>

namespace lbm {

enum { TM = 0, TE = 1, D3 = 2 };

struct Box {
    int lo[3], hi[3];
};

// Unique index of a node on the surface of a node box (2-D: nz == 1 box with
// lo[2] == hi[2]).  Ordering: 2-D bottom edge, top edge, left edge without
// corners, right edge without corners; 3-D faces z_lo, z_hi (full), y_lo,
// y_hi (z strictly inside), x_lo, x_hi (y and z strictly inside).
__host__ __device__ inline int64_t box_nodes(const Box &b, int dim) {
    int64_t nbx = b.hi[0] - b.lo[0] + 1, nby = b.hi[1] - b.lo[1] + 1, nbz = b.hi[2] - b.lo[2] + 1;
    if (dim == 2) return 2 * nbx + 2 * (nby - 2);
    return 2 * nbx * nby + 2 * nbx * (nbz - 2) + 2 * (nby - 2) * (nbz - 2);
}

__host__ __device__ inline int64_t box_node_index(const Box &b, int dim, int x, int y, int z) {
    int64_t nbx = b.hi[0] - b.lo[0] + 1, nby = b.hi[1] - b.lo[1] + 1, nbz = b.hi[2] - b.lo[2] + 1;
    int64_t dx = x - b.lo[0], dy = y - b.lo[1], dz = z - b.lo[2];
    if (dim == 2) {
        if (y == b.lo[1]) return dx;
        if (y == b.hi[1]) return nbx + dx;
        if (x == b.lo[0]) return 2 * nbx + (dy - 1);
        return 2 * nbx + (nby - 2) + (dy - 1);
    }
    int64_t fxy = nbx * nby, fxz = nbx * (nbz - 2), fyz = (nby - 2) * (nbz - 2);
    if (z == b.lo[2]) return dy * nbx + dx;
    if (z == b.hi[2]) return fxy + dy * nbx + dx;
    if (y == b.lo[1]) return 2 * fxy + (dz - 1) * nbx + dx;
    if (y == b.hi[1]) return 2 * fxy + fxz + (dz - 1) * nbx + dx;
    if (x == b.lo[0]) return 2 * fxy + 2 * fxz + (dz - 1) * (nby - 2) + (dy - 1);
    return 2 * fxy + 2 * fxz + fyz + (dz - 1) * (nby - 2) + (dy - 1);
}

__host__ __device__ inline bool on_box(const Box &b, int dim, int x, int y, int z) {
    bool in = x >= b.lo[0] && x <= b.hi[0] && y >= b.lo[1] && y <= b.hi[1] &&
              z >= b.lo[2] && z <= b.hi[2];
    if (!in) return false;
    bool sx = x == b.lo[0] || x == b.hi[0];
    bool sy = y == b.lo[1] || y == b.hi[1];
    if (dim == 2) return sx || sy;
    return sx || sy || z == b.lo[2] || z == b.hi[2];
}

// Everything one step needs.  Per-step quantities (source ramp and phase,
// DFT factor) are derived in the kernel from the step index t, so the same
// launch can be replayed from a graph with t read from device memory.
template <typename T> struct Cplx;
template <> struct Cplx<float> { typedef float2 type; };
template <> struct Cplx<double> { typedef double2 type; };

// Steps of the incident line kept in its table: one captured graph chunk.
constexpr int kLineSlots = 64;
// Most planes one block of the 3-D two-step kernel marches (its z chunk
// plus the two extra planes); the host caps the chunk length accordingly.
constexpr int kX3MaxPlanes = 1024;

// x/3 and x/6 as if the constants were exact.  The collision is
// f* = 2 f^eq - f with 2 f^eq = combination / 3, and the rounded 1/3 of
// FP32 is 3.0e-8 too large (FP64: 1.9e-17 too small): multiplying by it
// scales the moments D and B, which the collision conserves exactly, by
// (1 + 6e-8) every step -- a systematic gain of 1e-4 along the ~1500 steps
// a wave needs to cross a 1024^2 grid.  Splitting the constant into its
// rounded head and the tail, fma(x, head, x * tail), rounds x/3 correctly
// in all but rare ties, so the remaining rounding errors have no bias.
// sixth(2x) == third(x) bit for bit (the halved head and tail are exact).
template <typename T> struct Frac3;
template <> struct Frac3<float> {
    static constexpr float hi = 1.0f / 3.0f;
    static constexpr float lo = (float)(1.0 / 3.0 - (double)(1.0f / 3.0f));   // -9.93e-9
};
template <> struct Frac3<double> {
    static constexpr double hi = 1.0 / 3.0;
    static constexpr double lo = 1.850371707708594e-17;   // 1/3 - hi = 2^-54 / 3
};
template <typename T>
__device__ inline T third(T x) {
    return fma(x, Frac3<T>::hi, x * Frac3<T>::lo);
}
template <typename T>
__device__ inline T sixth(T x) {
    return fma(x, Frac3<T>::hi * T(0.5), x * (Frac3<T>::lo * T(0.5)));
}

template <typename T>
struct StepArgs {
    int nx, ny, nz;
    int64_t sy, sz, plane;      // element strides: row, slab, plane
    int W[3];                   // absorbing width per axis, 0 = periodic
    T inv_w[3];                 // 1 / W (0 on a periodic axis)
    T sigma_max;
    const T *__restrict__ src;  // f*(t-1), nplanes planes
    T *__restrict__ dst;        // f*(t)
    const T *__restrict__ eps;
    const T *__restrict__ mu;   // relative permeability, read by the MU variants only
    const int64_t *t_base;      // graph replay: t = *t_base + t_off; else NULL
    int64_t t_off;
    // plane-wave source (phase tables: see plane_wave)
    int src_on;
    int period;                 // T = 3 lambda steps
    double amp, t_ramp;
    T ehat[3], hhat[3];         // E and H directions of the incident wave
    const double *ramp;         // g(t) for t < t_ramp
    const double2 *wave_t;      // e^{2 pi j k / T}, k < T
    const typename Cplx<T>::type *wave_x, *wave_y, *wave_z;   // e^{2 pi j u_a} per column / row / slab
    // running DFT on the contour box + probe node
    int dft_on;
    Box box;
    int probe[3];
    int64_t nnodes;
    int64_t win0, winlen;
    double *acc;                // (nnodes + 1) x 6 x (re, im)
    int tiles_x, tiles_y;       // tile grid of the launch (3-D: per z slab)
    // inverse design: record d = dE/deps (at fixed pulled populations) for
    // the cells of the design rectangle [dlo, dhi] into hist[t - hist_t0]
    T *hist;
    int dlo[2], dhi[2];
    int64_t hist_t0;
    // exact incident line (2-D, incidence along axis line_axis, line_n cells
    // on it): post-collision populations of the line at step t in slot
    // t mod kLineSlots (kLineSlots x 11 planes x line_n).  The grid's kernels read line_tab; the
    // line's own kernel writes line_rec and its phasors line_acc (line_n x 12).
    const T *line_tab;
    T *line_rec;
    double *line_acc;
    int line_axis, line_n;
    // 3-D: per plane z, the box (x_lo, x_hi, y_lo, y_hi) holding every cell
    // whose eps_r differs from 1 or whose rest populations may be non-zero
    // (empty: x_lo > x_hi); NULL: no plane is known to be vacuum
    const int4 *vbox;
};

// Layer strength at coordinate x of an axis of n cells with a layer of W
// cells at each end: sigma_max (d / W)^2 at depth d (1 .. W), 0 inside.
// inv_w = 1 / W (0 on a periodic axis) comes precomputed from the host.
template <typename T>
__device__ inline T sigma_axis(int x, int n, int W, T inv_w, T smax) {
    int d = 0;
    if (W > 0) {
        if (x < W) d = W - x;
        else if (x >= n - W) d = x - (n - W) + 1;
    }
    const T u = T(d) * inv_w;
    return smax * u * u;
}

__device__ inline int64_t step_time(const int64_t *t_base, int64_t t_off) {
    return (t_base ? *t_base : 0) + t_off;
}

// Per-step quantities shared by every cell of a launch (or of one work item
// of a batched launch), formed once from the step index t.
//
// Source: the incident value w = g(t) E0 sin(omega t - k khat.(r - rc)) at
// a cell.  With tau = (t mod T) / T and u = khat.(r - rc) / lambda split per
// axis as u = u_x(x) + u_y(y) + u_z(z),
//   w = g E0 sin(2 pi tau) cos(2 pi u) - g E0 cos(2 pi tau) sin(2 pi u),
// where e^{2 pi j u} is the product of per-axis factors.  Every factor comes
// from FP64 tables the host fills when the source is set (each phase reduced
// modulo one period first), so a cell pays two or three gathers and a few
// multiplies instead of an FP64 sine.
// DFT: inside the window, the factor (2 / winlen) e^{-j omega t}.
template <typename T>
struct StepConst {
    int64_t t;
    T gs, gc;           // g(t) E0 sin(2 pi tau), g(t) E0 cos(2 pi tau)
    bool dft;           // t lies in the DFT window
    double cr, ci;      // (2 / winlen) (cos, -sin)(2 pi tau)
};

// The step's constants from its period phasor ph = wave_t[t mod T] and its
// ramp value r = g(t) (1 past the ramp).
template <typename T>
__device__ inline StepConst<T> form_step_const(const StepArgs<T> &a, int64_t t, double2 ph, double r) {
    StepConst<T> c{t, T(0), T(0), false, 0.0, 0.0};
    const double g = r * a.amp;
    c.gs = (T)(g * ph.y);
    c.gc = (T)(g * ph.x);
    if (a.dft_on && t >= a.win0 && t < a.win0 + a.winlen) {
        const double sc = 2.0 / (double)a.winlen;
        c.dft = true;
        c.cr = sc * ph.x;
        c.ci = -sc * ph.y;
    }
    return c;
}

template <typename T>
__device__ inline StepConst<T> step_const(const StepArgs<T> &a, int64_t t) {
    if (!a.src_on) return StepConst<T>{t, T(0), T(0), false, 0.0, 0.0};   // the DFT needs the source's period too
    return form_step_const(a, t, a.wave_t[t % a.period], (double)t < a.t_ramp ? a.ramp[t] : 1.0);
}

// The constants of steps t and t + 1 (the same values as step_const), their
// table reads issued together.
template <typename T>
__device__ inline void step_consts2(const StepArgs<T> &a, int64_t t, StepConst<T> &c0, StepConst<T> &c1) {
    if (!a.src_on) {
        c0 = StepConst<T>{t, T(0), T(0), false, 0.0, 0.0};
        c1 = StepConst<T>{t + 1, T(0), T(0), false, 0.0, 0.0};
        return;
    }
    const int64_t k0 = t % a.period, k1 = k0 + 1 == a.period ? 0 : k0 + 1;
    const double2 ph0 = a.wave_t[k0], ph1 = a.wave_t[k1];
    double r0 = 1.0, r1 = 1.0;
    if ((double)(t + 1) < a.t_ramp) {
        r0 = a.ramp[t];
        r1 = a.ramp[t + 1];
    } else if ((double)t < a.t_ramp) {
        r0 = a.ramp[t];
    }
    c0 = form_step_const(a, t, ph0, r0);
    c1 = form_step_const(a, t + 1, ph1, r1);
}

// The x-y part e^{2 pi j (u_x(x) + u_y(y))} of a cell's phase factor.
template <typename T>
__device__ inline typename Cplx<T>::type xy_phase(const StepArgs<T> &a, int x, int y) {
    const auto px = a.wave_x[x], py = a.wave_y[y];
    typename Cplx<T>::type w;
    w.x = px.x * py.x - px.y * py.y;
    w.y = px.x * py.y + px.y * py.x;
    return w;
}

// The incident value at a 3-D cell from its x-y factor and the z factor of
// its plane.
template <typename T>
__device__ inline T plane_wave_xyz(const StepConst<T> &sc, typename Cplx<T>::type wxy, typename Cplx<T>::type pz) {
    const T ur = wxy.x * pz.x - wxy.y * pz.y;
    const T ui = wxy.x * pz.y + wxy.y * pz.x;
    return sc.gs * ur - sc.gc * ui;
}

// The incident value at a cell, in the arithmetic type of the run (the
// per-axis tables are stored in it).
template <typename T, int DIM>
__device__ inline T plane_wave(const StepArgs<T> &a, const StepConst<T> &sc, int x, int y, int z) {
    const auto w = xy_phase(a, x, y);
    if (DIM == 3) return plane_wave_xyz(sc, w, a.wave_z[z]);
    return sc.gs * w.x - sc.gc * w.y;
}

// 1 / eps: for FP32 the hardware reciprocal refined by one Newton step
// (within an ulp of the rounded quotient, exact for eps = 1), for FP64 the
// rounded quotient.  Every kernel uses this, so they stay bit-identical.
template <typename T>
__device__ inline T recip(T e) {
    if constexpr (sizeof(T) == 4) {
        const float r = __builtin_amdgcn_rcpf(e);
        return __builtin_fmaf(r, __builtin_fmaf(-e, r, 1.0f), r);
    } else {
        return 1.0 / e;
    }
}

// Fields at a cell from pulled 2-D reduced populations.
//   TM: F = (E_z, H_x, H_y); TE: F = (E_x, E_y, H_z).
// MU: the cell has permeability mu (inv_mu = 1/mu); else mu_r = 1.  In the
// MU variant mu == 0 flags a perfect conductor: E = 0 there, and H is
// recovered with mu_r = 1 (the rest populations of such a cell stay zero).
template <typename T, int POL, bool MU = false>
__device__ inline void fields2d(const T s[11], T eps, T inv_eps, T F[3], T mu = T(1), T inv_mu = T(1)) {
    const T rest = fma(T(6), eps, T(-4));  // z-pair (x2) plus slaved rest population
    const bool pec = MU && mu == T(0);
    if (MU && pec) {
        mu = T(1);
        inv_mu = T(1);
    }
    if (POL == TM) {
        F[0] = pec ? T(0) : fma(rest, s[8], s[0] + s[1] + s[2] + s[3]) * inv_eps;
        if (MU) {
            const T rest_h = fma(T(6), mu, T(-4));
            F[1] = fma(rest_h, s[9], s[4] + s[5] + s[2] - s[3]) * inv_mu;
            F[2] = fma(rest_h, s[10], s[6] + s[7] - s[0] + s[1]) * inv_mu;
        } else {
            F[1] = fma(T(2), s[9], s[4] + s[5] + s[2] - s[3]);
            F[2] = fma(T(2), s[10], s[6] + s[7] - s[0] + s[1]);
        }
    } else {
        F[0] = pec ? T(0) : fma(rest, s[8], s[0] + s[1] + s[2] + s[3]) * inv_eps;
        F[1] = pec ? T(0) : fma(rest, s[9], s[4] + s[5] + s[6] + s[7]) * inv_eps;
        if (MU) F[2] = fma(fma(T(6), mu, T(-4)), s[10], s[4] - s[5] - s[2] + s[3]) * inv_mu;
        else F[2] = fma(T(2), s[10], s[4] - s[5] - s[2] + s[3]);
    }
}

// Equilibrium of the 11 reduced scalars for fields F, scaled by `scale`
// (scale = 2 gives 2 f^eq for the collision, 1 the plain equilibrium).
template <typename T, int POL>
__device__ inline void equilibrium2d(const T F[3], T scale, T q[11]) {
    const T c = scale / T(6);
    if (POL == TM) {
        const T Ez = F[0], Hx = F[1], Hy = F[2];
        q[0] = c * (Ez - Hy);
        q[1] = c * (Ez + Hy);
        q[2] = c * (Ez + Hx);
        q[3] = c * (Ez - Hx);
        q[4] = q[5] = c * Hx;
        q[6] = q[7] = c * Hy;
        q[8] = c * Ez;
        q[9] = c * Hx;
        q[10] = c * Hy;
    } else {
        const T Ex = F[0], Ey = F[1], Hz = F[2];
        q[0] = q[1] = c * Ex;
        q[2] = c * (Ex - Hz);
        q[3] = c * (Ex + Hz);
        q[4] = c * (Ey + Hz);
        q[5] = c * (Ey - Hz);
        q[6] = q[7] = c * Ey;
        q[8] = c * Ex;
        q[9] = c * Ey;
        q[10] = c * Hz;
    }
}

// 2 f^eq - f for the eleven scalars from the fields' thirds F3 = F/3
// (each rounded correctly by third() or sixth(), so no bias from the
// rounded constant; the combinations and the subtraction then round
// without bias too).
template <typename T, int POL>
__device__ inline void collide2d_thirds(const T F3[3], T f[11]) {
    if (POL == TM) {
        const T ez = F3[0], hx = F3[1], hy = F3[2];
        f[0] = (ez - hy) - f[0];
        f[1] = (ez + hy) - f[1];
        f[2] = (ez + hx) - f[2];
        f[3] = (ez - hx) - f[3];
        f[4] = hx - f[4];
        f[5] = hx - f[5];
        f[6] = hy - f[6];
        f[7] = hy - f[7];
        f[8] = ez - f[8];
        f[9] = hx - f[9];
        f[10] = hy - f[10];
    } else {
        const T ex = F3[0], ey = F3[1], hz = F3[2];
        f[0] = ex - f[0];
        f[1] = ex - f[1];
        f[2] = (ex - hz) - f[2];
        f[3] = (ex + hz) - f[3];
        f[4] = (ey + hz) - f[4];
        f[5] = (ey - hz) - f[5];
        f[6] = ey - f[6];
        f[7] = ey - f[7];
        f[8] = ex - f[8];
        f[9] = ey - f[9];
        f[10] = hz - f[10];
    }
}

// Collision at tau = 1/2: f <- 2 f^eq(F) - f, every population a
// combination of the fields divided by 3.
template <typename T, int POL>
__device__ inline void collide2d(const T F[3], T f[11]) {
    const T F3[3] = {third(F[0]), third(F[1]), third(F[2])};
    collide2d_thirds<T, POL>(F3, f);
}

// Accumulate the running DFT of the fields at a contour / probe node.
// F = (Ex, Ey, Ez, Hx, Hy, Hz); only the components in MASK (bit c for
// F[c]) are non-zero for this field layout and are accumulated.
template <int MASK, typename T>
__device__ inline void dft_accumulate(const StepArgs<T> &a, const StepConst<T> &st, int dim, int x, int y,
                                      int z, const double F[6]) {
    if (!st.dft) return;
    bool surf = on_box(a.box, dim, x, y, z);
    bool probe = x == a.probe[0] && y == a.probe[1] && z == a.probe[2];
    if (!surf && !probe) return;
    const double cr = st.cr, ci = st.ci;
    for (int pass = 0; pass < 2; ++pass) {
        int64_t node;
        if (pass == 0) {
            if (!surf) continue;
            node = box_node_index(a.box, dim, x, y, z);
        } else {
            if (!probe) continue;
            node = a.nnodes;
        }
        double *p = a.acc + node * 12;
#pragma unroll
        for (int c = 0; c < 6; ++c)
            if ((MASK >> c) & 1) {
                p[2 * c] += F[c] * cr;
                p[2 * c + 1] += F[c] * ci;
            }
    }
}

// Pull neighbours with the open boundary (clamp) or periodic wrap.
__device__ inline int pull_lo(int x, int n, int W) { return x > 0 ? x - 1 : (W ? 0 : n - 1); }
__device__ inline int pull_hi(int x, int n, int W) { return x < n - 1 ? x + 1 : (W ? n - 1 : 0); }

// The in-domain coordinate that a coordinate outside [0, n) stands for: the
// wrapped one on a periodic axis, the nearest face on an absorbing one.
// Tiles and rings that reach past the domain compute such cells; on a
// periodic axis they are exactly the wrapped neighbours, on an absorbing
// axis their results are never used.
__device__ inline int fold(int x, int n, int W) {
    if (x >= 0 && x < n) return x;
    if (W) return x < 0 ? 0 : n - 1;
    x %= n;
    return x < 0 ? x + n : x;
}

// Element i of an array with a wave-uniform base.  The offset is formed in
// 32 bits (every plane is below 4 GiB, checked at create), which maps onto
// the scalar-base + 32-bit vector-offset form of the global memory
// instructions instead of per-lane 64-bit address arithmetic.
template <typename T>
__device__ inline T *at(T *base, uint32_t i) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T *>(reinterpret_cast<B *>(base) + (size_t)(i * (uint32_t)sizeof(T)));
}

// ---------------------------------------------------------------------------
// Vector loads/stores: each thread updates VX consecutive x-cells.  Aligned
// accesses use VX*sizeof(T)-aligned vectors; the +-x pulls are the same
// vectors shifted by one element (only element alignment), which gfx950
// serves with a single dwordx4 / dwordx2 access.
// ---------------------------------------------------------------------------
template <typename T, int N> struct Vec;
template <> struct Vec<float, 4> {
    typedef float u __attribute__((ext_vector_type(4), aligned(4)));
    typedef float a __attribute__((ext_vector_type(4), aligned(16)));
};
template <> struct Vec<float, 2> {
    typedef float u __attribute__((ext_vector_type(2), aligned(4)));
    typedef float a __attribute__((ext_vector_type(2), aligned(8)));
};
template <> struct Vec<double, 2> {
    typedef double u __attribute__((ext_vector_type(2), aligned(8)));
    typedef double a __attribute__((ext_vector_type(2), aligned(16)));
};

template <typename T, int N>
__device__ inline void load_shifted(T (&o)[N], const T *p) {
    if constexpr (N == 1) {
        o[0] = p[0];
    } else {
        typename Vec<T, N>::u v = *(const typename Vec<T, N>::u *)p;
#pragma unroll
        for (int k = 0; k < N; ++k) o[k] = v[k];
    }
}
template <typename T, int N>
__device__ inline void load_aligned(T (&o)[N], const T *p) {
    if constexpr (N == 1) {
        o[0] = p[0];
    } else {
        typename Vec<T, N>::a v = *(const typename Vec<T, N>::a *)p;
#pragma unroll
        for (int k = 0; k < N; ++k) o[k] = v[k];
    }
}
template <typename T, int N>
__device__ inline void store_aligned(T *p, const T (&i)[N]) {
    if constexpr (N == 1) {
        p[0] = i[0];
    } else {
        typename Vec<T, N>::a v;
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = i[k];
        *(typename Vec<T, N>::a *)p = v;
    }
}

template <typename T>
__device__ inline T sigma2d(const StepArgs<T> &a, int x, int y) {
    return fmax(sigma_axis<T>(x, a.nx, a.W[0], a.inv_w[0], a.sigma_max),
                sigma_axis<T>(y, a.ny, a.W[1], a.inv_w[1], a.sigma_max));
}

// ---------------------------------------------------------------------------
// 2-D per-cell update: moments, DFT sample, collision, layer/source blend.
// f holds the pulled populations on entry and f*(t) on exit; inv_eps = 1/eps
// and sig = sigma2d(x, y) come from the caller (the two-step kernel reuses
// them for the second step).  record: the cell is in the domain and owned by
// this thread, so it may add DFT samples and design-region history.
// ---------------------------------------------------------------------------
// PH: the cell's incident-wave phase factor (ur, ui) = e^{2 pi j u} was
// gathered by the caller (the two-step kernel prefetches it for the tiles
// that touch the layer), else it is gathered here.  MU: the cell has
// permeability mu (inv_mu = 1/mu).  LINE: background layer cells follow the
// exact incident line (see below).  LREC: this is the line's own update; it
// records the post-collision populations and the phasors of every cell.
// MODE (without MU / LINE / LREC, which keep collision then layer): 0 the
// plain collision where sig = 0 and the one-pass collision + layer where
// sig > 0; 1 the one-pass form for every cell (the caller's cells include
// layer cells; for sig = 0 it reproduces the plain collision bit for bit);
// 2 the plain collision only (the caller guarantees sig = 0).
template <typename T, int POL, bool HIST = false, bool PH = false, bool MU = false, bool LINE = false,
          bool LREC = false, int MODE = 0>
__device__ inline void cell_update2d(const StepArgs<T> &a, const StepConst<T> &st, int x, int y, T eps,
                                     T inv_eps, T sig, T f[11], bool record, T ur = T(0), T ui = T(0),
                                     T mu = T(1), T inv_mu = T(1), const T *fl = nullptr, int fl_stride = 0) {
    const int64_t t = st.t;
    T F[3];
    fields2d<T, POL, MU>(f, eps, inv_eps, F, mu, inv_mu);
    if (LREC) {
        if (st.dft && record) {
            // line phasors, one node per line cell, same transform as the contour's
            double *p = a.line_acc + (int64_t)(a.line_axis == 0 ? x : y) * 12;
            const int c0 = POL == TM ? 2 : 0, c1 = POL == TM ? 3 : 1, c2 = POL == TM ? 4 : 5;
            p[2 * c0] += (double)F[0] * st.cr;
            p[2 * c0 + 1] += (double)F[0] * st.ci;
            p[2 * c1] += (double)F[1] * st.cr;
            p[2 * c1 + 1] += (double)F[1] * st.ci;
            p[2 * c2] += (double)F[2] * st.cr;
            p[2 * c2 + 1] += (double)F[2] * st.ci;
        }
    } else if (st.dft && record) {
        double G[6] = {0, 0, 0, 0, 0, 0};
        if (POL == TM) {
            G[2] = F[0]; G[3] = F[1]; G[4] = F[2];
            dft_accumulate<0x1c>(a, st, 2, x, y, 0, G);
        } else {
            G[0] = F[0]; G[1] = F[1]; G[5] = F[2];
            dft_accumulate<0x23>(a, st, 2, x, y, 0, G);
        }
    }
    if (HIST && record && x >= a.dlo[0] && x <= a.dhi[0] && y >= a.dlo[1] && y <= a.dhi[1]) {
        // E = (sum of the E-carrying populations + (6 eps - 4) z-pair)/eps,
        // so dE/deps = (6 zpair - E)/eps at fixed populations
        const int64_t dw = a.dhi[0] - a.dlo[0] + 1, dh = a.dhi[1] - a.dlo[1] + 1;
        const int64_t cell = (int64_t)(y - a.dlo[1]) * dw + (x - a.dlo[0]);
        T *h = a.hist + (t - a.hist_t0) * dw * dh * (POL == TM ? 1 : 2);
        if (POL == TM) h[cell] = (T(6) * f[8] - F[0]) * inv_eps;
        else {
            h[2 * cell] = (T(6) * f[8] - F[0]) * inv_eps;
            h[2 * cell + 1] = (T(6) * f[9] - F[1]) * inv_eps;
        }
    }
    if (!LINE && !LREC && !MU) {
        // Collision and layer in one pass: with f* = 2 f^eq(F) - f and
        // f' = f* + sig (f^eq(R) - f*), linearity of f^eq gives
        // f' = f^eq(G) - s f, G = 2F + sig (R - 2F), s = 1 - sig: the plain
        // collision's combinations of G/6 with -s f fused in, which for
        // sig = 0 (G = 2F exactly, s = 1, sixth(2x) == third(x), fma(-1, f,
        // q) == q - f) is the plain collision bit for bit.
        if (MODE == 2 || (MODE == 0 && !(sig > T(0)))) {
            collide2d<T, POL>(F, f);
            return;
        }
        T R[3] = {0, 0, 0};
        if (a.src_on && eps == T(1) && (!MU || mu == T(1))) {
            const T w = PH ? st.gs * ur - st.gc * ui : plane_wave<T, 2>(a, st, x, y, 0);
            if (POL == TM) { R[0] = w * a.ehat[2]; R[1] = w * a.hhat[0]; R[2] = w * a.hhat[1]; }
            else { R[0] = w * a.ehat[0]; R[1] = w * a.ehat[1]; R[2] = w * a.hhat[2]; }
        }
        T G[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T F2 = F[k] + F[k];
            G[k] = fma(sig, R[k] - F2, F2);
        }
        const T sc = T(1) - sig;
        const T g0 = sixth(G[0]), g1 = sixth(G[1]), g2 = sixth(G[2]);
        T q[11];
        if (POL == TM) {
            const T ez = g0, hx = g1, hy = g2;
            q[0] = ez - hy; q[1] = ez + hy; q[2] = ez + hx; q[3] = ez - hx;
            q[4] = q[5] = q[9] = hx;
            q[6] = q[7] = q[10] = hy;
            q[8] = ez;
        } else {
            const T ex = g0, ey = g1, hz = g2;
            q[0] = q[1] = q[8] = ex;
            q[2] = ex - hz; q[3] = ex + hz; q[4] = ey + hz; q[5] = ey - hz;
            q[6] = q[7] = q[9] = ey;
            q[10] = hz;
        }
#pragma unroll
        for (int i = 0; i < 11; ++i) f[i] = fma(-sc, f[i], q[i]);
        return;
    }
    collide2d<T, POL>(F, f);
    if (LREC) {
        T *r = a.line_rec + (int64_t)(t & (kLineSlots - 1)) * 11 * a.line_n + (a.line_axis == 0 ? x : y);
#pragma unroll
        for (int i = 0; i < 11; ++i) r[(int64_t)i * a.line_n] = f[i];
    }
    if (sig > T(0)) {
        // relax towards the incident wave's equilibrium (zero where eps != 1
        // or mu != 1, which includes a conductor's mu == 0): f + sig (f_ref - f),
        // one fused multiply-add per population
        T R[3] = {0, 0, 0};
        const bool background = a.src_on && eps == T(1) && (!MU || mu == T(1));
        if (background) {
            const T w = PH ? st.gs * ur - st.gc * ui : plane_wave<T, 2>(a, st, x, y, 0);
            if (POL == TM) { R[0] = w * a.ehat[2]; R[1] = w * a.hhat[0]; R[2] = w * a.hhat[1]; }
            else { R[0] = w * a.ehat[0]; R[1] = w * a.ehat[1]; R[2] = w * a.hhat[2]; }
        }
        T qr[11];
        equilibrium2d<T, POL>(R, T(1), qr);
        if (LINE && background) {
            // exact incident line: damp the scattered part f - f_l towards
            // zero and add the line's own relaxation, f_l + sig_a (f_ref - f_l)
            // with sig_a its layer strength here; where f == f_l this is
            // the line's update operation for operation.  fl: the line's
            // post-collision populations of this step at this coordinate
            // (plane i at fl[i * fl_stride]).
            const int ax = a.line_axis, u = ax == 0 ? x : y;
            const T sa = sigma_axis<T>(u, ax == 0 ? a.nx : a.ny, a.W[ax], a.inv_w[ax], a.sigma_max);
#pragma unroll
            for (int i = 0; i < 11; ++i) {
                const T l = fl[i * fl_stride];
                f[i] = fma(sa, qr[i] - l, fma(sig, l - f[i], f[i]));
            }
        } else {
#pragma unroll
            for (int i = 0; i < 11; ++i) f[i] = fma(sig, qr[i] - f[i], f[i]);
        }
    }
}

// Pulled populations and eps of the VX cells x0 .. x0+VX-1 of row y
// (0 <= y < ny, x0 a multiple of VX; cells outside [0, nx) are folded).
template <typename T, int VX>
__device__ inline void pull_row(const StepArgs<T> &a, int x0, int y, T (&v)[11][VX], T (&e)[VX]) {
    const int64_t P = a.plane;
    const T *s = a.src;
    const uint32_t sy = (uint32_t)a.sy;
    const uint32_t row = (uint32_t)y * sy;
    const uint32_t rm = (uint32_t)pull_lo(y, a.ny, a.W[1]) * sy;
    const uint32_t rp = (uint32_t)pull_hi(y, a.ny, a.W[1]) * sy;
    if (x0 > 0 && x0 + VX < a.nx) {
        const uint32_t c = row + (uint32_t)x0;
        load_shifted<T, VX>(v[0], at(s + 0 * P, c - 1));   // +x movers from x-1
        load_shifted<T, VX>(v[4], at(s + 4 * P, c - 1));
        load_shifted<T, VX>(v[1], at(s + 1 * P, c + 1));   // -x movers from x+1
        load_shifted<T, VX>(v[5], at(s + 5 * P, c + 1));
    } else {
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const int x = fold(x0 + k, a.nx, a.W[0]);
            const uint32_t cm = row + (uint32_t)pull_lo(x, a.nx, a.W[0]);
            const uint32_t cp = row + (uint32_t)pull_hi(x, a.nx, a.W[0]);
            v[0][k] = *at(s + 0 * P, cm);
            v[4][k] = *at(s + 4 * P, cm);
            v[1][k] = *at(s + 1 * P, cp);
            v[5][k] = *at(s + 5 * P, cp);
        }
    }
    if (x0 >= 0 && x0 + VX <= a.nx) {
        const uint32_t c = (uint32_t)x0;
        load_aligned<T, VX>(v[2], at(s + 2 * P, rm + c));   // +y movers from y-1
        load_aligned<T, VX>(v[6], at(s + 6 * P, rm + c));
        load_aligned<T, VX>(v[3], at(s + 3 * P, rp + c));   // -y movers from y+1
        load_aligned<T, VX>(v[7], at(s + 7 * P, rp + c));
        load_aligned<T, VX>(v[8], at(s + 8 * P, row + c));  // z-pair: no move
        load_aligned<T, VX>(v[9], at(s + 9 * P, row + c));
        load_aligned<T, VX>(v[10], at(s + 10 * P, row + c));
        load_aligned<T, VX>(e, at(a.eps, row + c));
    } else {
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const uint32_t c = (uint32_t)fold(x0 + k, a.nx, a.W[0]);
            v[2][k] = *at(s + 2 * P, rm + c);
            v[6][k] = *at(s + 6 * P, rm + c);
            v[3][k] = *at(s + 3 * P, rp + c);
            v[7][k] = *at(s + 7 * P, rp + c);
            v[8][k] = *at(s + 8 * P, row + c);
            v[9][k] = *at(s + 9 * P, row + c);
            v[10][k] = *at(s + 10 * P, row + c);
            e[k] = *at(a.eps, row + c);
        }
    }
}

// Store the cells x0 .. x0+VX-1 of row y that lie in the domain.
template <typename T, int VX>
__device__ inline void store_row(const StepArgs<T> &a, int x0, int y, const T (&v)[11][VX]) {
    const int64_t P = a.plane;
    T *d = a.dst;
    const uint32_t c = (uint32_t)y * (uint32_t)a.sy + (uint32_t)x0;
    if (x0 + VX <= a.nx) {
#pragma unroll
        for (int i = 0; i < 11; ++i) store_aligned<T, VX>(at(d + i * P, c), v[i]);
    } else {
#pragma unroll
        for (int k = 0; k < VX; ++k)
            if (x0 + k < a.nx)
#pragma unroll
                for (int i = 0; i < 11; ++i) *at(d + i * P, c + k) = v[i][k];
    }
}

// ---------------------------------------------------------------------------
// 2-D fused step: pull + moments + DFT + collision + layer/source + store.
// The calling thread updates cells x0 .. x0+VX-1 of row y.
// ---------------------------------------------------------------------------
// MU: the permeability variant (a.mu is read per cell).  LINE / LREC: see
// cell_update2d.
template <typename T, int POL, int VX, bool HIST = false, bool MU = false, bool LINE = false, bool LREC = false>
__device__ inline void step2d_cells(const StepArgs<T> &a, int x0, int y, const StepConst<T> &st) {
    if (x0 >= a.nx || y >= a.ny) return;
    T v[11][VX], e[VX], m[VX];
    pull_row<T, VX>(a, x0, y, v, e);
    if (MU) {
        const uint32_t row = (uint32_t)y * (uint32_t)a.sy;
        if (x0 >= 0 && x0 + VX <= a.nx) load_aligned<T, VX>(m, at(a.mu, row + (uint32_t)x0));
        else
#pragma unroll
            for (int k = 0; k < VX; ++k) m[k] = *at(a.mu, row + (uint32_t)fold(x0 + k, a.nx, a.W[0]));
    }
#pragma unroll
    for (int k = 0; k < VX; ++k) {
        const int x = fold(x0 + k, a.nx, a.W[0]);
        T f[11];
#pragma unroll
        for (int i = 0; i < 11; ++i) f[i] = v[i][k];
        const T *fl = nullptr;
        if (LINE) fl = a.line_tab + (int64_t)(st.t & (kLineSlots - 1)) * 11 * a.line_n + (a.line_axis == 0 ? x : y);
        if (MU)
            cell_update2d<T, POL, false, false, true, LINE, LREC>(a, st, x, y, e[k], recip(e[k]), sigma2d<T>(a, x, y),
                                                                  f, x0 + k < a.nx, T(0), T(0), m[k], recip(m[k]), fl,
                                                                  a.line_n);
        else
            cell_update2d<T, POL, HIST, false, false, LINE, LREC>(a, st, x, y, e[k], recip(e[k]), sigma2d<T>(a, x, y),
                                                                  f, x0 + k < a.nx, T(0), T(0), T(1), T(1), fl,
                                                                  a.line_n);
#pragma unroll
        for (int i = 0; i < 11; ++i) v[i][k] = f[i];
    }
    store_row<T, VX>(a, x0, y, v);
}

// HIST: also record dE/deps of the design cells into a.hist (checkpointed
// forward pass of the adjoint).  MU: permeability map a.mu (never with HIST).
// LINE: the layer follows the exact incident line a.line_tab.
template <typename T, int POL, int VX, bool HIST = false, bool MU = false, bool LINE = false>
__global__ void __launch_bounds__(256) k_step2d(StepArgs<T> a) {
    static_assert(!(HIST && (MU || LINE)), "the design-region history assumes mu_r = 1 and no line");
    const int x0 = (blockIdx.x * blockDim.x + threadIdx.x) * VX;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    step2d_cells<T, POL, VX, HIST, MU, LINE>(a, x0, y, step_const(a, step_time(a.t_base, a.t_off)));
}

// The exact incident line's own steps (one or two per launch, matching the
// grid's launch): a single block walks the line's cells with the grid's
// per-cell update, records each step's post-collision populations in slot
// t & 1 of a.line_rec for the grid's launch that follows, and accumulates
// the line's phasors.  a0 / a1: the arguments of the two steps (buffers
// swapped); a barrier separates them (one workgroup: its release/acquire
// at workgroup scope makes the first step's global writes visible).
template <typename T, int POL>
__global__ void __launch_bounds__(1024) k_line(StepArgs<T> a0, StepArgs<T> a1, int nsteps) {
    for (int s = 0; s < nsteps; ++s) {
        const StepArgs<T> &a = s == 0 ? a0 : a1;
        const StepConst<T> st = step_const(a, step_time(a.t_base, a.t_off));
        for (int u = threadIdx.x; u < a.line_n; u += blockDim.x) {
            if (a.line_axis == 0) step2d_cells<T, POL, 1, false, false, false, true>(a, u, 0, st);
            else step2d_cells<T, POL, 1, false, false, false, true>(a, 0, u, st);
        }
        if (s + 1 < nsteps) __syncthreads();   // a workgroup barrier orders the global writes too
    }
}

// The same line steps with the line's state held in LDS for a whole run of
// nsteps (up to one graph chunk): one block, at most 2 * 1024 cells; the
// state is read from a.src once and written to dst at the end (dst may be
// a.src).  Pulls follow the grid's rules: on the line axis from the
// neighbours (clamped on an absorbing axis, wrapped on a periodic one), the
// movers of the other axis (a single periodic cell) from the cell itself.
template <typename T, int POL>
__global__ void __launch_bounds__(1024) k_line_lds(StepArgs<T> a, T *dst, int nsteps) {
    extern __shared__ unsigned char line_raw[];
    T *S = reinterpret_cast<T *>(line_raw);     // 11 planes x n
    const int n = a.line_n, ax = a.line_axis, NT = blockDim.x, tid = threadIdx.x;
    const int64_t P = a.plane;
    const int64_t cstride = ax == 0 ? 1 : a.sy;  // the line's cells in its own layout
    const int Wl = a.W[ax];
    for (int k = tid; k < 11 * n; k += NT) S[k] = a.src[(k / n) * P + (k % n) * cstride];
    __syncthreads();
    const int64_t t0 = step_time(a.t_base, a.t_off);
    for (int s = 0; s < nsteps; ++s) {
        const StepConst<T> st = step_const(a, t0 + s);
        T out[2][11];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int u = tid + c * NT;
            if (u >= n) continue;
            const int lo = pull_lo(u, n, Wl), hi = pull_hi(u, n, Wl);
            T f[11];
#pragma unroll
            for (int i = 0; i < 11; ++i) f[i] = S[i * n + u];
            if (ax == 0) {            // +x movers from u - 1, -x movers from u + 1
                f[0] = S[0 * n + lo];
                f[4] = S[4 * n + lo];
                f[1] = S[1 * n + hi];
                f[5] = S[5 * n + hi];
            } else {                  // +y movers from u - 1, -y movers from u + 1
                f[2] = S[2 * n + lo];
                f[6] = S[6 * n + lo];
                f[3] = S[3 * n + hi];
                f[7] = S[7 * n + hi];
            }
            const int x = ax == 0 ? u : 0, y = ax == 0 ? 0 : u;
            cell_update2d<T, POL, false, false, false, false, true>(a, st, x, y, T(1), recip(T(1)),
                                                                    sigma2d<T>(a, x, y), f, true);
#pragma unroll
            for (int i = 0; i < 11; ++i) out[c][i] = f[i];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int u = tid + c * NT;
            if (u >= n) continue;
#pragma unroll
            for (int i = 0; i < 11; ++i) S[i * n + u] = out[c][i];
        }
        __syncthreads();
    }
    for (int k = tid; k < 11 * n; k += NT) dst[(k / n) * P + (k % n) * cstride] = S[k];
}


// Batched persistent step: one launch advances many 2-D instances of
// different sizes.  The work list is every (instance, tile) pair, tiles of
// bx*VX x by cells, instances one after another; a grid sized to the chip
// strides over it.  tile_first[i] is the first work item of instance i,
// tile_inst[w] the instance of work item w.  Per-instance arguments live in
// device memory; the step index is shared.
template <typename T, int POL, int VX>
__global__ void __launch_bounds__(256) k_step2d_batch(const StepArgs<T> *__restrict__ descs,
                                                      const int *__restrict__ tile_inst,
                                                      const int *__restrict__ tile_first, int ntiles,
                                                      const int64_t *t_base, int64_t t_off) {
    const int64_t t = step_time(t_base, t_off);
    for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
        const int inst = tile_inst[w];
        const StepArgs<T> &a = descs[inst];
        const int local = w - tile_first[inst];
        const int tx = local % a.tiles_x, ty = local / a.tiles_x;
        const int x0 = (tx * (int)blockDim.x + (int)threadIdx.x) * VX;
        const int y = ty * (int)blockDim.y + (int)threadIdx.y;
        step2d_cells<T, POL, VX>(a, x0, y, step_const(a, t));
    }
}

// ---------------------------------------------------------------------------
// Two time steps per launch (temporal blocking through LDS).
//
// A 256-thread block owns a TX x TY output tile, cut into 256 row segments
// of VX = 16 bytes / sizeof(T) cells, one per thread.  Step t runs on
// the tile's segments and on a one-cell ring around it, pulling from global
// memory exactly as the one-step kernel does.  Each moving population goes
// to LDS only where step t+1 will pull it from: the +x movers (planes 0, 4)
// of the tile and of the ring column on the left, the -x movers (1, 5) of
// the tile and the right ring column, the +y movers (2, 6) of the tile and
// the ring row above, the -y movers (3, 7) of the tile and the ring row
// below.  The non-moving z-pair, eps, 1/eps and the layer strength of a
// thread's own cells stay in its registers.  Step t+1 then pulls from LDS --
// the open-boundary clamp becomes "read your own value" on the domain faces
// -- and writes the tile.  Every cell goes through the same per-cell code as
// in the one-step kernel, so the result is bit-identical; ring cells never
// record DFT samples.  HBM traffic per two steps: the state is read once
// (plus the ring) and written once.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY>
struct alignas(16) X2Lds {
    static constexpr int VX = 16 / (int)sizeof(T);
    static constexpr int SX = TX + VX;   // padded row of the x-moving planes
    T xm[2][TY][SX];                     // planes 0, 4: tile column ox at VX + ox, left ring at VX - 1
    T xp[2][TY][SX];                     // planes 1, 5: tile column ox at ox, right ring at TX
    T ym[2][TY + 1][TX];                 // planes 2, 6: ring row above at 0, tile row oy at oy + 1
    T yp[2][TY + 1][TX];                 // planes 3, 7: tile row oy at oy, ring row below at TY
};

// One segment of VX cells per thread: blocks of (TX / VX) * TY threads,
// 256, 512 or 1024 (the larger tiles re-read a smaller halo fraction; the
// LDS tile grows with them, up to ~140 KB of the 160 KB of a CU).
template <typename T, int TX, int TY>
__host__ __device__ constexpr int x2_threads() {
    return (TX / (16 / (int)sizeof(T))) * TY;
}
template <typename T, int TX, int TY>
__host__ __device__ constexpr bool x2_tile_ok() {
    constexpr int VX = 16 / (int)sizeof(T), NT = x2_threads<T, TX, TY>();
    return TX % VX == 0 && (NT == 256 || NT == 512 || NT == 1024);
}

template <typename T, int N>
__device__ inline void lds_load(T (&o)[N], const T *p) { load_aligned<T, N>(o, p); }
template <typename T, int N>
__device__ inline void lds_store(T *p, const T (&i)[N]) { store_aligned<T, N>(p, i); }

// MU: permeability map a.mu (never with HIST); mu and 1/mu of the thread's
// own cells stay in registers like eps.  LINE: exact incident line.
// Line slab of the two-step kernel: the incident line's post-collision
// populations of steps t and t+1 at the tile's coordinates along the line
// (with the ring), staged in LDS by tiles that reach into the layer.
template <int TX, int TY>
__host__ __device__ constexpr int x2_line_n() { return (TX > TY ? TX : TY) + 2; }

// OWN: cell_update2d's MODE for the tile's own cells (1: the tile has layer
// cells, 2: it has none, 0: decide per cell); ring cells decide per cell.
// DFT = false: the launch lies outside the DFT window, and the contour
// accumulation is compiled out (it costs registers the plain steps do not
// need).
template <typename T, int POL, int TX, int TY, bool HIST = false, bool MU = false, bool LINE = false, int OWN = 0,
          bool DFT = true>
__device__ inline void step2d_x2_tile(const StepArgs<T> &a, X2Lds<T, TX, TY> &L, int x0, int y0, int64_t t,
                                      T *lslab = nullptr) {
    StepConst<T> s0, s1;   // formed once the own state's loads are issued
    constexpr int VX = X2Lds<T, TX, TY>::VX;
    constexpr int TPR = TX / VX;             // segments per tile row
    constexpr int NT = x2_threads<T, TX, TY>();
    constexpr int NR = 2 * TX + 2 * TY;      // ring cells
    static_assert(x2_tile_ok<T, TX, TY>(), "two-step tile shape");
    const int tid = threadIdx.x;
    const int sx = (tid % TPR) * VX, sy = tid / TPR;   // the thread's segment in the tile
    const int x = x0 + sx, y = y0 + sy;
    T zp[3][VX], ep[VX], ip[VX], sg[VX], mp[VX], imp[VX];

    // tiles that reach into the absorbing layer prefetch the incident-wave
    // phase factors of their cells with the state (block-uniform test)
    const bool layer_tile = a.src_on && ((a.W[0] && (x0 < a.W[0] || x0 + TX > a.nx - a.W[0])) ||
                                         (a.W[1] && (y0 < a.W[1] || y0 + TY > a.ny - a.W[1])));
    T ur[VX], ui[VX];
    // slab coordinates: entry j of a slab row is coordinate u0 + j on the line
    constexpr int NL = x2_line_n<TX, TY>();
    const int lu0 = (a.line_axis == 0 ? x0 : y0) - 1;

    // step t on the thread's own segment
    {
        const int yf = fold(y, a.ny, a.W[1]);
        T v[11][VX], e[VX];
        pull_row<T, VX>(a, x, yf, v, e);
        step_consts2(a, t, s0, s1);
        if (!DFT) s0.dft = s1.dft = false;
#pragma unroll
        for (int k = 0; k < VX; ++k) mp[k] = imp[k] = T(1);
        // tiles whose cells or ring cells reach into the layer stage the
        // line's populations of steps t and t+1 (after the own pulls were
        // issued, so their latencies overlap)
        const bool line_tile = a.src_on && ((a.W[0] && (x0 - 1 < a.W[0] || x0 + TX + 1 > a.nx - a.W[0])) ||
                                            (a.W[1] && (y0 - 1 < a.W[1] || y0 + TY + 1 > a.ny - a.W[1])));
        if (LINE && line_tile) {
            // a fixed number of loads per thread, all in flight before the
            // first LDS store (rows past the tile's extent along a y line
            // are loaded too, folded into the grid, and never read)
            const int ax = a.line_axis, na = a.line_n;
            constexpr int NLOAD = 2 * 11 * NL, J = (NLOAD + NT - 1) / NT;
            T lv[J];
#pragma unroll
            for (int q = 0; q < J; ++q) {
                const int k = tid + q * NT;
                if (k < NLOAD) {
                    const int j = k % NL, r = k / NL;       // r = step (0, 1) * 11 + plane
                    const int u = fold(lu0 + j, na, a.W[ax]);
                    lv[q] = a.line_tab[((int64_t)((t + r / 11) & (kLineSlots - 1)) * 11 + r % 11) * na + u];
                }
            }
#pragma unroll
            for (int q = 0; q < J; ++q) {
                const int k = tid + q * NT;
                if (k < NLOAD) lslab[k] = lv[q];
            }
            __syncthreads();
        }
        if (MU) {
            const uint32_t row = (uint32_t)yf * (uint32_t)a.sy;
            if (x >= 0 && x + VX <= a.nx) load_aligned<T, VX>(mp, at(a.mu, row + (uint32_t)x));
            else
#pragma unroll
                for (int k = 0; k < VX; ++k) mp[k] = *at(a.mu, row + (uint32_t)fold(x + k, a.nx, a.W[0]));
#pragma unroll
            for (int k = 0; k < VX; ++k) imp[k] = recip(mp[k]);
        }
#pragma unroll
        for (int k = 0; k < VX; ++k) ur[k] = ui[k] = T(0);
        if (layer_tile) {
            const auto py = a.wave_y[yf];
#pragma unroll
            for (int k = 0; k < VX; ++k) {
                const auto px = a.wave_x[fold(x + k, a.nx, a.W[0])];
                ur[k] = px.x * py.x - px.y * py.y;
                ui[k] = px.x * py.y + px.y * py.x;
            }
        }
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const int xf = fold(x + k, a.nx, a.W[0]);
            ep[k] = e[k];
            ip[k] = recip(e[k]);
            sg[k] = sigma2d<T>(a, xf, yf);
            T f[11];
#pragma unroll
            for (int i = 0; i < 11; ++i) f[i] = v[i][k];
            cell_update2d<T, POL, HIST, true, MU, LINE, false, OWN>(a, s0, xf, yf, e[k], ip[k], sg[k], f,
                                                                    x + k < a.nx && y < a.ny, ur[k], ui[k], mp[k],
                                                                    imp[k], lslab + ((a.line_axis == 0 ? x + k : y) - lu0),
                                                                    NL);
#pragma unroll
            for (int i = 0; i < 11; ++i) v[i][k] = f[i];
            zp[0][k] = f[8];
            zp[1][k] = f[9];
            zp[2][k] = f[10];
        }
        lds_store<T, VX>(&L.xm[0][sy][VX + sx], v[0]);
        lds_store<T, VX>(&L.xm[1][sy][VX + sx], v[4]);
        lds_store<T, VX>(&L.xp[0][sy][sx], v[1]);
        lds_store<T, VX>(&L.xp[1][sy][sx], v[5]);
        lds_store<T, VX>(&L.ym[0][sy + 1][sx], v[2]);
        lds_store<T, VX>(&L.ym[1][sy + 1][sx], v[6]);
        lds_store<T, VX>(&L.yp[0][sy][sx], v[3]);
        lds_store<T, VX>(&L.yp[1][sy][sx], v[7]);
    }
    // step t on the ring, one cell per thread: the rows above and below the
    // tile and the columns to its left and right (no corners: nothing pulls
    // from them)
    for (int r = tid; r < NR; r += NT) {
        int rx, ry;
        if (r < TX) { rx = x0 + r; ry = y0 - 1; }
        else if (r < 2 * TX) { rx = x0 + (r - TX); ry = y0 + TY; }
        else if (r < 2 * TX + TY) { rx = x0 - 1; ry = y0 + (r - 2 * TX); }
        else { rx = x0 + TX; ry = y0 + (r - 2 * TX - TY); }
        const int xf = fold(rx, a.nx, a.W[0]), yf = fold(ry, a.ny, a.W[1]);
        T v[11][1], e[1];
        pull_row<T, 1>(a, xf, yf, v, e);
        T f[11];
#pragma unroll
        for (int i = 0; i < 11; ++i) f[i] = v[i][0];
        if (MU) {
            const T m = *at(a.mu, (uint32_t)yf * (uint32_t)a.sy + (uint32_t)xf);
            cell_update2d<T, POL, false, false, true, LINE>(a, s0, xf, yf, e[0], recip(e[0]), sigma2d<T>(a, xf, yf),
                                                            f, false, T(0), T(0), m, recip(m),
                                                            lslab + ((a.line_axis == 0 ? rx : ry) - lu0), NL);
        } else {
            cell_update2d<T, POL, false, false, false, LINE>(a, s0, xf, yf, e[0], recip(e[0]), sigma2d<T>(a, xf, yf),
                                                             f, false, T(0), T(0), T(1), T(1),
                                                             lslab + ((a.line_axis == 0 ? rx : ry) - lu0), NL);
        }
        if (r < TX) {
            L.ym[0][0][r] = f[2];
            L.ym[1][0][r] = f[6];
        } else if (r < 2 * TX) {
            L.yp[0][TY][r - TX] = f[3];
            L.yp[1][TY][r - TX] = f[7];
        } else if (r < 2 * TX + TY) {
            L.xm[0][ry - y0][VX - 1] = f[0];
            L.xm[1][ry - y0][VX - 1] = f[4];
        } else {
            L.xp[0][ry - y0][TX] = f[1];
            L.xp[1][ry - y0][TX] = f[5];
        }
    }
    __syncthreads();

    // step t+1 on the thread's own segment
    if (x >= a.nx || y >= a.ny) return;
    {
        T v[11][VX];
        {   // +x movers from the left neighbour (own value on an absorbing left face)
            T o0[VX], o4[VX];
            lds_load<T, VX>(o0, &L.xm[0][sy][VX + sx]);
            lds_load<T, VX>(o4, &L.xm[1][sy][VX + sx]);
            const bool clamp = a.W[0] && x == 0;
            v[0][0] = clamp ? o0[0] : L.xm[0][sy][VX + sx - 1];
            v[4][0] = clamp ? o4[0] : L.xm[1][sy][VX + sx - 1];
#pragma unroll
            for (int k = 1; k < VX; ++k) {
                v[0][k] = o0[k - 1];
                v[4][k] = o4[k - 1];
            }
        }
        {   // -x movers from the right neighbour (own value on an absorbing right face)
            T o1[VX], o5[VX];
            lds_load<T, VX>(o1, &L.xp[0][sy][sx]);
            lds_load<T, VX>(o5, &L.xp[1][sy][sx]);
            const T n1 = L.xp[0][sy][sx + VX], n5 = L.xp[1][sy][sx + VX];
#pragma unroll
            for (int k = 0; k < VX; ++k) {
                const bool clamp = a.W[0] && x + k == a.nx - 1;
                v[1][k] = clamp ? o1[k] : (k + 1 < VX ? o1[(k + 1) % VX] : n1);
                v[5][k] = clamp ? o5[k] : (k + 1 < VX ? o5[(k + 1) % VX] : n5);
            }
        }
        {   // +y movers from the row above, -y movers from the row below
            const int rm = (a.W[1] && y == 0) ? sy + 1 : sy;
            const int rp = (a.W[1] && y == a.ny - 1) ? sy : sy + 1;
            lds_load<T, VX>(v[2], &L.ym[0][rm][sx]);
            lds_load<T, VX>(v[6], &L.ym[1][rm][sx]);
            lds_load<T, VX>(v[3], &L.yp[0][rp][sx]);
            lds_load<T, VX>(v[7], &L.yp[1][rp][sx]);
        }
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const int xf = fold(x + k, a.nx, a.W[0]);
            T f[11];
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = v[i][k];
            f[8] = zp[0][k];
            f[9] = zp[1][k];
            f[10] = zp[2][k];
            cell_update2d<T, POL, HIST, true, MU, LINE, false, OWN>(a, s1, xf, y, ep[k], ip[k], sg[k], f, x + k < a.nx,
                                                                    ur[k], ui[k], mp[k], imp[k],
                                                                    lslab + 11 * NL + ((a.line_axis == 0 ? x + k : y) - lu0),
                                                                    NL);
#pragma unroll
            for (int i = 0; i < 11; ++i) v[i][k] = f[i];
        }
        store_row<T, VX>(a, x, y, v);
    }
}

// XCD-aware tile order.  The work-groups of a launch are dealt round-robin
// to the 8 XCDs, each with its own L2: block b runs on XCD b mod 8.  Giving
// every XCD one contiguous band of row-major tiles keeps a tile and the
// neighbours whose edge rows and columns it re-reads in the same L2.
__device__ inline int xcd_tile(int b, int ntiles) {
    constexpr int NXCD = 8;
    const int xcd = b % NXCD, j = b / NXCD;
    const int q = ntiles / NXCD, r = ntiles % NXCD;
    return xcd * q + (xcd < r ? xcd : r) + j;
}

// One block per tile, a 1-D grid of tiles_x * tiles_y blocks.  The launch
// bound asks for 4 waves per SIMD (at most 128 VGPRs).
// HIST: also record dE/deps of the design cells (recompute of the adjoint).
// MU: permeability map a.mu.  LINE: exact incident line.  DFT: the launch
// may meet the DFT window.
template <typename T, int POL, int TX, int TY, bool HIST = false, bool MU = false, bool LINE = false, bool DFT = true>
__global__ void __launch_bounds__((x2_threads<T, TX, TY>()), (1024 / x2_threads<T, TX, TY>()))
    k_step2d_x2(StepArgs<T> a) {
    static_assert(!(HIST && (MU || LINE)), "the design-region history assumes mu_r = 1 and no line");
    __shared__ X2Lds<T, TX, TY> lds;
    __shared__ T lslab[LINE ? 2 * 11 * x2_line_n<TX, TY>() : 1];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % a.tiles_x) * TX, y0 = (tile / a.tiles_x) * TY;
    const int64_t t = step_time(a.t_base, a.t_off);
    // tiles with layer cells take the one-pass collision + layer for every
    // own cell, the others the plain collision (block-uniform choice)
    const bool in_layer = (a.W[0] && (x0 < a.W[0] || x0 + TX > a.nx - a.W[0])) ||
                          (a.W[1] && (y0 < a.W[1] || y0 + TY > a.ny - a.W[1]));
    if (in_layer) step2d_x2_tile<T, POL, TX, TY, HIST, MU, LINE, 1, DFT>(a, lds, x0, y0, t, lslab);
    else step2d_x2_tile<T, POL, TX, TY, HIST, MU, LINE, 2, DFT>(a, lds, x0, y0, t, lslab);
}

// One step on the two-step kernel's tiles (batched; a trailing odd step).
template <typename T, int POL, int TX, int TY>
__global__ void __launch_bounds__((x2_threads<T, TX, TY>())) k_step2d_tile_batch(const StepArgs<T> *__restrict__ descs,
                                                           const int *__restrict__ tile_inst,
                                                           const int *__restrict__ tile_first, int ntiles,
                                                           const int64_t *t_base, int64_t t_off) {
    constexpr int VX = X2Lds<T, TX, TY>::VX, TPR = TX / VX;
    const int64_t t = step_time(t_base, t_off);
    for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
        const int inst = tile_inst[w];
        const StepArgs<T> &a = descs[inst];
        const int local = w - tile_first[inst];
        const int x0 = (local % a.tiles_x) * TX, y0 = (local / a.tiles_x) * TY;
        const StepConst<T> st = step_const(a, t);
        for (int seg = threadIdx.x; seg < TPR * TY; seg += blockDim.x)
            step2d_cells<T, POL, VX>(a, x0 + (seg % TPR) * VX, y0 + seg / TPR, st);
    }
}

// Batched form of the two-step kernel: a chip-sized grid strides over the
// (instance, tile) work list (tiles of TX x TY cells); a barrier separates
// consecutive tiles of a block because they share the LDS tile.  DFT: the
// launch may meet the DFT window of an instance.
template <typename T, int POL, int TX, int TY, bool DFT = true>
__global__ void __launch_bounds__((x2_threads<T, TX, TY>()), (1024 / x2_threads<T, TX, TY>()))
    k_step2d_x2_batch(const StepArgs<T> *__restrict__ descs,
                                                         const int *__restrict__ tile_inst,
                                                         const int *__restrict__ tile_first, int ntiles,
                                                         const int64_t *t_base, int64_t t_off) {
    __shared__ X2Lds<T, TX, TY> lds;
    const int64_t t = step_time(t_base, t_off);
    for (int w0 = blockIdx.x; w0 < ntiles; w0 += gridDim.x) {
        // one block per work item: XCD-banded order as in k_step2d_x2
        const int w = (int)gridDim.x == ntiles ? xcd_tile(w0, ntiles) : w0;
        const int inst = tile_inst[w];
        const StepArgs<T> &a = descs[inst];
        const int local = w - tile_first[inst];
        const int x0 = (local % a.tiles_x) * TX, y0 = (local / a.tiles_x) * TY;
        const bool in_layer = (a.W[0] && (x0 < a.W[0] || x0 + TX > a.nx - a.W[0])) ||
                              (a.W[1] && (y0 < a.W[1] || y0 + TY > a.ny - a.W[1]));
        if (in_layer) step2d_x2_tile<T, POL, TX, TY, false, false, false, 1, DFT>(a, lds, x0, y0, t);
        else step2d_x2_tile<T, POL, TX, TY, false, false, false, 2, DFT>(a, lds, x0, y0, t);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 3-D fused step (27 scalars)
// ---------------------------------------------------------------------------
__device__ constexpr int C3[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

template <typename T>
__device__ inline void cross3(const T a[3], const T b[3], T o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T>
__device__ inline void fields3d(const T f[27], T inv_eps, T E[3], T H[3]) {
    T D[3] = {f[24], f[25], f[26]}, B[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const T *e = f + 4 * d;
        const T eta = f[4 * d + 3];
        T cv[3] = {T(C3[d][0]), T(C3[d][1]), T(C3[d][2])}, cxe[3];
        cross3(cv, e, cxe);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            D[k] += e[k];
            B[k] += eta * cv[k] + cxe[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        E[k] = D[k] * inv_eps;
        H[k] = B[k];
    }
}

template <typename T>
__device__ inline void equilibrium3d(const T E[3], const T H[3], T eps, T scale, T q[27]) {
    const T c = scale / T(6);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        T cv[3] = {T(C3[d][0]), T(C3[d][1]), T(C3[d][2])}, cxh[3];
        cross3(cv, H, cxh);
#pragma unroll
        for (int k = 0; k < 3; ++k) q[4 * d + k] = c * (E[k] - cxh[k]);
        q[4 * d + 3] = c * (cv[0] * H[0] + cv[1] * H[1] + cv[2] * H[2]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) q[24 + k] = scale * (eps - T(1)) * E[k];
}

template <typename T>
__device__ inline T sigma3d(const StepArgs<T> &a, int x, int y, int z) {
    return fmax(fmax(sigma_axis<T>(x, a.nx, a.W[0], a.inv_w[0], a.sigma_max),
                     sigma_axis<T>(y, a.ny, a.W[1], a.inv_w[1], a.sigma_max)),
                sigma_axis<T>(z, a.nz, a.W[2], a.inv_w[2], a.sigma_max));
}

// 3-D per-cell update (moments, DFT sample, collision, layer/source);
// inv_eps = 1/eps and sig = sigma3d(x, y, z) from the caller; record: the
// cell is in the domain and owned by this thread (DFT samples).
// PH: the caller passes the cell's x-y phase factor wxy = xy_phase(x, y) and
// its plane's z factor wz = wave_z[z] (the same value as from the tables).
template <typename T, bool LINE = false, bool LREC = false, bool DFT = true, bool PH = false>
__device__ inline void cell_update3d(const StepArgs<T> &a, const StepConst<T> &st, int x, int y, int z, T eps,
                                     T inv_eps, T sig, T f[27], bool record, const T *fl = nullptr,
                                     int fl_stride = 0, typename Cplx<T>::type wxy = {},
                                     typename Cplx<T>::type wz = {}) {
    T E[3], H[3];
    fields3d(f, inv_eps, E, H);
    if (LREC) {
        if (st.dft && record) {
            // line phasors, one node per line cell
            double *pa = a.line_acc + (int64_t)(a.line_axis == 0 ? x : a.line_axis == 1 ? y : z) * 12;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pa[2 * c] += (double)E[c] * st.cr;
                pa[2 * c + 1] += (double)E[c] * st.ci;
                pa[6 + 2 * c] += (double)H[c] * st.cr;
                pa[6 + 2 * c + 1] += (double)H[c] * st.ci;
            }
        }
    } else if (DFT && st.dft && record) {
        const double G[6] = {E[0], E[1], E[2], H[0], H[1], H[2]};
        dft_accumulate<0x3f>(a, st, 3, x, y, z, G);
    }
    if (!LINE && !LREC && sig > T(0)) {
        // layer cell: collision and relaxation towards the incident
        // equilibrium in one pass.  Both are linear in (E, H), so
        //   f' = (1 - sig)(2 f^eq(E, H) - f) + sig f^eq(E_ref, H_ref)
        //      = f^eq(G_E, G_H) - (1 - sig) f,   G = 2 F + sig (F_ref - 2 F),
        // one fused multiply-add per population and no second equilibrium
        // held in registers
        T Er[3] = {0, 0, 0}, Hr[3] = {0, 0, 0};
        if (a.src_on && eps == T(1)) {
            const T w = PH ? plane_wave_xyz(st, wxy, wz) : plane_wave<T, 3>(a, st, x, y, z);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Er[k] = w * a.ehat[k];
                Hr[k] = w * a.hhat[k];
            }
        }
        T GE[3], GH[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T E2 = E[k] + E[k], H2 = H[k] + H[k];
            GE[k] = fma(sig, Er[k] - E2, E2);
            GH[k] = fma(sig, Hr[k] - H2, H2);
        }
        const T sc = T(1) - sig, r = eps - T(1);
        const T GE6[3] = {sixth(GE[0]), sixth(GE[1]), sixth(GE[2])};
        const T GH6[3] = {sixth(GH[0]), sixth(GH[1]), sixth(GH[2])};
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const T cv[3] = {T(C3[d][0]), T(C3[d][1]), T(C3[d][2])};
            T cxh[3];
            cross3(cv, GH6, cxh);     // exact: permuted, signed components
#pragma unroll
            for (int k = 0; k < 3; ++k) f[4 * d + k] = fma(-sc, f[4 * d + k], GE6[k] - cxh[k]);
            f[4 * d + 3] = fma(-sc, f[4 * d + 3], cv[0] * GH6[0] + cv[1] * GH6[1] + cv[2] * GH6[2]);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) f[24 + k] = fma(r, GE[k], -(sc * f[24 + k]));
        return;
    }
    // collision f <- 2 f^eq - f, every population a combination of E/3 and
    // H/3 (each rounded correctly by third()) minus f
    {
        const T r = T(2) * (eps - T(1));
        const T E3[3] = {third(E[0]), third(E[1]), third(E[2])};
        const T H3[3] = {third(H[0]), third(H[1]), third(H[2])};
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const T cv[3] = {T(C3[d][0]), T(C3[d][1]), T(C3[d][2])};
            T cxh[3];
            cross3(cv, H3, cxh);      // exact: permuted, signed components
#pragma unroll
            for (int k = 0; k < 3; ++k) f[4 * d + k] = (E3[k] - cxh[k]) - f[4 * d + k];
            f[4 * d + 3] = (cv[0] * H3[0] + cv[1] * H3[1] + cv[2] * H3[2]) - f[4 * d + 3];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) f[24 + k] = fma(r, E[k], -f[24 + k]);
    }
    if (LREC) {
        T *rp = a.line_rec + (int64_t)(st.t & (kLineSlots - 1)) * 27 * a.line_n +
                (a.line_axis == 0 ? x : a.line_axis == 1 ? y : z);
#pragma unroll
        for (int i = 0; i < 27; ++i) rp[(int64_t)i * a.line_n] = f[i];
    }
    if (sig > T(0)) {
        T Er[3] = {0, 0, 0}, Hr[3] = {0, 0, 0};
        const bool background = a.src_on && eps == T(1);
        if (background) {
            const T w = PH ? plane_wave_xyz(st, wxy, wz) : plane_wave<T, 3>(a, st, x, y, z);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Er[k] = w * a.ehat[k];
                Hr[k] = w * a.hhat[k];
            }
        }
        T qr[27];
        equilibrium3d(Er, Hr, eps, T(1), qr);
        if (LINE && background) {
            // exact incident line (see cell_update2d); fl: the line's
            // post-collision populations of this step at this coordinate
            const int ax = a.line_axis, u = ax == 0 ? x : ax == 1 ? y : z;
            const int nax = ax == 0 ? a.nx : ax == 1 ? a.ny : a.nz;
            const T sa = sigma_axis<T>(u, nax, a.W[ax], a.inv_w[ax], a.sigma_max);
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                const T l = fl[i * fl_stride];
                f[i] = fma(sa, qr[i] - l, fma(sig, l - f[i], f[i]));
            }
        } else {
#pragma unroll
            for (int i = 0; i < 27; ++i) f[i] = fma(sig, qr[i] - f[i], f[i]);
        }
    }
}

// Pulled populations and eps of the in-domain cell (x, y, z): direction d
// (planes 4d .. 4d+3) from r - c_d with the open-boundary clamp or wrap.
// vac: the cell is vacuum with zero rest populations (eps_r = 1 and e_0 = 0
// exactly; see vacuum_plane), so neither is read.
template <typename T>
__device__ inline void pull3d(const StepArgs<T> &a, int x, int y, int z, T f[27], T &e, bool vac = false) {
    const int64_t P = a.plane;
    const T *s = a.src;
    const uint32_t sy = (uint32_t)a.sy, sz = (uint32_t)a.sz;
    const uint32_t zo = (uint32_t)z * sz, yo = (uint32_t)y * sy;
    const uint32_t c = zo + yo + (uint32_t)x;
    const uint32_t src[6] = {zo + yo + (uint32_t)pull_lo(x, a.nx, a.W[0]), zo + yo + (uint32_t)pull_hi(x, a.nx, a.W[0]),
                             zo + (uint32_t)pull_lo(y, a.ny, a.W[1]) * sy + (uint32_t)x,
                             zo + (uint32_t)pull_hi(y, a.ny, a.W[1]) * sy + (uint32_t)x,
                             (uint32_t)pull_lo(z, a.nz, a.W[2]) * sz + yo + (uint32_t)x,
                             (uint32_t)pull_hi(z, a.nz, a.W[2]) * sz + yo + (uint32_t)x};
#pragma unroll
    for (int d = 0; d < 6; ++d)
#pragma unroll
        for (int k = 0; k < 4; ++k) f[4 * d + k] = *at(s + (4 * d + k) * P, src[d]);
    if (vac) {
        f[24] = f[25] = f[26] = T(0);
        e = T(1);
        return;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) f[24 + k] = *at(s + (24 + k) * P, c);
    e = *at(a.eps, c);
}

// Whether every cell of the rectangle [xl, xh] x [yl, yh] of plane z is
// vacuum with zero rest populations.  A cell with eps_r = 1 whose e_0 is zero
// keeps e_0 = 0: its equilibrium (eps_r - 1) E is zero, the collision only
// flips the sign and the layer relaxes towards zero.  Such a cell needs
// neither e_0 nor eps_r from memory, and its stored e_0 stays zero.
template <typename T>
__device__ inline bool vacuum_plane(const StepArgs<T> &a, int z, int xl, int xh, int yl, int yh) {
    if (!a.vbox) return false;
    const int4 b = a.vbox[z];
    return b.x > b.y || b.y < xl || b.x > xh || b.w < yl || b.z > yh;
}

// LINE: the layer follows the exact incident line a.line_tab.
template <typename T, int VX, bool LINE = false>
__global__ void __launch_bounds__(256) k_step3d(StepArgs<T> a) {
    const int x0 = (blockIdx.x * blockDim.x + threadIdx.x) * VX;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x0 >= a.nx || y >= a.ny) return;
    const int ym = pull_lo(y, a.ny, a.W[1]), yp = pull_hi(y, a.ny, a.W[1]);
    const int zm = pull_lo(z, a.nz, a.W[2]), zp = pull_hi(z, a.nz, a.W[2]);
    const int64_t P = a.plane;
    const uint32_t sy = (uint32_t)a.sy, sz = (uint32_t)a.sz;
    const uint32_t base = (uint32_t)z * sz + (uint32_t)y * sy;
    // row start of the source of each direction (x handled separately)
    const uint32_t srow[6] = {base, base, (uint32_t)z * sz + (uint32_t)ym * sy, (uint32_t)z * sz + (uint32_t)yp * sy,
                              (uint32_t)zm * sz + (uint32_t)y * sy, (uint32_t)zp * sz + (uint32_t)y * sy};
    const T *s = a.src;
    const bool full = x0 + VX <= a.nx;
    const bool inner = full && x0 > 0 && x0 + VX < a.nx;
    T v[27][VX], e[VX];
    if (inner) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            load_shifted<T, VX>(v[k], at(s + k * P, base + x0 - 1));            // +x from x-1
            load_shifted<T, VX>(v[4 + k], at(s + (4 + k) * P, base + x0 + 1));  // -x from x+1
        }
    } else {
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            const int x = x0 + j < a.nx ? x0 + j : a.nx - 1;
            const uint32_t xm = (uint32_t)pull_lo(x, a.nx, a.W[0]), xp = (uint32_t)pull_hi(x, a.nx, a.W[0]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[k][j] = *at(s + k * P, base + xm);
                v[4 + k][j] = *at(s + (4 + k) * P, base + xp);
            }
        }
    }
    if (full) {
#pragma unroll
        for (int d = 2; d < 6; ++d)
#pragma unroll
            for (int k = 0; k < 4; ++k) load_aligned<T, VX>(v[4 * d + k], at(s + (4 * d + k) * P, srow[d] + x0));
#pragma unroll
        for (int k = 0; k < 3; ++k) load_aligned<T, VX>(v[24 + k], at(s + (24 + k) * P, base + x0));
        load_aligned<T, VX>(e, at(a.eps, base + x0));
    } else {
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            const uint32_t x = (uint32_t)(x0 + j < a.nx ? x0 + j : a.nx - 1);
#pragma unroll
            for (int d = 2; d < 6; ++d)
#pragma unroll
                for (int k = 0; k < 4; ++k) v[4 * d + k][j] = *at(s + (4 * d + k) * P, srow[d] + x);
#pragma unroll
            for (int k = 0; k < 3; ++k) v[24 + k][j] = *at(s + (24 + k) * P, base + x);
            e[j] = *at(a.eps, base + x);
        }
    }
    const StepConst<T> st = step_const(a, step_time(a.t_base, a.t_off));
#pragma unroll
    for (int j = 0; j < VX; ++j) {
        T f[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) f[i] = v[i][j];
        const int xj = x0 + j < a.nx ? x0 + j : a.nx - 1;
        const T *fl = nullptr;
        if (LINE)
            fl = a.line_tab + (int64_t)(st.t & (kLineSlots - 1)) * 27 * a.line_n +
                 (a.line_axis == 0 ? xj : a.line_axis == 1 ? y : z);
        cell_update3d<T, LINE>(a, st, xj, y, z, e[j], recip(e[j]), sigma3d<T>(a, xj, y, z), f, x0 + j < a.nx, fl,
                               a.line_n);
#pragma unroll
        for (int i = 0; i < 27; ++i) v[i][j] = f[i];
    }
    T *d = a.dst;
    if (full) {
#pragma unroll
        for (int i = 0; i < 27; ++i) store_aligned<T, VX>(at(d + i * P, base + x0), v[i]);
    } else {
#pragma unroll
        for (int j = 0; j < VX; ++j)
            if (x0 + j < a.nx)
#pragma unroll
                for (int i = 0; i < 27; ++i) *at(d + i * P, base + x0 + j) = v[i][j];
    }
}

// ---------------------------------------------------------------------------
// 3-D, two time steps per launch: a z march with a one-plane lag.
//
// A block of TX * TY threads (one cell each) owns an x-y tile and a chunk of
// z planes [zb, ze).  Iteration p computes step t on plane p (the tile and a
// one-cell x-y ring, pulling f*(t-1) from global memory) and then step t+1
// on plane p - 1.  Step t+1 on plane q pulls its x/y movers from plane q's
// neighbours -- kept in LDS, double-buffered by plane parity, each where it
// is pulled from -- and its z movers from planes q - 1 and q + 1 of its own
// column, which the same thread computed: the +z movers of the two previous
// planes, the rest scalars, eps, 1/eps and sigma of plane p - 1 stay in its
// registers.  Planes zb - 1 and ze (outside the chunk, folded at the domain
// faces) are computed for their z movers only; they record nothing.  Every
// cell runs cell_update3d, so the result is bit-identical to two one-step
// launches.  HBM bytes per two steps: the state read once (plus the x-y ring
// and the two extra planes per chunk) and written once.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY>
struct X3Lds {
    T xm[4][TY][TX + 1];   // +x movers (planes 0..3): left ring at column 0, tile column ox at ox + 1
    T xp[4][TY][TX + 1];   // -x movers (planes 4..7): tile column ox at ox, right ring at TX
    T ym[4][TY + 1][TX];   // +y movers (planes 8..11): ring row above at 0, tile row oy at oy + 1
    T yp[4][TY + 1][TX];   // -y movers (planes 12..15): tile row oy at oy, ring row below at TY
};

// LINE: exact incident line along z (the only direction a 3-D line takes):
// its values depend on the plane alone, so each iteration stages the next
// iteration's 2 x 27 values in LDS before its second barrier.
// DFT: the launch may fall into the DFT window (the contour accumulation is
// compiled in only then: it costs registers the plain steps do not need).
// Planes on which the tile and its ring are vacuum (vacuum_plane) neither
// read nor write the rest populations and read no eps_r.
template <typename T, int TX, int TY, bool LINE = false, bool DFT = true>
__global__ void __launch_bounds__(TX * TY, 1024 / (TX * TY)) k_step3d_x2(StepArgs<T> a, int zc) {
    constexpr int NT = TX * TY;
    constexpr int NR = 2 * TX + 2 * TY;
    static_assert(NR <= NT, "ring larger than the block");
    static_assert(NT >= 54, "line staging needs 54 threads");
    __shared__ X3Lds<T, TX, TY> L[2];
    __shared__ T lz[2][2][27];   // [plane parity][step t, t+1][population]
    const int tiles = a.tiles_x * a.tiles_y;
    // XCD-banded order: neighbouring tiles of a chunk share an L2, so the
    // ring cells' reads of a neighbour's plane hit it
    const int bid = xcd_tile(blockIdx.x, gridDim.x);
    const int tile = bid % tiles, chunk = bid / tiles;
    const int x0 = (tile % a.tiles_x) * TX, y0 = (tile / a.tiles_x) * TY;
    const int zb = chunk * zc, ze = min(zb + zc, a.nz);
    const int tid = threadIdx.x;
    const int ox = tid % TX, oy = tid / TX;
    const int x = x0 + ox, y = y0 + oy;
    const bool own = x < a.nx && y < a.ny;
    const int xf = fold(x, a.nx, a.W[0]), yf = fold(y, a.ny, a.W[1]);
    const int64_t t = step_time(a.t_base, a.t_off);
    StepConst<T> s0, s1;
    step_consts2(a, t, s0, s1);
    // this thread's ring cell (same x-y position on every plane)
    const bool ring = tid < NR;
    int rx = 0, ry = 0;
    if (tid < TX) { rx = x0 + tid; ry = y0 - 1; }
    else if (tid < 2 * TX) { rx = x0 + (tid - TX); ry = y0 + TY; }
    else if (tid < 2 * TX + TY) { rx = x0 - 1; ry = y0 + (tid - 2 * TX); }
    else { rx = x0 + TX; ry = y0 + (tid - 2 * TX - TY); }
    const int rxf = fold(rx, a.nx, a.W[0]), ryf = fold(ry, a.ny, a.W[1]);
    // folded x and y ranges of the tile and its ring (a periodic axis whose
    // ring wraps takes the whole axis)
    auto span = [](int lo, int hi, int n, int W, int &l, int &h) {
        if (W) { l = max(lo, 0); h = min(hi, n - 1); }
        else if (lo < 0 || hi >= n) { l = 0; h = n - 1; }
        else { l = lo; h = hi; }
    };
    int vxl, vxh, vyl, vyh;
    span(x0 - 1, x0 + TX, a.nx, a.W[0], vxl, vxh);
    span(y0 - 1, y0 + TY, a.ny, a.W[1], vyl, vyh);
    // which of the chunk's planes zb - 1 .. ze are vacuum for the tile and
    // its ring, one bit per plane, formed once so that the march does not
    // wait on the box table at every plane
    __shared__ unsigned long long vbits[kX3MaxPlanes / 64];
    const int np = ze - zb + 2;
    for (int i0 = 0; i0 < np; i0 += NT) {
        const int i = i0 + tid;
        const bool v = i < np && vacuum_plane(a, fold(zb - 1 + i, a.nz, a.W[2]), vxl, vxh, vyl, vyh);
        const unsigned long long m = __ballot(v);
        if ((tid & 63) == 0 && i < np) vbits[i >> 6] = m;
    }
    bool vprev = false;   // plane p - 1 was vacuum
    // the incident wave's x-y phase factors of the own and the ring cell
    // (fixed for the whole march) and the z factor of plane p - 1
    using C2 = typename Cplx<T>::type;
    C2 wo{}, wg{}, wzq{};
    if (a.src_on) {
        wo = xy_phase(a, xf, yf);
        if (ring) wg = xy_phase(a, rxf, ryf);
    }
    // per-column history: +z movers of planes p-2 (pz0) and p-1 (pz1); rest
    // scalars, eps, 1/eps and sigma of plane p-1
    T pz0[4], pz1[4], rest[3], ep = T(1), ip = T(1), sg = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) pz0[k] = pz1[k] = T(0);
    rest[0] = rest[1] = rest[2] = T(0);
    const int64_t P = a.plane;
    const uint32_t sy = (uint32_t)a.sy, sz = (uint32_t)a.sz;
    // the line's populations of step t on plane p and of step t+1 on plane
    // p - 1, for iteration p, into lz[p & 1]
    auto stage_line = [&](int p) {
        if (tid < 54) {
            const int st1 = tid / 27, i = tid % 27;
            const int zz = st1 ? fold(p - 1, a.nz, a.W[2]) : fold(p, a.nz, a.W[2]);
            lz[p & 1][st1][i] = a.line_tab[((int64_t)((t + st1) & (kLineSlots - 1)) * 27 + i) * a.line_n + zz];
        }
    };
    if (LINE) stage_line(zb - 1);
    __syncthreads();

    for (int p = zb - 1; p <= ze; ++p) {
        const int pf = fold(p, a.nz, a.W[2]);
        X3Lds<T, TX, TY> &B = L[p & 1];
        const int vi = p - zb + 1;
        const bool vp = (vbits[vi >> 6] >> (vi & 63)) & 1ull;
        // the plane's z phase factor, loaded with the state
        C2 wzp{};
        if (a.src_on) wzp = a.wave_z[pf];
        // step t on plane p: own cell ...
        T f[27], e;
        pull3d<T>(a, xf, yf, pf, f, e, vp);
        const T ie = recip(e), sgp = sigma3d<T>(a, xf, yf, pf);
        cell_update3d<T, LINE, false, DFT, true>(a, s0, xf, yf, pf, e, ie, sgp, f, own && p >= zb && p < ze,
                                                 lz[p & 1][0], 1, wo, wzp);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            B.xm[k][oy][ox + 1] = f[k];
            B.xp[k][oy][ox] = f[4 + k];
            B.ym[k][oy + 1][ox] = f[8 + k];
            B.yp[k][oy][ox] = f[12 + k];
        }
        // ... and the ring cell (only the movers that step t+1 pulls)
        if (ring) {
            T g[27], ge;
            pull3d<T>(a, rxf, ryf, pf, g, ge, vp);
            cell_update3d<T, LINE, false, DFT, true>(a, s0, rxf, ryf, pf, ge, recip(ge), sigma3d<T>(a, rxf, ryf, pf),
                                                     g, false, lz[p & 1][0], 1, wg, wzp);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (tid < TX) B.ym[k][0][tid] = g[8 + k];
                else if (tid < 2 * TX) B.yp[k][TY][tid - TX] = g[12 + k];
                else if (tid < 2 * TX + TY) B.xm[k][ry - y0][0] = g[k];
                else B.xp[k][ry - y0][TX] = g[4 + k];
            }
        }
        __syncthreads();
        // step t+1 on plane q = p - 1
        const int q = p - 1;
        if (q >= zb) {
            const X3Lds<T, TX, TY> &A = L[q & 1];
            T h[27];
            const int cxm = (a.W[0] && x == 0) ? ox + 1 : ox;          // +x movers from x-1 (own on the face)
            const int cxp = (a.W[0] && x == a.nx - 1) ? ox : ox + 1;   // -x movers from x+1
            const int rym = (a.W[1] && y == 0) ? oy + 1 : oy;          // +y movers from y-1
            const int ryp = (a.W[1] && y == a.ny - 1) ? oy : oy + 1;   // -y movers from y+1
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                h[k] = A.xm[k][oy][cxm];
                h[4 + k] = A.xp[k][oy][cxp];
                h[8 + k] = A.ym[k][rym][ox];
                h[12 + k] = A.yp[k][ryp][ox];
                h[16 + k] = pz0[k];        // +z movers from plane q - 1
                h[20 + k] = f[20 + k];     // -z movers from plane q + 1 = p
            }
            h[24] = rest[0];
            h[25] = rest[1];
            h[26] = rest[2];
            cell_update3d<T, LINE, false, DFT, true>(a, s1, xf, yf, q, ep, ip, sg, h, own, lz[p & 1][1], 1, wo, wzq);
            if (own) {
                // streamed out: the next launch reads it from HBM
                const uint32_t c = (uint32_t)q * sz + (uint32_t)y * sy + (uint32_t)x;
#pragma unroll
                for (int i = 0; i < 24; ++i) __builtin_nontemporal_store(h[i], at(a.dst + i * P, c));
                if (!vprev)
#pragma unroll
                    for (int i = 24; i < 27; ++i) __builtin_nontemporal_store(h[i], at(a.dst + i * P, c));
            }
        }
        if (LINE && p < ze) stage_line(p + 1);
        __syncthreads();
        // plane p becomes the previous plane
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pz0[k] = pz1[k];
            pz1[k] = f[16 + k];
        }
        rest[0] = f[24];
        rest[1] = f[25];
        rest[2] = f[26];
        ep = e;
        ip = ie;
        sg = sgp;
        vprev = vp;
        wzq = wzp;
    }
}

// The 3-D incident line (along z; the line handle is 1 x 1 x n) held in
// LDS for nsteps: the same per-cell update as the grid's cells, pulling
// the +z movers from u - 1 and the -z movers from u + 1, the x/y movers
// (a single periodic cell) from the cell itself.
template <typename T>
__global__ void __launch_bounds__(1024) k_line3d_lds(StepArgs<T> a, T *dst, int nsteps) {
    extern __shared__ unsigned char line_raw3[];
    T *S = reinterpret_cast<T *>(line_raw3);    // 27 planes x n
    const int n = a.line_n, NT = blockDim.x, tid = threadIdx.x;
    const int64_t P = a.plane, cstride = a.sz;
    const int Wl = a.W[2];
    for (int k = tid; k < 27 * n; k += NT) S[k] = a.src[(k / n) * P + (k % n) * cstride];
    __syncthreads();
    const int64_t t0 = step_time(a.t_base, a.t_off);
    for (int s = 0; s < nsteps; ++s) {
        const StepConst<T> st = step_const(a, t0 + s);
        T out[27];
        const int u = tid;
        if (u < n) {
            const int lo = pull_lo(u, n, Wl), hi = pull_hi(u, n, Wl);
            T f[27];
#pragma unroll
            for (int i = 0; i < 27; ++i) f[i] = S[i * n + u];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                f[16 + k] = S[(16 + k) * n + lo];
                f[20 + k] = S[(20 + k) * n + hi];
            }
            cell_update3d<T, false, true>(a, st, 0, 0, u, T(1), recip(T(1)), sigma3d<T>(a, 0, 0, u), f, true);
#pragma unroll
            for (int i = 0; i < 27; ++i) out[i] = f[i];
        }
        __syncthreads();
        if (u < n)
#pragma unroll
            for (int i = 0; i < 27; ++i) S[i * n + u] = out[i];
        __syncthreads();
    }
    for (int k = tid; k < 27 * n; k += NT) dst[(k / n) * P + (k % n) * cstride] = S[k];
}

// The 3-D incident line's own steps through global memory (lines longer
// than the LDS holds): one block walks the line's cells with the same pulls
// and per-cell update as k_line3d_lds, one or two steps per launch (a0 / a1:
// the arguments of the two steps, buffers swapped), recording each step's
// post-collision populations for the grid launch that follows.  A barrier
// separates the two steps (one workgroup: its release/acquire at workgroup
// scope orders the first step's global writes).
template <typename T>
__global__ void __launch_bounds__(1024) k_line3d(StepArgs<T> a0, StepArgs<T> a1, int nsteps) {
    for (int s = 0; s < nsteps; ++s) {
        const StepArgs<T> &a = s == 0 ? a0 : a1;
        const StepConst<T> st = step_const(a, step_time(a.t_base, a.t_off));
        const uint32_t sz = (uint32_t)a.sz;
        for (int u = threadIdx.x; u < a.line_n; u += blockDim.x) {
            T f[27], e;
            pull3d<T>(a, 0, 0, u, f, e);    // x/y movers from the cell itself (a single periodic cell)
            cell_update3d<T, false, true>(a, st, 0, 0, u, T(1), recip(T(1)), sigma3d<T>(a, 0, 0, u), f, true);
#pragma unroll
            for (int i = 0; i < 27; ++i) *at(a.dst + i * a.plane, (uint32_t)u * sz) = f[i];
        }
        if (s + 1 < nsteps) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Discrete adjoint of the 2-D step (inverse design).
//
// Forward, per step t:  s(t) = Pi x(t) (pull with the open-boundary clamp),
// F(t) = L s(t) (fields), x(t+1) = K s(t) + source, K = (1 - sigma)(2 Q L - I)
// (Q: fields -> equilibria).  For an objective J(F) the adjoint
// mu(t) = dJ/ds(t) obeys  mu(t) = K^T lambda(t+1) + L^T dJ/dF(t),
// lambda(t) = Pi^T mu(t), and  dJ/deps = sum_t lambda(t+1) . (dK/deps) s(t).
// The buffer holds mu; one adjoint launch per step reverse-pulls mu(t+1)
// (population i from r + c_i; a face node whose forward pull was clamped
// also keeps its own value), accumulates the gradient, applies K^T and adds
// the objective's source at contour nodes inside the DFT window.
// ---------------------------------------------------------------------------
template <typename T>
struct AdjArgs {
    int nx, ny;
    int64_t sy, plane;
    int W[2];
    T inv_w[2];
    T sigma_max;
    const T *__restrict__ src;   // mu(t+1)
    T *__restrict__ dst;         // mu(t)
    const T *__restrict__ eps;
    int64_t t;
    // objective source: G (complex, per contour node and component c of
    // Ex..Hz) so that dJ/dF_c(t) = 2 Re(G_c (2/winlen) e^{-j omega t})
    Box box;
    int64_t win0, winlen;
    int period;
    const double *G;             // (nnodes) x 6 x (re, im)
    // gradient
    const T *hist;               // d for step t, design rectangle
    const T *hist_prev;          // d for step t - 1 (two-step kernel)
    double *grad;                // design rectangle, accumulated
    int dlo[2], dhi[2];
    int tiles_x;                 // tile grid (two-step kernel)
};

// L^T u for the 11 reduced scalars (u: TM (Ez, Hx, Hy), TE (Ex, Ey, Hz)).
template <typename T, int POL>
__device__ inline void fields2d_T(const T u[3], T eps, T inv_eps, T o[11]) {
    const T re = (T(6) * eps - T(4)) * inv_eps;
    if (POL == TM) {
        const T e = u[0] * inv_eps;
        o[0] = e - u[2]; o[1] = e + u[2]; o[2] = e + u[1]; o[3] = e - u[1];
        o[4] = o[5] = u[1];
        o[6] = o[7] = u[2];
        o[8] = re * u[0]; o[9] = T(2) * u[1]; o[10] = T(2) * u[2];
    } else {
        const T ex = u[0] * inv_eps, ey = u[1] * inv_eps;
        o[0] = ex; o[1] = ex; o[2] = ex - u[2]; o[3] = ex + u[2];
        o[4] = ey + u[2]; o[5] = ey - u[2]; o[6] = ey; o[7] = ey;
        o[8] = re * u[0]; o[9] = re * u[1]; o[10] = T(2) * u[2];
    }
}

// Q^T l: the equilibrium map transposed (fields <- 11 scalars).
template <typename T, int POL>
__device__ inline void equilibrium2d_T(const T l[11], T u[3]) {
    // the factor 1/6 through sixth(): no bias from the rounded constant
    if (POL == TM) {
        u[0] = sixth(l[0] + l[1] + l[2] + l[3] + l[8]);
        u[1] = sixth(l[2] - l[3] + l[4] + l[5] + l[9]);
        u[2] = sixth(-l[0] + l[1] + l[6] + l[7] + l[10]);
    } else {
        u[0] = sixth(l[0] + l[1] + l[2] + l[3] + l[8]);
        u[1] = sixth(l[4] + l[5] + l[6] + l[7] + l[9]);
        u[2] = sixth(-l[2] + l[3] + l[4] - l[5] + l[10]);
    }
}

// Reverse pull of one cell: l_i = mu_i(r + c_i) (zero past an absorbing
// face) plus, on an absorbing face whose forward pull was clamped, the
// cell's own mu_i.  m = mu(t+1).
template <typename T>
__device__ inline void adj_pull_cell(const AdjArgs<T> &a, int x, int y, T l[11]) {
    const int64_t P = a.plane;
    const T *m = a.src;
    const uint32_t sy = (uint32_t)a.sy;
    const uint32_t row = (uint32_t)y * sy, c = row + (uint32_t)x;
    {   // +x populations (forward pull from x-1): adjoint from x+1
        const bool in = x + 1 < a.nx || a.W[0] == 0;
        const uint32_t n = row + (uint32_t)(x + 1 < a.nx ? x + 1 : 0);
        const bool self = a.W[0] && x == 0;
        for (int i : {0, 4}) l[i] = (in ? *at(m + i * P, n) : T(0)) + (self ? *at(m + i * P, c) : T(0));
    }
    {   // -x populations: adjoint from x-1
        const bool in = x > 0 || a.W[0] == 0;
        const uint32_t n = row + (uint32_t)(x > 0 ? x - 1 : a.nx - 1);
        const bool self = a.W[0] && x == a.nx - 1;
        for (int i : {1, 5}) l[i] = (in ? *at(m + i * P, n) : T(0)) + (self ? *at(m + i * P, c) : T(0));
    }
    {   // +y populations: adjoint from y+1
        const bool in = y + 1 < a.ny || a.W[1] == 0;
        const uint32_t n = (uint32_t)(y + 1 < a.ny ? y + 1 : 0) * sy + (uint32_t)x;
        const bool self = a.W[1] && y == 0;
        for (int i : {2, 6}) l[i] = (in ? *at(m + i * P, n) : T(0)) + (self ? *at(m + i * P, c) : T(0));
    }
    {   // -y populations: adjoint from y-1
        const bool in = y > 0 || a.W[1] == 0;
        const uint32_t n = (uint32_t)(y > 0 ? y - 1 : a.ny - 1) * sy + (uint32_t)x;
        const bool self = a.W[1] && y == a.ny - 1;
        for (int i : {3, 7}) l[i] = (in ? *at(m + i * P, n) : T(0)) + (self ? *at(m + i * P, c) : T(0));
    }
    l[8] = *at(m + 8 * P, c);
    l[9] = *at(m + 9 * P, c);
    l[10] = *at(m + 10 * P, c);
}

// Reverse pull of the VX cells x0 .. x0+VX-1 of row y (0 <= y < ny) and
// their eps: the same values as adj_pull_cell per cell, with vector loads
// when the segment has both x neighbours inside the domain.
template <typename T, int VX>
__device__ inline void adj_pull_row(const AdjArgs<T> &a, int x0, int y, T (&l)[11][VX], T (&e)[VX]) {
    const uint32_t sy = (uint32_t)a.sy;
    if (!(x0 > 0 && x0 + VX < a.nx)) {
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const int xf = fold(x0 + k, a.nx, a.W[0]);
            T f[11];
            adj_pull_cell<T>(a, xf, y, f);
#pragma unroll
            for (int i = 0; i < 11; ++i) l[i][k] = f[i];
            e[k] = *at(a.eps, (uint32_t)y * sy + (uint32_t)xf);
        }
        return;
    }
    const int64_t P = a.plane;
    const T *m = a.src;
    const uint32_t c = (uint32_t)y * sy + (uint32_t)x0;
    T v[VX];
    // x movers: both neighbours inside, no face term
    for (int i : {0, 4}) {
        load_shifted<T, VX>(v, at(m + i * P, c + 1));
#pragma unroll
        for (int k = 0; k < VX; ++k) l[i][k] = v[k] + T(0);
    }
    for (int i : {1, 5}) {
        load_shifted<T, VX>(v, at(m + i * P, c - 1));
#pragma unroll
        for (int k = 0; k < VX; ++k) l[i][k] = v[k] + T(0);
    }
    // y movers: the row rules are uniform over the segment
    const bool inp = y + 1 < a.ny || a.W[1] == 0, selfp = a.W[1] && y == 0;
    const bool inm = y > 0 || a.W[1] == 0, selfm = a.W[1] && y == a.ny - 1;
    const uint32_t cp = (uint32_t)(y + 1 < a.ny ? y + 1 : 0) * sy + (uint32_t)x0;
    const uint32_t cm = (uint32_t)(y > 0 ? y - 1 : a.ny - 1) * sy + (uint32_t)x0;
    T o[VX];
    for (int i : {2, 6}) {
        load_aligned<T, VX>(v, at(m + i * P, cp));
        load_aligned<T, VX>(o, at(m + i * P, c));
#pragma unroll
        for (int k = 0; k < VX; ++k) l[i][k] = (inp ? v[k] : T(0)) + (selfp ? o[k] : T(0));
    }
    for (int i : {3, 7}) {
        load_aligned<T, VX>(v, at(m + i * P, cm));
        load_aligned<T, VX>(o, at(m + i * P, c));
#pragma unroll
        for (int k = 0; k < VX; ++k) l[i][k] = (inm ? v[k] : T(0)) + (selfm ? o[k] : T(0));
    }
    load_aligned<T, VX>(l[8], at(m + 8 * P, c));
    load_aligned<T, VX>(l[9], at(m + 9 * P, c));
    load_aligned<T, VX>(l[10], at(m + 10 * P, c));
    load_aligned<T, VX>(e, at(a.eps, c));
}

// One adjoint cell update at step t: l holds the reverse-pulled mu(t+1) on
// entry and mu(t) on exit; hist = the recorded dE/deps of step t.  record:
// the cell is in the domain and owned by this thread, so it adds its
// gradient term.  The objective's source is part of mu(t) itself and is
// applied to every cell, ring copies included.
template <typename T, int POL>
__device__ inline void adj_cell2d(const AdjArgs<T> &a, int64_t t, const T *hist, int x, int y, T eps, T inv_eps,
                                  T sig, T l[11], bool record) {
    T u[3];
    equilibrium2d_T<T, POL>(l, u);
    // gradient: lambda . dK/deps s = 2 (Q^T lambda)_E . dE/deps
    if (record && hist && x >= a.dlo[0] && x <= a.dhi[0] && y >= a.dlo[1] && y <= a.dhi[1]) {
        const int64_t dw = a.dhi[0] - a.dlo[0] + 1;
        const int64_t cell = (int64_t)(y - a.dlo[1]) * dw + (x - a.dlo[0]);
        double g;
        if (POL == TM) g = 2.0 * (double)u[0] * (double)hist[cell];
        else g = 2.0 * ((double)u[0] * (double)hist[2 * cell] + (double)u[1] * (double)hist[2 * cell + 1]);
        a.grad[cell] += g;
    }
    // K^T lambda = (1 - sigma)(2 L^T Q^T lambda - lambda)
    T o[11];
    fields2d_T<T, POL>(u, eps, inv_eps, o);
#pragma unroll
    for (int i = 0; i < 11; ++i) l[i] = (T(1) - sig) * (T(2) * o[i] - l[i]);
    // objective source L^T dJ/dF at contour nodes inside the DFT window
    if (a.G && t >= a.win0 && t < a.win0 + a.winlen && on_box(a.box, 2, x, y, 0)) {
        const int64_t node = box_node_index(a.box, 2, x, y, 0);
        const double ph = 2.0 * M_PI * (double)(t % a.period) / (double)a.period;
        const double sc = 2.0 / (double)a.winlen;
        const double cr = sc * cos(ph), ci = -sc * sin(ph);
        const double *g = a.G + node * 12;
        double dF[6];
        for (int k = 0; k < 6; ++k) dF[k] = 2.0 * (g[2 * k] * cr - g[2 * k + 1] * ci);
        T v[3];
        if (POL == TM) { v[0] = (T)dF[2]; v[1] = (T)dF[3]; v[2] = (T)dF[4]; }
        else { v[0] = (T)dF[0]; v[1] = (T)dF[1]; v[2] = (T)dF[5]; }
        T q[11];
        fields2d_T<T, POL>(v, eps, inv_eps, q);
#pragma unroll
        for (int i = 0; i < 11; ++i) l[i] += q[i];
    }
}

template <typename T>
__device__ inline T adj_sigma(const AdjArgs<T> &a, int x, int y) {
    return fmax(sigma_axis<T>(x, a.nx, a.W[0], a.inv_w[0], a.sigma_max),
                sigma_axis<T>(y, a.ny, a.W[1], a.inv_w[1], a.sigma_max));
}

template <typename T, int POL>
__global__ void __launch_bounds__(256) k_adjoint2d(AdjArgs<T> a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    T l[11];
    adj_pull_cell<T>(a, x, y, l);
    const uint32_t c = (uint32_t)y * (uint32_t)a.sy + (uint32_t)x;
    const T eps = *at(a.eps, c);
    adj_cell2d<T, POL>(a, a.t, a.hist, x, y, eps, recip(eps), adj_sigma<T>(a, x, y), l, true);
    T *d = a.dst;
#pragma unroll
    for (int i = 0; i < 11; ++i) *at(d + i * a.plane, c) = l[i];
}

// Two adjoint steps per launch (t, then t - 1), the transpose of the
// two-step forward kernel's blocking: step t on the tile's segments and a
// one-cell ring, reverse-pulling mu(t+1) from global memory; the moving
// populations of mu(t) go to LDS where step t - 1 reverse-pulls them (the
// +x movers of the tile and the right ring column, the -x movers and the
// left column, the +y movers and the row below, the -y movers and the row
// above); step t - 1 then writes mu(t-1).  Same per-cell function as the
// one-step adjoint kernel, so the result is bit-identical; ring cells add
// no gradient (their owners do).
template <typename T, int POL, int TX, int TY>
__global__ void __launch_bounds__((x2_threads<T, TX, TY>()), (1024 / x2_threads<T, TX, TY>()))
    k_adjoint2d_x2(AdjArgs<T> a) {
    constexpr int VX = X2Lds<T, TX, TY>::VX;
    constexpr int TPR = TX / VX;
    constexpr int NT = x2_threads<T, TX, TY>();
    constexpr int NR = 2 * TX + 2 * TY;
    static_assert(x2_tile_ok<T, TX, TY>(), "two-step tile shape");
    // LDS roles (reverse pulls): xp holds planes 0, 4 (tile, right ring);
    // xm planes 1, 5 (left ring, tile); yp planes 2, 6 (tile, row below);
    // ym planes 3, 7 (row above, tile)
    __shared__ X2Lds<T, TX, TY> L;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % a.tiles_x) * TX, y0 = (tile / a.tiles_x) * TY;
    const int tid = threadIdx.x;
    const int sx = (tid % TPR) * VX, sy = tid / TPR;
    const int x = x0 + sx, y = y0 + sy;
    const int64_t t = a.t;
    const int yf = fold(y, a.ny, a.W[1]);
    T zp[3][VX], ep[VX], ip[VX], sg[VX];

    // step t on the thread's segment
    {
        T l[11][VX], e[VX];
        adj_pull_row<T, VX>(a, x, yf, l, e);
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const int xf = fold(x + k, a.nx, a.W[0]);
            T f[11];
#pragma unroll
            for (int i = 0; i < 11; ++i) f[i] = l[i][k];
            ep[k] = e[k];
            ip[k] = recip(e[k]);
            sg[k] = adj_sigma<T>(a, xf, yf);
            adj_cell2d<T, POL>(a, t, a.hist, xf, yf, e[k], ip[k], sg[k], f, x + k < a.nx && y < a.ny);
#pragma unroll
            for (int i = 0; i < 11; ++i) l[i][k] = f[i];
            zp[0][k] = f[8];
            zp[1][k] = f[9];
            zp[2][k] = f[10];
        }
        lds_store<T, VX>(&L.xp[0][sy][sx], l[0]);
        lds_store<T, VX>(&L.xp[1][sy][sx], l[4]);
        lds_store<T, VX>(&L.xm[0][sy][VX + sx], l[1]);
        lds_store<T, VX>(&L.xm[1][sy][VX + sx], l[5]);
        lds_store<T, VX>(&L.yp[0][sy][sx], l[2]);
        lds_store<T, VX>(&L.yp[1][sy][sx], l[6]);
        lds_store<T, VX>(&L.ym[0][sy + 1][sx], l[3]);
        lds_store<T, VX>(&L.ym[1][sy + 1][sx], l[7]);
    }
    // step t on the ring: rows above (feeds -y movers) and below (+y
    // movers), columns left (-x movers) and right (+x movers)
    for (int r = tid; r < NR; r += NT) {
        int rx, ry;
        if (r < TX) { rx = x0 + r; ry = y0 - 1; }
        else if (r < 2 * TX) { rx = x0 + (r - TX); ry = y0 + TY; }
        else if (r < 2 * TX + TY) { rx = x0 - 1; ry = y0 + (r - 2 * TX); }
        else { rx = x0 + TX; ry = y0 + (r - 2 * TX - TY); }
        const int xf = fold(rx, a.nx, a.W[0]), yf2 = fold(ry, a.ny, a.W[1]);
        T f[11];
        adj_pull_cell<T>(a, xf, yf2, f);
        const T e = *at(a.eps, (uint32_t)yf2 * (uint32_t)a.sy + (uint32_t)xf);
        adj_cell2d<T, POL>(a, t, a.hist, xf, yf2, e, recip(e), adj_sigma<T>(a, xf, yf2), f, false);
        if (r < TX) {
            L.ym[0][0][r] = f[3];
            L.ym[1][0][r] = f[7];
        } else if (r < 2 * TX) {
            L.yp[0][TY][r - TX] = f[2];
            L.yp[1][TY][r - TX] = f[6];
        } else if (r < 2 * TX + TY) {
            L.xm[0][ry - y0][VX - 1] = f[1];
            L.xm[1][ry - y0][VX - 1] = f[5];
        } else {
            L.xp[0][ry - y0][TX] = f[0];
            L.xp[1][ry - y0][TX] = f[4];
        }
    }
    __syncthreads();

    // step t - 1 on the thread's segment, reverse-pulling mu(t) from LDS
    if (x >= a.nx || y >= a.ny) return;
    T l[11][VX];
    {   // +x movers from the right neighbour (none past an absorbing face;
        // plus the own value on the absorbing left face)
        T o0[VX], o4[VX];
        lds_load<T, VX>(o0, &L.xp[0][sy][sx]);
        lds_load<T, VX>(o4, &L.xp[1][sy][sx]);
        const T n0 = L.xp[0][sy][sx + VX], n4 = L.xp[1][sy][sx + VX];
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const bool in = x + k + 1 < a.nx || a.W[0] == 0;
            const bool self = a.W[0] && x + k == 0;
            const T v0 = k + 1 < VX ? o0[(k + 1) % VX] : n0, v4 = k + 1 < VX ? o4[(k + 1) % VX] : n4;
            l[0][k] = (in ? v0 : T(0)) + (self ? o0[k] : T(0));
            l[4][k] = (in ? v4 : T(0)) + (self ? o4[k] : T(0));
        }
    }
    {   // -x movers from the left neighbour
        T o1[VX], o5[VX];
        lds_load<T, VX>(o1, &L.xm[0][sy][VX + sx]);
        lds_load<T, VX>(o5, &L.xm[1][sy][VX + sx]);
        const T n1 = L.xm[0][sy][VX + sx - 1], n5 = L.xm[1][sy][VX + sx - 1];
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const bool in = x + k > 0 || a.W[0] == 0;
            const bool self = a.W[0] && x + k == a.nx - 1;
            const T v1 = k > 0 ? o1[(k + VX - 1) % VX] : n1, v5 = k > 0 ? o5[(k + VX - 1) % VX] : n5;
            l[1][k] = (in ? v1 : T(0)) + (self ? o1[k] : T(0));
            l[5][k] = (in ? v5 : T(0)) + (self ? o5[k] : T(0));
        }
    }
    {   // +y movers from the row below, -y movers from the row above
        const bool inp = y + 1 < a.ny || a.W[1] == 0, selfp = a.W[1] && y == 0;
        const bool inm = y > 0 || a.W[1] == 0, selfm = a.W[1] && y == a.ny - 1;
        T n2[VX], n6[VX], o2[VX], o6[VX], n3[VX], n7[VX], o3[VX], o7[VX];
        lds_load<T, VX>(n2, &L.yp[0][sy + 1][sx]);
        lds_load<T, VX>(n6, &L.yp[1][sy + 1][sx]);
        lds_load<T, VX>(o2, &L.yp[0][sy][sx]);
        lds_load<T, VX>(o6, &L.yp[1][sy][sx]);
        lds_load<T, VX>(n3, &L.ym[0][sy][sx]);
        lds_load<T, VX>(n7, &L.ym[1][sy][sx]);
        lds_load<T, VX>(o3, &L.ym[0][sy + 1][sx]);
        lds_load<T, VX>(o7, &L.ym[1][sy + 1][sx]);
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            l[2][k] = (inp ? n2[k] : T(0)) + (selfp ? o2[k] : T(0));
            l[6][k] = (inp ? n6[k] : T(0)) + (selfp ? o6[k] : T(0));
            l[3][k] = (inm ? n3[k] : T(0)) + (selfm ? o3[k] : T(0));
            l[7][k] = (inm ? n7[k] : T(0)) + (selfm ? o7[k] : T(0));
        }
    }
    const uint32_t c = (uint32_t)y * (uint32_t)a.sy + (uint32_t)x;
#pragma unroll
    for (int k = 0; k < VX; ++k) {
        T f[11];
#pragma unroll
        for (int i = 0; i < 8; ++i) f[i] = l[i][k];
        f[8] = zp[0][k];
        f[9] = zp[1][k];
        f[10] = zp[2][k];
        const int xf = fold(x + k, a.nx, a.W[0]);
        adj_cell2d<T, POL>(a, t - 1, a.hist_prev, xf, y, ep[k], ip[k], sg[k], f, x + k < a.nx);
#pragma unroll
        for (int i = 0; i < 11; ++i) l[i][k] = f[i];
    }
    T *d = a.dst;
    if (x + VX <= a.nx) {
#pragma unroll
        for (int i = 0; i < 11; ++i) store_aligned<T, VX>(at(d + i * a.plane, c), l[i]);
    } else {
#pragma unroll
        for (int k = 0; k < VX; ++k)
            if (x + k < a.nx)
#pragma unroll
                for (int i = 0; i < 11; ++i) *at(d + i * a.plane, c + k) = l[i][k];
    }
}

// Objective weights for the adjoint source.  J = sum_a w_a kappa |P_a|^2
// with P_a the complex far-field combination of angle a (k_ntff output,
// scattered phasors); per unique contour node p and component c:
//   G_{p,c} = sum_a w_a kappa conj(P_a) dP_a/dX_{p,c},
// dP/dX from the same edge integrals as k_ntff (trapezoid weights, one
// contribution per edge containing the node).  One thread per node.
struct AdjWeightArgs {
    Box box;
    int pol;
    double k, kappa;
    double center[3], khat[3];
    const double *theta;   // radians, relative to khat
    const double *w;
    const double *P;       // (n_angles) x 4 (P1 re, im, P2 re, im)
    int n_angles;
    int64_t nnodes;
    double *G;             // (nnodes) x 6 x (re, im)
};

static __global__ void k_adjoint_weights2d(AdjWeightArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.nnodes) return;
    const Box &b = a.box;
    // recover the node's coordinates from its unique index
    const int64_t nbx = b.hi[0] - b.lo[0] + 1, nby = b.hi[1] - b.lo[1] + 1;
    int x, y;
    if (p < nbx) { x = b.lo[0] + (int)p; y = b.lo[1]; }
    else if (p < 2 * nbx) { x = b.lo[0] + (int)(p - nbx); y = b.hi[1]; }
    else if (p < 2 * nbx + nby - 2) { x = b.lo[0]; y = b.lo[1] + 1 + (int)(p - 2 * nbx); }
    else { x = b.hi[0]; y = b.lo[1] + 1 + (int)(p - 2 * nbx - (nby - 2)); }
    double G[12];
    for (int k = 0; k < 12; ++k) G[k] = 0.0;
    for (int seg = 0; seg < 4; ++seg) {
        const int ax = seg / 2;
        const int side = (seg & 1) ? 1 : -1;
        const int pos = side < 0 ? b.lo[ax] : b.hi[ax];
        const int xy[2] = {x, y};
        if (xy[ax] != pos) continue;                 // node not on this edge
        const int ua = 1 - ax;
        const bool end = xy[ua] == b.lo[ua] || xy[ua] == b.hi[ua];
        const double wn = end ? 0.5 : 1.0;
        double n[2] = {0, 0};
        n[ax] = side;
        for (int ia = 0; ia < a.n_angles; ++ia) {
            const double th = a.theta[ia];
            const double ct = cos(th), st = sin(th);
            const double r0 = ct * a.khat[0] - st * a.khat[1], r1 = ct * a.khat[1] + st * a.khat[0];
            const double rp = r0 * ((double)x - a.center[0]) + r1 * ((double)y - a.center[1]);
            double sn, cs;
            sincos(a.k * rp, &sn, &cs);
            // conj(P) * w * kappa * wn * e^{j k r.r'}
            const double pr = a.P[4 * ia], pi = -a.P[4 * ia + 1];
            const double sc = a.w[ia] * a.kappa * wn;
            const double zr = sc * (pr * cs - pi * sn), zi = sc * (pr * sn + pi * cs);
            const double rn = r0 * n[0] + r1 * n[1];
            double coef[6] = {0, 0, 0, 0, 0, 0};   // dP/dX_c per unit phase factor
            if (a.pol == TM) { coef[2] = -rn; coef[3] = -n[1]; coef[4] = n[0]; }
            else { coef[0] = n[1]; coef[1] = -n[0]; coef[5] = -rn; }
            for (int c = 0; c < 6; ++c) {
                G[2 * c] += zr * coef[c];
                G[2 * c + 1] += zi * coef[c];
            }
        }
    }
    for (int k = 0; k < 12; ++k) a.G[p * 12 + k] = G[k];
}

// ---------------------------------------------------------------------------
// Field snapshot at the current time: pull + moments only.
// ---------------------------------------------------------------------------
template <typename T, int POL>
__global__ void __launch_bounds__(256) k_fields(StepArgs<T> a, T *E, T *H) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int64_t P = a.plane;
    const int64_t cell = ((int64_t)z * a.ny + y) * a.nx + x;   // dense output index
    T Ev[3] = {0, 0, 0}, Hv[3] = {0, 0, 0};
    const int xm = pull_lo(x, a.nx, a.W[0]), xp = pull_hi(x, a.nx, a.W[0]);
    const int ym = pull_lo(y, a.ny, a.W[1]), yp = pull_hi(y, a.ny, a.W[1]);
    if (POL != D3) {
        const int64_t row = (int64_t)y * a.sy, c = row + x;
        const int64_t rm = (int64_t)ym * a.sy, rp = (int64_t)yp * a.sy;
        const T *s = a.src;
        T f[11] = {s[0 * P + row + xm], s[1 * P + row + xp], s[2 * P + rm + x], s[3 * P + rp + x],
                   s[4 * P + row + xm], s[5 * P + row + xp], s[6 * P + rm + x], s[7 * P + rp + x],
                   s[8 * P + c],        s[9 * P + c],        s[10 * P + c]};
        const T eps = a.eps[c];
        T F[3];
        if (a.mu) {
            const T mu = a.mu[c];
            fields2d<T, POL, true>(f, eps, recip(eps), F, mu, recip(mu));
        } else {
            fields2d<T, POL>(f, eps, recip(eps), F);
        }
        if (POL == TM) { Ev[2] = F[0]; Hv[0] = F[1]; Hv[1] = F[2]; }
        else { Ev[0] = F[0]; Ev[1] = F[1]; Hv[2] = F[2]; }
    } else {
        const int zm = pull_lo(z, a.nz, a.W[2]), zp = pull_hi(z, a.nz, a.W[2]);
        const int64_t c = (int64_t)z * a.sz + (int64_t)y * a.sy + x;
        const int64_t src_cell[6] = {
            (int64_t)z * a.sz + (int64_t)y * a.sy + xm, (int64_t)z * a.sz + (int64_t)y * a.sy + xp,
            (int64_t)z * a.sz + (int64_t)ym * a.sy + x, (int64_t)z * a.sz + (int64_t)yp * a.sy + x,
            (int64_t)zm * a.sz + (int64_t)y * a.sy + x, (int64_t)zp * a.sz + (int64_t)y * a.sy + x};
        T f[27];
        for (int d = 0; d < 6; ++d)
            for (int k = 0; k < 4; ++k) f[4 * d + k] = a.src[(4 * d + k) * P + src_cell[d]];
        for (int k = 0; k < 3; ++k) f[24 + k] = a.src[(24 + k) * P + c];
        fields3d(f, recip(a.eps[c]), Ev, Hv);
    }
    for (int k = 0; k < 3; ++k) {
        E[cell * 3 + k] = Ev[k];
        H[cell * 3 + k] = Hv[k];
    }
}

// Write v into the pitched material plane wherever the dense [z][y][x]
// byte mask is set (perfect-conductor cells: v = 0 in the mu plane).
template <typename T>
__global__ void k_mask_fill(const unsigned char *mask, T *plane, T v, int nx, int ny, int64_t sy, int64_t sz) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    if (x >= nx) return;
    if (mask[((int64_t)z * ny + y) * nx + x]) plane[(int64_t)z * sz + (int64_t)y * sy + x] = v;
}

// Copy a dense [z][y][x] array into the pitched eps buffer (any dtype in).
template <typename Tin, typename T>
__global__ void k_load_eps(const Tin *in, T *eps, int nx, int ny, int nz, int64_t sy, int64_t sz) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    if (x >= nx) return;
    eps[(int64_t)z * sz + (int64_t)y * sy + x] = (T)in[((int64_t)z * ny + y) * nx + x];
}

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Plain streaming copy, 16 bytes per thread (measured bandwidth ceiling and
// counter calibration).
static __global__ void __launch_bounds__(256) k_copy16(const float4 *__restrict__ a, float4 *__restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// Element-wise equality check (autotuner) over the first `cells` elements
// of every plane of stride P (the gap after them is never written): any
// mismatch sets *flag = 1.
template <typename T>
__global__ void k_compare(const T *a, const T *b, int64_t n, int64_t P, int64_t cells, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && i % P < cells && a[i] != b[i]) flag[0] = 1;
}

// Device step counter for graph replays (vector store from one lane).
static __global__ void k_set_time(int64_t *t, int64_t value) {
    if (threadIdx.x == 0) t[0] = value;
}
static __global__ void k_advance_time(int64_t *t, int64_t by) {
    if (threadIdx.x == 0) t[0] = t[0] + by;
}

// ---------------------------------------------------------------------------
// Near-to-far-field transform: one 256-thread block per observation angle.
// Scattered phasors X - X_inc on every edge (2-D) / face (3-D) of the box,
// trapezoid weights, J = n x H, M = -n x E, N = sum w J e^{jk rhat.r'},
// L = sum w M e^{jk rhat.r'}; reduced with wavefront shuffles + LDS in FP64.
// out[angle] = (P1re, P1im, P2re, P2im):
//   2-D TM: P1 = N_z - (rhat x L)_z;  2-D TE: P1 = L_z + (rhat x N)_z;
//   3-D:    P1 = N_theta + L_phi, P2 = N_phi - L_theta.
// ---------------------------------------------------------------------------
struct NtffArgs {
    const double *acc;      // total-run phasors (nnodes+1) x 12
    const double *acc_inc;  // incident-run phasors or NULL
    Box box;
    int dim, pol;
    double k;
    double center[3];
    double khat[3], ehat[3], bhat[3];   // bhat = khat x ehat (3-D frame)
    const double *theta;    // radians
    const double *phi;
    double *out;
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

static __global__ void __launch_bounds__(256) k_ntff(NtffArgs a) {
    const int ang = blockIdx.x;
    const double th = a.theta[ang], ph = a.phi[ang];
    const double ct = cos(th), st = sin(th), cp = cos(ph), sp = sin(ph);
    double r[3];
    if (a.dim == 2) {
        // in-plane: rhat = cos(th) khat + sin(th) (z x khat)
        r[0] = ct * a.khat[0] - st * a.khat[1];
        r[1] = ct * a.khat[1] + st * a.khat[0];
        r[2] = 0.0;
    } else {
        for (int k = 0; k < 3; ++k) r[k] = ct * a.khat[k] + st * (cp * a.ehat[k] + sp * a.bhat[k]);
    }
    double acc[12];   // N (re,im) x3, L (re,im) x3
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;

    const Box &b = a.box;
    const int nseg = a.dim == 2 ? 4 : 6;
    for (int seg = 0; seg < nseg; ++seg) {
        const int ax = seg / 2;                     // normal axis
        const int side = (seg & 1) ? 1 : -1;
        const int pos = side < 0 ? b.lo[ax] : b.hi[ax];
        int ua = ax == 0 ? 1 : 0, va = ax == 2 ? 1 : 2;   // in-face axes
        const int nu = b.hi[ua] - b.lo[ua] + 1;
        const int nv = a.dim == 2 ? 1 : b.hi[va] - b.lo[va] + 1;
        const int64_t cnt = (int64_t)nu * nv;
        for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int iu = (int)(i % nu), iv = (int)(i / nu);
            int xyz[3];
            xyz[ax] = pos;
            xyz[ua] = b.lo[ua] + iu;
            if (a.dim == 3) xyz[va] = b.lo[va] + iv;
            else xyz[2] = 0;
            double w = (iu == 0 || iu == nu - 1) ? 0.5 : 1.0;
            if (a.dim == 3) w *= (iv == 0 || iv == nv - 1) ? 0.5 : 1.0;
            const int64_t node = box_node_index(b, a.dim, xyz[0], xyz[1], xyz[2]);
            const double *X = a.acc + node * 12;
            const double *Xi = a.acc_inc ? a.acc_inc + node * 12 : nullptr;
            double Er[3], Ei[3], Hr[3], Hi[3];
            for (int k = 0; k < 3; ++k) {
                Er[k] = X[2 * k] - (Xi ? Xi[2 * k] : 0.0);
                Ei[k] = X[2 * k + 1] - (Xi ? Xi[2 * k + 1] : 0.0);
                Hr[k] = X[6 + 2 * k] - (Xi ? Xi[6 + 2 * k] : 0.0);
                Hi[k] = X[6 + 2 * k + 1] - (Xi ? Xi[6 + 2 * k + 1] : 0.0);
            }
            double n[3] = {0, 0, 0};
            n[ax] = side;
            // J = n x H, M = -n x E  (complex: real and imaginary parts)
            double Jr[3], Ji[3], Mr[3], Mi[3];
            cross3(n, Hr, Jr);
            cross3(n, Hi, Ji);
            cross3(n, Er, Mr);
            cross3(n, Ei, Mi);
            double rp = 0.0;
            for (int k = 0; k < 3; ++k) rp += r[k] * ((double)xyz[k] - a.center[k]);
            double sn, cs;
            sincos(a.k * rp, &sn, &cs);
            cs *= w;
            sn *= w;
            for (int k = 0; k < 3; ++k) {
                acc[2 * k] += Jr[k] * cs - Ji[k] * sn;
                acc[2 * k + 1] += Jr[k] * sn + Ji[k] * cs;
                acc[6 + 2 * k] += -(Mr[k] * cs - Mi[k] * sn);
                acc[6 + 2 * k + 1] += -(Mr[k] * sn + Mi[k] * cs);
            }
        }
    }
    __shared__ double red[4][12];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 12; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[12];
        for (int k = 0; k < 12; ++k) s[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        // complex vectors N = (s0+is1, s2+is3, s4+is5), L = (s6+is7, ...)
        double Nr[3] = {s[0], s[2], s[4]}, Ni[3] = {s[1], s[3], s[5]};
        double Lr[3] = {s[6], s[8], s[10]}, Li[3] = {s[7], s[9], s[11]};
        double p1r, p1i, p2r = 0.0, p2i = 0.0;
        if (a.dim == 2) {
            double rxLr[3], rxLi[3], rxNr[3], rxNi[3];
            cross3(r, Lr, rxLr);
            cross3(r, Li, rxLi);
            cross3(r, Nr, rxNr);
            cross3(r, Ni, rxNi);
            if (a.pol == TM) { p1r = Nr[2] - rxLr[2]; p1i = Ni[2] - rxLi[2]; }
            else { p1r = Lr[2] + rxNr[2]; p1i = Li[2] + rxNi[2]; }
        } else {
            double tv[3], pv[3];
            for (int k = 0; k < 3; ++k) {
                tv[k] = -st * a.khat[k] + ct * (cp * a.ehat[k] + sp * a.bhat[k]);
                pv[k] = -sp * a.ehat[k] + cp * a.bhat[k];
            }
            double Ntr = 0, Nti = 0, Npr = 0, Npi = 0, Ltr = 0, Lti = 0, Lpr = 0, Lpi = 0;
            for (int k = 0; k < 3; ++k) {
                Ntr += Nr[k] * tv[k]; Nti += Ni[k] * tv[k];
                Npr += Nr[k] * pv[k]; Npi += Ni[k] * pv[k];
                Ltr += Lr[k] * tv[k]; Lti += Li[k] * tv[k];
                Lpr += Lr[k] * pv[k]; Lpi += Li[k] * pv[k];
            }
            p1r = Ntr + Lpr; p1i = Nti + Lpi;
            p2r = Npr - Ltr; p2i = Npi - Lti;
        }
        a.out[4 * ang + 0] = p1r;
        a.out[4 * ang + 1] = p1i;
        a.out[4 * ang + 2] = p2r;
        a.out[4 * ang + 3] = p2i;
    }
}

}  // namespace lbm
