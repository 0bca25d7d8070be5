/*
 * lbm_oracle.c -- FP64 reference implementation of the electromagnetic
 * lattice Boltzmann scheme of "Lattice Boltzmann method for electromagnetic
 * wave scattering" (Khan, Thampi, Roy; arXiv 2510.11042).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: a plain, slow,
 * literal implementation used by tests/, by the smoke check and by the CPU
 * baseline leg of the benchmark.  The product library never links, loads or
 * calls it, and it shares no code, header or table with the HIP kernels.
 *
 * What it computes (paper section 2.1, Eq. LBGK_equation and Eq. EDF):
 *   - D3Q7 lattice: c_0 = 0, c_1..6 = +x,-x,+y,-y,+z,-z.
 *   - Every cell holds the full vector distributions e_i, h_i (i = 0..6),
 *     i.e. 42 doubles per cell, stored cell-major ("array of structures").
 *   - Update in PUSH form, exactly as the paper writes it:
 *         e_i(r + c_i, t+1) = 2 e_i^eq(r,t) - e_i(r,t)   (same for h_i),
 *     with e_i^eq = (E - c_i x H)/6, h_i^eq = (H + c_i x E)/6 for i != 0,
 *     e_0^eq = (eps_r - 1) E, h_0^eq = (mu_r - 1) H.
 *   - Fields from the zeroth moments: sum_i e_i^eq = eps_r E and collision
 *     must conserve that moment, so E = (sum_i e_i)/eps_r, H = (sum_i h_i)/mu_r
 *     (section 2.1: fields are reconstructed from zeroth-order moments).
 *   - Open boundary (section 2.2, OBC equation): on every absorbing face the
 *     incoming populations of the boundary node are copied from the first
 *     interior node after streaming: f_i^L = f_i^{L-dx}.
 *
 * Readings where the paper is silent (identical in the GPU library, which
 * implements them independently):
 *   - Absorbing layer (the paper names PML-like layers as future work, section
 *     4): W cells on each face of a non-periodic axis.  After collision,
 *         f* <- f* - sigma(r) (f* - f^eq(E_ref, H_ref; eps_r, mu_r)),
 *     sigma = sigma_max (d/W)^2, d = 1..W the depth counted from the inner
 *     edge of the layer (d = W on the outermost node); corners take the
 *     maximum over axes.
 *   - Plane-wave source: in layer cells whose medium is the background
 *     (eps_r = mu_r = 1) the reference field is the incident plane wave
 *         E_ref = g(t) E0 ehat sin(omega t - k khat.(r - r_c)),
 *         H_ref = khat x E_ref  (unit impedance: c = 1/3 with eps = mu = 1),
 *     omega = 2 pi / (3 lambda), k = 2 pi / lambda, and
 *     g(t) = sin^2(pi t / (2 t_r)) for t < t_r, 1 afterwards.  In other layer
 *     cells the reference field is zero.
 *   - Running DFT over a window of steps [t0, t0 + M T) of the fields at a
 *     list of cells: F_hat += (2/(M T)) F(t) exp(-j omega t)  (section 2.4:
 *     record the boundary fields over one period, then Fourier transform).
 *   - Perfect electric conductor (section 3.2.1 scatters off PEC cylinders;
 *     its boundary rule is given only in the authors' earlier work): a cell
 *     flagged PEC has zero electric field.  Its moments give H = B (mu_r and
 *     eps_r play no role there, so the rest populations stay zero), E is set
 *     to 0 before the DFT sample and the collision, and the absorbing layer
 *     imposes no incident wave on it.  The adjoint does not cover PEC cells.
 *   - Exact incident line (a total-field / scattered-field-like forcing for
 *     axis-aligned incidence, which section 4 names as future work): an
 *     auxiliary one-cell-wide run along the incidence axis (same layers on that
 *     axis, background medium, same source) is advanced with the grid.  In a
 *     background layer cell the update becomes
 *         f' = f* + sigma (f_l* - f*) + sigma_a (f^eq_ref - f_l*),
 *     with f_l* the line's post-collision populations at the cell's
 *     coordinate along the axis and sigma_a the line's own layer strength
 *     there: the scattered part f* - f_l* is damped by sigma and the line's
 *     own forcing is added, so a background-only run reproduces the line
 *     exactly, and the line's DFT is the incident field.
 *
 * Order inside one time step t (paper section 2.1): moments -> DFT sample ->
 * collision -> absorbing-layer/source blend -> push streaming -> open
 * boundary copy -> t+1.
 *
 * The discrete adjoint (for the inverse-design gradient) is the transpose
 * of that step, taken operation by operation in reverse order; see
 * oracle_adjoint() at the end of this file.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 7            /* D3Q7 velocities             */
#define NV 42           /* 7 x (e: 3 + h: 3) per cell  */

static const int CV[NQ][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

typedef struct lbm_oracle_s {
    int n[3];           /* nx, ny, nz                                     */
    int W[3];           /* absorbing width per axis; 0 = periodic axis    */
    double sigma_max;
    int64_t ncell;
    double *f;          /* populations at time t (pre-collision), NV per cell */
    double *g;          /* scratch: post-collision / streamed                 */
    double *eps, *mu;   /* per-cell relative permittivity / permeability      */
    unsigned char *pec; /* per-cell PEC flag (NULL: no conductor)             */
    /* exact incident line */
    struct lbm_oracle_s *line;  /* the one-row auxiliary run, NULL: off      */
    int line_axis;              /* 0: along x, 1: along y                    */
    double *star;               /* if set: post-collision populations of the */
                                /* current step are stored here (NV / cell)  */
    double *E, *H;      /* fields at time t, 3 per cell                       */
    int64_t t;
    /* plane wave */
    int src_on;
    double lambda, omega, k, khat[3], ehat[3], amp, t_ramp, rc[3];
    /* running DFT */
    int64_t ndft;
    int64_t *dft_cell;
    double *dft;        /* ndft x 6 components x (re, im) */
    int64_t win0, winlen;
} lbm_oracle;

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static void cross(const double a[3], const double b[3], double out[3]) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static void cell_xyz(const lbm_oracle *o, int64_t c, int xyz[3]) {
    xyz[0] = (int)(c % o->n[0]);
    xyz[1] = (int)((c / o->n[0]) % o->n[1]);
    xyz[2] = (int)(c / ((int64_t)o->n[0] * o->n[1]));
}

static int64_t cell_index(const lbm_oracle *o, const int xyz[3]) {
    return ((int64_t)xyz[2] * o->n[1] + xyz[1]) * o->n[0] + xyz[0];
}

/* ------------------------------------------------------------------ */
/* Equilibria, Eq. EDF                                                 */
/* ------------------------------------------------------------------ */
/* feq[i*6 + 0..2] = e_i^eq, feq[i*6 + 3..5] = h_i^eq */
static void equilibrium(const double E[3], const double H[3], double eps, double mu,
                        double feq[NV]) {
    for (int i = 0; i < NQ; ++i) {
        double *e = feq + i * 6, *h = feq + i * 6 + 3;
        if (i == 0) {
            for (int a = 0; a < 3; ++a) {
                e[a] = (eps - 1.0) * E[a];
                h[a] = (mu - 1.0) * H[a];
            }
        } else {
            double c[3] = {CV[i][0], CV[i][1], CV[i][2]}, cxH[3], cxE[3];
            cross(c, H, cxH);
            cross(c, E, cxE);
            for (int a = 0; a < 3; ++a) {
                e[a] = (E[a] - cxH[a]) / 6.0;
                h[a] = (H[a] + cxE[a]) / 6.0;
            }
        }
    }
}

/* Zeroth moments -> fields (section 2.1): E = sum e_i / eps, H = sum h_i / mu */
static void moments(const double f[NV], double eps, double mu, double E[3], double H[3]) {
    double D[3] = {0, 0, 0}, B[3] = {0, 0, 0};
    for (int i = 0; i < NQ; ++i)
        for (int a = 0; a < 3; ++a) {
            D[a] += f[i * 6 + a];
            B[a] += f[i * 6 + 3 + a];
        }
    for (int a = 0; a < 3; ++a) {
        E[a] = D[a] / eps;
        H[a] = B[a] / mu;
    }
}

/* Absorbing-layer strength at a cell (reading: quadratic profile). */
static double sigma_at(const lbm_oracle *o, const int xyz[3]) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        int W = o->W[a];
        if (W <= 0) continue;
        int n = o->n[a], x = xyz[a], d = 0;
        if (x < W) d = W - x;                     /* low face: x = 0 -> d = W   */
        else if (x >= n - W) d = x - (n - W) + 1; /* high face: x = n-1 -> d = W */
        if (d > 0) {
            double u = (double)d / W, sa = o->sigma_max * u * u;
            if (sa > s) s = sa;
        }
    }
    return s;
}

/* Material seen by the update at a cell: eps_r and mu_r, or 1 and 1 in a
 * PEC cell, whose field recovery then zeroes E. */
static int cell_material(const lbm_oracle *o, int64_t c, double *eps, double *mu) {
    const int pec = o->pec && o->pec[c];
    *eps = pec ? 1.0 : o->eps[c];
    *mu = pec ? 1.0 : o->mu[c];
    return pec;
}

/* Fields at a cell from its (pre-collision) populations. */
static void cell_fields(const lbm_oracle *o, int64_t c, const double f[NV], double E[3], double H[3]) {
    double eps, mu;
    const int pec = cell_material(o, c, &eps, &mu);
    moments(f, eps, mu, E, H);
    if (pec) E[0] = E[1] = E[2] = 0.0;
}

/* Incident plane wave at a cell (reading; zero outside background cells). */
static void reference_field(const lbm_oracle *o, const int xyz[3], double eps, double mu,
                            int64_t t, double Er[3], double Hr[3]) {
    Er[0] = Er[1] = Er[2] = Hr[0] = Hr[1] = Hr[2] = 0.0;
    if (!o->src_on || eps != 1.0 || mu != 1.0) return;
    double g = 1.0;
    if ((double)t < o->t_ramp) {
        double s = sin(M_PI * (double)t / (2.0 * o->t_ramp));
        g = s * s;
    }
    double kr = 0.0;
    for (int a = 0; a < 3; ++a) kr += o->khat[a] * ((double)xyz[a] - o->rc[a]);
    double w = g * o->amp * sin(o->omega * (double)t - o->k * kr);
    for (int a = 0; a < 3; ++a) Er[a] = w * o->ehat[a];
    cross(o->khat, Er, Hr);
}

/* ------------------------------------------------------------------ */
/* public API                                                          */
/* ------------------------------------------------------------------ */
lbm_oracle *oracle_create(int nx, int ny, int nz, int Wx, int Wy, int Wz, double sigma_max) {
    if (nx < 1 || ny < 1 || nz < 1) return NULL;
    int n[3] = {nx, ny, nz}, W[3] = {Wx, Wy, Wz};
    for (int a = 0; a < 3; ++a)
        if (W[a] < 0 || (W[a] > 0 && 2 * W[a] > n[a]) || (W[a] > 0 && n[a] < 2)) return NULL;
    lbm_oracle *o = (lbm_oracle *)calloc(1, sizeof(lbm_oracle));
    memcpy(o->n, n, sizeof n);
    memcpy(o->W, W, sizeof W);
    o->sigma_max = sigma_max;
    o->ncell = (int64_t)nx * ny * nz;
    o->f = (double *)calloc((size_t)o->ncell * NV, sizeof(double));
    o->g = (double *)calloc((size_t)o->ncell * NV, sizeof(double));
    o->eps = (double *)malloc((size_t)o->ncell * sizeof(double));
    o->mu = (double *)malloc((size_t)o->ncell * sizeof(double));
    o->E = (double *)calloc((size_t)o->ncell * 3, sizeof(double));
    o->H = (double *)calloc((size_t)o->ncell * 3, sizeof(double));
    for (int64_t c = 0; c < o->ncell; ++c) o->eps[c] = o->mu[c] = 1.0;
    return o;
}

void oracle_destroy(lbm_oracle *o) {
    if (!o) return;
    free(o->f); free(o->g); free(o->eps); free(o->mu); free(o->pec); free(o->E); free(o->H);
    free(o->dft_cell); free(o->dft);
    if (o->line) {
        free(o->line->star);
        oracle_destroy(o->line);
    }
    free(o);
}

void oracle_set_eps(lbm_oracle *o, const double *eps) {
    memcpy(o->eps, eps, (size_t)o->ncell * sizeof(double));
}
void oracle_set_mu(lbm_oracle *o, const double *mu) {
    memcpy(o->mu, mu, (size_t)o->ncell * sizeof(double));
}
/* PEC flags, one byte per cell (non-zero: conductor); NULL clears them. */
void oracle_set_pec(lbm_oracle *o, const unsigned char *flags) {
    free(o->pec);
    o->pec = NULL;
    if (!flags) return;
    o->pec = (unsigned char *)malloc((size_t)o->ncell);
    memcpy(o->pec, flags, (size_t)o->ncell);
}

/* lambda in cells; khat, ehat unit vectors (ehat perpendicular to khat);
 * t_ramp in steps; rc = phase reference point (cell coordinates). */
void oracle_set_source(lbm_oracle *o, double lambda, const double khat[3], const double ehat[3],
                       double amp, double t_ramp, const double rc[3]) {
    o->src_on = 1;
    o->lambda = lambda;
    o->omega = 2.0 * M_PI / (3.0 * lambda);
    o->k = 2.0 * M_PI / lambda;
    o->amp = amp;
    o->t_ramp = t_ramp;
    for (int a = 0; a < 3; ++a) {
        o->khat[a] = khat[a];
        o->ehat[a] = ehat[a];
        o->rc[a] = rc[a];
    }
}

void oracle_clear_source(lbm_oracle *o) { o->src_on = 0; }

/* Cells (linear indices) whose fields are Fourier transformed over the
 * window [win0, win0 + winlen) at the source frequency. */
void oracle_set_dft(lbm_oracle *o, int64_t n, const int64_t *cells, int64_t win0, int64_t winlen) {
    free(o->dft_cell);
    free(o->dft);
    o->ndft = n;
    o->dft_cell = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    o->dft = (double *)calloc((size_t)(n > 0 ? n : 1) * 12, sizeof(double));
    if (n > 0) memcpy(o->dft_cell, cells, (size_t)n * sizeof(int64_t));
    o->win0 = win0;
    o->winlen = winlen;
    if (o->line) {
        const int na = o->n[o->line_axis];
        int64_t *all = (int64_t *)malloc((size_t)na * sizeof(int64_t));
        for (int u = 0; u < na; ++u) all[u] = u;
        oracle_set_dft(o->line, na, all, win0, winlen);
        free(all);
    }
}

/* Exact incident line along axis (0: x, 1: y, 2: z) for a grid whose source
 * propagates along that axis; axis < 0 removes it.  The line starts from a
 * zero state at the grid's current time, so set it before stepping.  The
 * line records its fields at all its cells over the DFT window of the most
 * recent oracle_set_dft call.  Returns 0, or -1 if the grid or the source
 * does not allow a line. */
int oracle_set_incident_line(lbm_oracle *o, int axis) {
    if (o->line) {
        free(o->line->star);
        oracle_destroy(o->line);
        o->line = NULL;
    }
    if (axis < 0) return 0;
    if (axis > 2 || !o->src_on || fabs(fabs(o->khat[axis]) - 1.0) > 1e-12) return -1;
    const int na = o->n[axis];
    int ln[3] = {1, 1, 1}, lw[3] = {0, 0, 0};
    ln[axis] = na;
    lw[axis] = o->W[axis];
    lbm_oracle *l = oracle_create(ln[0], ln[1], ln[2], lw[0], lw[1], lw[2], o->sigma_max);
    if (!l) return -1;
    oracle_set_source(l, o->lambda, o->khat, o->ehat, o->amp, o->t_ramp, o->rc);
    l->t = o->t;
    l->star = (double *)calloc((size_t)na * NV, sizeof(double));
    if (o->ndft > 0) {
        int64_t *cells = (int64_t *)malloc((size_t)na * sizeof(int64_t));
        for (int u = 0; u < na; ++u) cells[u] = u;
        oracle_set_dft(l, na, cells, o->win0, o->winlen);
        free(cells);
    }
    o->line = l;
    o->line_axis = axis;
    return 0;
}

/* The line's phasors: n_axis x 6 components x (re, im). */
void oracle_get_line_dft(const lbm_oracle *o, double *out) {
    if (o->line) memcpy(out, o->line->dft, (size_t)o->line->ndft * 12 * sizeof(double));
}

void oracle_get_dft(const lbm_oracle *o, double *out) {
    memcpy(out, o->dft, (size_t)o->ndft * 12 * sizeof(double));
}

int64_t oracle_time(const lbm_oracle *o) { return o->t; }
void oracle_set_time(lbm_oracle *o, int64_t t) { o->t = t; }

void oracle_get_state(const lbm_oracle *o, double *out) {
    memcpy(out, o->f, (size_t)o->ncell * NV * sizeof(double));
}
void oracle_set_state(lbm_oracle *o, const double *in) {
    memcpy(o->f, in, (size_t)o->ncell * NV * sizeof(double));
}

/* Fields of the current state: E, H as [cell][3]. */
void oracle_fields(lbm_oracle *o, double *E, double *H) {
    for (int64_t c = 0; c < o->ncell; ++c)
        cell_fields(o, c, o->f + c * NV, E + 3 * c, H + 3 * c);
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Collision and absorbing-layer blend of one cell, in place:
 * f <- 2 f^eq - f, then f <- f - sigma (f - f^eq_ref). */
/* Layer strength of the incident line at coordinate u along its axis. */
static double line_sigma(const lbm_oracle *o, int u) {
    const lbm_oracle *l = o->line;
    int xyz[3] = {0, 0, 0};
    xyz[o->line_axis] = u;
    return sigma_at(l, xyz);
}

static void collide_cell(const lbm_oracle *o, int64_t c, int64_t t, double f[NV]) {
    int xyz[3];
    cell_xyz(o, c, xyz);
    double E[3], H[3], feq[NV], eps, mu;
    const int pec = cell_material(o, c, &eps, &mu);
    cell_fields(o, c, f, E, H);
    equilibrium(E, H, eps, mu, feq);
    for (int v = 0; v < NV; ++v) f[v] = 2.0 * feq[v] - f[v];
    if (o->star) memcpy(o->star + c * NV, f, NV * sizeof(double));
    double s = sigma_at(o, xyz);
    if (s > 0.0 && o->line && o->src_on && !pec && eps == 1.0 && mu == 1.0) {
        /* exact incident line: damp the scattered part, add the line's own
         * forcing (f_l* = the line's post-collision populations this step) */
        const int u = xyz[o->line_axis];
        const double *fl = o->line->star + (int64_t)u * NV;
        const double sa = line_sigma(o, u);
        double Er[3], Hr[3], fref[NV];
        reference_field(o, xyz, eps, mu, t, Er, Hr);
        equilibrium(Er, Hr, eps, mu, fref);
        for (int v = 0; v < NV; ++v) f[v] = f[v] + s * (fl[v] - f[v]) + sa * (fref[v] - fl[v]);
        return;
    }
    if (s > 0.0) {
        double Er[3] = {0, 0, 0}, Hr[3] = {0, 0, 0}, fref[NV];
        if (!pec) reference_field(o, xyz, eps, mu, t, Er, Hr);
        equilibrium(Er, Hr, eps, mu, fref);
        for (int v = 0; v < NV; ++v) f[v] = f[v] - s * (f[v] - fref[v]);
    }
}

/* Push streaming of post-collision populations `in` into `out`, followed
 * by the open-boundary copy (section 2.2): on every face of an absorbing
 * axis the incoming populations of the boundary node are copied from the
 * first interior node along the face normal.  Every slot of `out` is first
 * poisoned with NaN so that a slot nobody writes cannot go unnoticed. */
static void push_and_obc(const lbm_oracle *o, const double *in, double *out) {
    const int64_t N = o->ncell;
#pragma omp parallel for schedule(static) if (N > 4096)
    for (int64_t v = 0; v < N * NV; ++v) out[v] = NAN;

#pragma omp parallel for schedule(static) if (N > 4096)
    for (int64_t c = 0; c < N; ++c) {
        int xyz[3];
        cell_xyz(o, c, xyz);
        for (int i = 0; i < NQ; ++i) {
            int dst[3], inside = 1;
            for (int a = 0; a < 3; ++a) {
                dst[a] = xyz[a] + CV[i][a];
                if (o->W[a] == 0) {
                    dst[a] = (dst[a] % o->n[a] + o->n[a]) % o->n[a];
                } else if (dst[a] < 0 || dst[a] >= o->n[a]) {
                    inside = 0; /* leaves the domain */
                }
            }
            if (!inside) continue;
            memcpy(out + cell_index(o, dst) * NV + i * 6, in + c * NV + i * 6, 6 * sizeof(double));
        }
    }

    for (int a = 0; a < 3; ++a) {
        if (o->W[a] == 0) continue;
        int ip = 2 * a + 1, im = 2 * a + 2; /* +axis and -axis velocities */
#pragma omp parallel for schedule(static) if (N > 4096)
        for (int64_t c = 0; c < N; ++c) {
            int xyz[3];
            cell_xyz(o, c, xyz);
            if (xyz[a] == 0) { /* low face: incoming = +axis */
                int nb[3] = {xyz[0], xyz[1], xyz[2]};
                nb[a] = 1;
                memcpy(out + c * NV + ip * 6, out + cell_index(o, nb) * NV + ip * 6,
                       6 * sizeof(double));
            }
            if (xyz[a] == o->n[a] - 1) { /* high face: incoming = -axis */
                int nb[3] = {xyz[0], xyz[1], xyz[2]};
                nb[a] = o->n[a] - 2;
                memcpy(out + c * NV + im * 6, out + cell_index(o, nb) * NV + im * 6,
                       6 * sizeof(double));
            }
        }
    }
}

/* One time step. */
static void step_once(lbm_oracle *o) {
    const int64_t N = o->ncell;
    const int64_t t = o->t;

    /* 0. the incident line takes its step t first; its post-collision
     * populations of this step stay in line->star */
    if (o->line) step_once(o->line);

    /* 1. moments -> fields at time t */
#pragma omp parallel for schedule(static) if (N > 4096)
    for (int64_t c = 0; c < N; ++c)
        cell_fields(o, c, o->f + c * NV, o->E + 3 * c, o->H + 3 * c);

    /* 2. running DFT of the recorded cells */
    if (o->ndft > 0 && t >= o->win0 && t < o->win0 + o->winlen) {
        double ph = o->omega * (double)t;
        double cr = cos(ph), ci = -sin(ph), s = 2.0 / (double)o->winlen;
        for (int64_t p = 0; p < o->ndft; ++p) {
            int64_t c = o->dft_cell[p];
            for (int a = 0; a < 6; ++a) {
                double F = a < 3 ? o->E[3 * c + a] : o->H[3 * c + a - 3];
                o->dft[p * 12 + 2 * a] += s * F * cr;
                o->dft[p * 12 + 2 * a + 1] += s * F * ci;
            }
        }
    }

    /* 3-4. collision + absorbing layer, written to g */
#pragma omp parallel for schedule(static) if (N > 4096)
    for (int64_t c = 0; c < N; ++c) {
        double fl[NV];
        memcpy(fl, o->f + c * NV, sizeof fl);
        collide_cell(o, c, t, fl);
        memcpy(o->g + c * NV, fl, sizeof fl);
    }

    /* 5-6. push streaming g -> f, then the open-boundary copy */
    push_and_obc(o, o->g, o->f);
    o->t = t + 1;
}

void oracle_step(lbm_oracle *o, int64_t nsteps) {
    for (int64_t s = 0; s < nsteps; ++s) step_once(o);
}

/* ------------------------------------------------------------------ */
/* Discrete adjoint (inverse design).                                  */
/*                                                                     */
/* One forward step is  f(t+1) = P [ K_r f(t) + s_r(t) ]  where K_r is  */
/* the per-cell collision+layer matrix (linear in f), s_r the layer's   */
/* source term and P the push/open-boundary copy.  For an objective    */
/* J depending on the fields F(t) = moments(f(t)) the gradient with    */
/* respect to eps at a cell r is                                       */
/*   dJ/deps_r = sum_t  lam*(r,t) . d(K_r f(t) + s_r(t))/deps_r        */
/*             + sum_t  dJ/dF(r,t) . dF(r,t)/deps_r                     */
/* with the adjoint recursion                                          */
/*   lam*(t) = P^T lam(t+1),                                           */
/*   lam(t)  = K^T lam*(t) + (dF/df)^T dJ/dF(t),   lam(T) = 0.          */
/* K_r is obtained column by column by applying collide_cell() to unit */
/* vectors (with the source switched off), so the transpose is taken   */
/* of exactly the forward operation.                                    */
/* ------------------------------------------------------------------ */

/* Source slot of every streamed slot: f(t+1)[s][i] = g[src][i]. */
static int64_t push_source(const lbm_oracle *o, int64_t s, int i) {
    int xyz[3];
    cell_xyz(o, s, xyz);
    /* open-boundary copy: incoming population on a face node takes the value
     * of the first interior node */
    for (int a = 0; a < 3; ++a) {
        if (o->W[a] == 0) continue;
        if (xyz[a] == 0 && i == 2 * a + 1) xyz[a] = 1;
        else if (xyz[a] == o->n[a] - 1 && i == 2 * a + 2) xyz[a] = o->n[a] - 2;
    }
    for (int a = 0; a < 3; ++a) {
        xyz[a] -= CV[i][a];
        if (o->W[a] == 0) xyz[a] = (xyz[a] % o->n[a] + o->n[a]) % o->n[a];
    }
    return cell_index(o, xyz);
}

/* Transpose of the push + open-boundary copy: out = P^T in. */
void oracle_stream_transpose(const lbm_oracle *o, const double *in, double *out) {
    const int64_t N = o->ncell;
    memset(out, 0, (size_t)N * NV * sizeof(double));
    for (int64_t s = 0; s < N; ++s)
        for (int i = 0; i < NQ; ++i) {
            int64_t src = push_source(o, s, i);
            for (int k = 0; k < 6; ++k) out[src * NV + i * 6 + k] += in[s * NV + i * 6 + k];
        }
}

/* Forward push + open boundary applied to an arbitrary vector (test hook
 * for the dot-product check of oracle_stream_transpose). */
void oracle_stream_apply(const lbm_oracle *o, const double *in, double *out) {
    push_and_obc(o, in, out);
}

/* d f^eq(D/eps, B/mu; eps, mu) / d eps at fixed populations. */
static void dfeq_deps(const double E[3], double eps, double dfeq[NV]) {
    double dE[3] = {-E[0] / eps, -E[1] / eps, -E[2] / eps}, zero[3] = {0, 0, 0};
    equilibrium(dE, zero, eps, 1.0, dfeq);      /* moving populations: linear in dE */
    for (int a = 0; a < 3; ++a) {
        dfeq[a] = (eps - 1.0) * dE[a] + E[a];    /* e_0^eq = (eps-1) E  (product rule) */
        dfeq[3 + a] = 0.0;                       /* h_0^eq does not depend on eps      */
    }
}

/* Full adjoint sweep.
 *   history : states f(0..T-1), T*N*NV doubles (pre-collision, as stepped)
 *   dJdF    : T x N x 6 doubles, dJ/dE (0..2) and dJ/dH (3..5) per cell and step
 *   grad    : N doubles, output dJ/deps per cell
 * t0 is the time index of history[0] (needed for the layer source phase). */
void oracle_adjoint(lbm_oracle *o, int64_t T, int64_t t0, const double *history,
                    const double *dJdF, double *grad) {
    const int64_t N = o->ncell;
    double *lam = (double *)calloc((size_t)N * NV, sizeof(double));
    double *lstar = (double *)calloc((size_t)N * NV, sizeof(double));
    memset(grad, 0, (size_t)N * sizeof(double));
    int src_saved = o->src_on;
    for (int64_t t = T - 1; t >= 0; --t) {
        /* lam*(t) = P^T lam(t+1) */
        oracle_stream_transpose(o, lam, lstar);
        const double *ft = history + t * N * NV;
        for (int64_t c = 0; c < N; ++c) {
            int xyz[3];
            cell_xyz(o, c, xyz);
            double *ls = lstar + c * NV;
            /* gradient: lam* . d(K_r f + s_r)/deps.  The layer blend scales the
             * collision by (1 - sigma); its source term depends on eps only
             * through the background test, which the design region avoids. */
            double E[3], H[3], d[NV];
            moments(ft + c * NV, o->eps[c], o->mu[c], E, H);
            dfeq_deps(E, o->eps[c], d);
            double sg = sigma_at(o, xyz), acc = 0.0;
            for (int v = 0; v < NV; ++v) acc += ls[v] * 2.0 * (1.0 - sg) * d[v];
            /* direct term: dJ/dE . dE/deps, E = D/eps */
            const double *jf = dJdF + (t * N + c) * 6;
            acc += -(jf[0] * E[0] + jf[1] * E[1] + jf[2] * E[2]) / o->eps[c];
            grad[c] += acc;
            /* lam(t) = K_r^T lam*(t) + (dF/df)^T dJ/dF(t); K_r by columns */
            o->src_on = 0;
            double *lo = lam + c * NV;
            for (int col = 0; col < NV; ++col) {
                double u[NV];
                memset(u, 0, sizeof u);
                u[col] = 1.0;
                collide_cell(o, c, t0 + t, u);
                double s = 0.0;
                for (int v = 0; v < NV; ++v) s += u[v] * ls[v];
                /* moments: dE_a/de_{i,a} = 1/eps, dH_a/dh_{i,a} = 1/mu */
                int comp = col % 6;
                s += comp < 3 ? jf[comp] / o->eps[c] : jf[comp] / o->mu[c];
                lo[col] = s;
            }
            o->src_on = src_saved;
        }
    }
    free(lam);
    free(lstar);
}
