/*
 * FP64 CPU oracle for the weakly-compressible SPH step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no header, helper or constant
 * with the GPU path: both sides only share the canonical encoded input state.
 *
 * What it computes, and where the paper defines it (arXiv:2207.11328):
 *   - cell grid, cell-relative positions, Moore-neighbourhood search:
 *       section "Optimizing the neighbors search";
 *   - sort by cell, then particle type, then particle id:
 *       section "Changing perspective: from the particle to the cell";
 *   - fluid neighbours from the front of the list, boundary ones from the
 *       back: section "Efficient split neighbors list";
 *   - Wendland kernel w(q) = (2q+1)(1-q/2)^4, f(q) = (q-2)^3 with
 *       F = (1/r) dW/dr: listing l:ktemplate and eq. sph-field text;
 *   - Cole equation of state: section "A lightning introduction to the
 *       method";
 *   - continuity and momentum in the golden-rule form: eq. mass-cont-sph1 and
 *       eq. ns-sph1, with the sign, mass and viscosity readings documented in
 *       the design notes (F <= 0, so the continuity sum carries a plus sign;
 *       the pressure term carries m_j; viscosity is Monaghan's artificial term
 *       or the Morris laminar term of section "Minimizing complexity");
 *   - predictor/corrector integration with dt/2 then dt: section "Code
 *       structure" (read as the explicit midpoint scheme).
 *
 * Floating point: everything physical is evaluated in double.  The one
 * exception is the neighbour predicate, which the method defines on the
 * float32 cell-relative encoding; it is evaluated here in genuine float
 * arithmetic (compiled with -ffp-contract=off, no fast-math, SSE float) so
 * that neighbour sets can be compared bit-exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double origin[3];
    float cs[3];
    int32_t n[3];
    uint32_t periodic;
    int32_t cell_base;
} orc_grid;

typedef struct {
    double h, r_search, rho0, gamma, c0, alpha, eps_visc, nu;
    double g[3];
    double cfl;
    int32_t visc_model; /* laminar term added to Monaghan's artificial viscosity:
                           0 none, 1 Morris, 2 Monaghan's K form */
    double delta;       /* Molteni-Colagrossi density diffusion coefficient (0: off) */
    int32_t kernel;     /* smoothing kernel: 0 Wendland, 1 cubic spline, 2 quadratic, 3 Gaussian */
    int32_t formulation; /* 0 golden rule (eq. mass-cont-sph1, ns-sph1), 1 Landrini-Morris
                            (eq. mass-cont-sph2, ns-sph2) */
} orc_params;

enum { ORC_WENDLAND = 0, ORC_CUBIC_SPLINE = 1, ORC_QUADRATIC = 2, ORC_GAUSSIAN = 3 };

/* K of Monaghan's laminar form in 3D (section "Minimizing complexity" leaves
 * it open).  With the weight m_j/(rho_i rho_j) and the factor 2 mu_bar that
 * the form carries, sum_j V_j (u_ij . x_ij) x_ij F_ij / r^2 tends to
 * (lap u + 2 grad div u) / (2 (d + 2)), so the term reduces to nu lap u for a
 * divergence-free flow when K = d + 2. */
#define ORC_MONAGHAN_K 5.0

#define ORC_TYPE_SHIFT 30
#define ORC_BOUNDARY 1u

static inline uint32_t ptype(uint32_t info) { return info >> ORC_TYPE_SHIFT; }

static inline void cell_coords(const orc_grid *g, int32_t cell, int32_t c[3])
{
    int32_t lc = cell - g->cell_base;
    c[0] = lc % g->n[0];
    c[1] = (lc / g->n[0]) % g->n[1];
    c[2] = lc / (g->n[0] * g->n[1]);
}

static inline int32_t cell_linear(const orc_grid *g, const int32_t c[3])
{
    return c[0] + g->n[0] * (c[1] + g->n[1] * c[2]) + g->cell_base;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------------
 * Re-binning of cell-relative offsets (float32, as the encoding is float32).
 * Offsets live in [-cs/2, cs/2).  A particle that drifted out of its cell is
 * moved by whole cells (at most 4 per axis); periodic axes wrap the cell
 * index; a particle that leaves a non-periodic grid, or whose offset is not
 * finite, becomes invalid (cell = -1).  Returns the number of invalid ones.
 * ------------------------------------------------------------------------ */
int orc_rebin(const orc_grid *g, int n, int32_t *cell, float *pos4)
{
    int dropped = 0;
    for (int i = 0; i < n; ++i) {
        if (cell[i] < 0) { ++dropped; continue; }
        int32_t c[3];
        cell_coords(g, cell[i], c);
        int ok = 1;
        for (int d = 0; d < 3; ++d) {
            float o = pos4[4 * i + d];
            const float cs = g->cs[d];
            const float half = 0.5f * cs;
            for (int it = 0; it < 4; ++it) {
                if (o >= half) { o = o - cs; c[d] += 1; }
                else if (o < -half) { o = o + cs; c[d] -= 1; }
                else break;
            }
            if (!(o >= -half && o < half)) ok = 0;
            if ((g->periodic >> d) & 1u) {
                c[d] %= g->n[d];
                if (c[d] < 0) c[d] += g->n[d];
            } else if (c[d] < 0 || c[d] >= g->n[d]) {
                ok = 0;
            }
            pos4[4 * i + d] = o;
        }
        if (ok) cell[i] = cell_linear(g, c);
        else { cell[i] = -1; ++dropped; }
    }
    return dropped;
}

/* The same re-binning rule on double offsets [n][3] (double rollouts). */
int orc_rebin_f64(const orc_grid *g, int n, int32_t *cell, double *off3)
{
    int dropped = 0;
    for (int i = 0; i < n; ++i) {
        if (cell[i] < 0) { ++dropped; continue; }
        int32_t c[3];
        cell_coords(g, cell[i], c);
        int ok = 1;
        for (int d = 0; d < 3; ++d) {
            double o = off3[3 * (size_t)i + d];
            const double cs = (double)g->cs[d];
            const double half = 0.5 * cs;
            for (int it = 0; it < 4; ++it) {
                if (o >= half) { o = o - cs; c[d] += 1; }
                else if (o < -half) { o = o + cs; c[d] -= 1; }
                else break;
            }
            if (!(o >= -half && o < half)) ok = 0;
            if ((g->periodic >> d) & 1u) {
                c[d] %= g->n[d];
                if (c[d] < 0) c[d] += g->n[d];
            } else if (c[d] < 0 || c[d] >= g->n[d]) {
                ok = 0;
            }
            off3[3 * (size_t)i + d] = o;
        }
        if (ok) cell[i] = cell_linear(g, c);
        else { cell[i] = -1; ++dropped; }
    }
    return dropped;
}

/* ------------------------------------------------------------------------
 * Sort order: by cell, then type, then id (the info word is type<<30 | id).
 * Invalid particles (cell < 0) go last, in (type, id) order.
 * ------------------------------------------------------------------------ */
typedef struct { uint64_t key; int32_t idx; } orc_kv;

static int kv_cmp(const void *a, const void *b)
{
    const orc_kv *x = (const orc_kv *)a, *y = (const orc_kv *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return 0;
}

void orc_sort_perm(int n, const int32_t *cell, const uint32_t *info, int32_t *perm)
{
    orc_kv *kv = (orc_kv *)malloc(sizeof(orc_kv) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        uint32_t hi = cell[i] < 0 ? 0xFFFFFFFFu : (uint32_t)cell[i];
        kv[i].key = ((uint64_t)hi << 32) | (uint64_t)info[i];
        kv[i].idx = i;
    }
    qsort(kv, (size_t)n, sizeof(orc_kv), kv_cmp);
    for (int i = 0; i < n; ++i) perm[i] = kv[i].idx;
    free(kv);
}

/* Cell ranges of a sorted particle array: start = exclusive prefix sum of the
 * per-cell counts, end = start + count.  Cells are indexed from cell_base. */
void orc_cell_ranges(const orc_grid *g, int n, const int32_t *cell_sorted,
                     int32_t *start, int32_t *end)
{
    const int nc = g->n[0] * g->n[1] * g->n[2];
    int32_t *cnt = (int32_t *)calloc((size_t)nc, sizeof(int32_t));
    for (int i = 0; i < n; ++i)
        if (cell_sorted[i] >= 0) cnt[cell_sorted[i] - g->cell_base] += 1;
    int32_t acc = 0;
    for (int c = 0; c < nc; ++c) { start[c] = acc; acc += cnt[c]; end[c] = acc; }
    free(cnt);
}

/* ------------------------------------------------------------------------
 * Neighbour lists.  For a central particle i every particle j != i in the 27
 * cells around i's cell is a neighbour iff its separation, computed from the
 * cell-relative encoding, is below the search radius:
 *   per axis  k = c_i - c_j (one of -1, 0, 1),  t1 = o_i - o_j,  t2 = k cs,
 *             x = t2 + t1;      r2 = (x*x + y*y) + z*z;   keep iff r2 < rs*rs
 * evaluated in float on the float32 encoding pos4, or (pos4 == NULL) in
 * double on double offsets off3 (used by double-precision rollouts).  A boundary
 * particle only keeps fluid neighbours.  Output is particle-major:
 * fl[i*max + a] / bl[i*max + b] hold the a-th fluid / b-th boundary
 * neighbour, nf[i] / nb[i] their counts.  Returns the number of particles
 * whose nf + nb exceeds max (their lists are truncated).
 * ------------------------------------------------------------------------ */
/* Neighbours of one particle i; fl_row / bl_row receive its fluid / boundary
 * lists, *nf / *nb the numbers kept.  Returns 1 if the list overflowed. */
static int neighbors_of(const orc_grid *g, float r_search, int i, const int32_t *cell, const float *pos4,
                        const double *off3, const uint32_t *info, const int32_t *start, const int32_t *end,
                        int max_neibs, int32_t *nf, int32_t *nb, int32_t *fl_row, int32_t *bl_row)
{
    const float rs2f = r_search * r_search;
    const double rs2d = (double)r_search * (double)r_search;
    *nf = 0;
    *nb = 0;
    if (cell[i] < 0) return 0;
    int32_t ci[3];
    cell_coords(g, cell[i], ci);
    const uint32_t ti = ptype(info[i]);
    int cf = 0, cb = 0, wf = 0, wb = 0;
    for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
        const int off[3] = {dx, dy, dz};
        int32_t cj[3];
        int inside = 1;
        for (int d = 0; d < 3; ++d) {
            cj[d] = ci[d] + off[d];
            if ((g->periodic >> d) & 1u) {
                if (cj[d] < 0) cj[d] += g->n[d];
                if (cj[d] >= g->n[d]) cj[d] -= g->n[d];
            } else if (cj[d] < 0 || cj[d] >= g->n[d]) {
                inside = 0;
            }
        }
        if (!inside) continue;
        const int32_t lc = cell_linear(g, cj) - g->cell_base;
        for (int j = start[lc]; j < end[lc]; ++j) {
            if (j == i) continue;
            const uint32_t tj = ptype(info[j]);
            if (ti == ORC_BOUNDARY && tj == ORC_BOUNDARY) continue;
            int keep;
            if (pos4) {
                float x[3];
                for (int d = 0; d < 3; ++d) {
                    const float t1 = pos4[4 * (size_t)i + d] - pos4[4 * (size_t)j + d];
                    const float t2 = (float)(-off[d]) * g->cs[d];
                    x[d] = t2 + t1;
                }
                const float xx = x[0] * x[0];
                const float yy = x[1] * x[1];
                const float zz = x[2] * x[2];
                const float s = xx + yy;
                const float r2 = s + zz;
                keep = r2 < rs2f;
            } else {
                double r2 = 0.0;
                for (int d = 0; d < 3; ++d) {
                    const double x = (double)(-off[d]) * (double)g->cs[d]
                                   + (off3[3 * (size_t)i + d] - off3[3 * (size_t)j + d]);
                    r2 += x * x;
                }
                keep = r2 < rs2d;
            }
            if (!keep) continue;
            if (tj == ORC_BOUNDARY) {
                if (wf + wb < max_neibs) bl_row[wb++] = j;
                ++cb;
            } else {
                if (wf + wb < max_neibs) fl_row[wf++] = j;
                ++cf;
            }
        }
    }
    *nf = wf;
    *nb = wb;
    return cf + cb > max_neibs; /* truncated: only what fitted is kept */
}

int orc_neighbors(const orc_grid *g, float r_search, int n,
                  const int32_t *cell, const float *pos4, const double *off3,
                  const uint32_t *info, const int32_t *start, const int32_t *end,
                  int max_neibs, int32_t *nf, int32_t *nb, int32_t *fl, int32_t *bl)
{
    int overflow = 0;
#pragma omp parallel for schedule(static) reduction(+ : overflow)
    for (int i = 0; i < n; ++i)
        overflow += neighbors_of(g, r_search, i, cell, pos4, off3, info, start, end, max_neibs, nf + i, nb + i,
                                 fl + (size_t)i * max_neibs, bl + (size_t)i * max_neibs);
    return overflow;
}

/* The same for the particles rows[0..nrows) only (float32 predicate); row r
 * of the outputs belongs to particle rows[r].  For inputs too large to list
 * every particle. */
int orc_neighbors_rows(const orc_grid *g, float r_search, const int32_t *cell, const float *pos4,
                       const uint32_t *info, const int32_t *start, const int32_t *end, int max_neibs,
                       const int32_t *rows, int nrows, int32_t *nf, int32_t *nb, int32_t *fl, int32_t *bl)
{
    int overflow = 0;
#pragma omp parallel for schedule(static) reduction(+ : overflow)
    for (int r = 0; r < nrows; ++r)
        overflow += neighbors_of(g, r_search, rows[r], cell, pos4, NULL, info, start, end, max_neibs, nf + r,
                                 nb + r, fl + (size_t)r * max_neibs, bl + (size_t)r * max_neibs);
    return overflow;
}

/* ------------------------------------------------------------------------
 * Kernel and equation of state, double precision.
 * ------------------------------------------------------------------------ */

/* Smoothing kernels of listing l:ktemplate, 3D, all with support 2h (the
 * radius of the method), q = r/h, each normalised to unit integral (section
 * "A lightning introduction to the method"); F = (1/r) dW/dr.
 *   Wendland C2:  W = 21/(16 pi h^3) (1 - q/2)^4 (2q + 1)
 *   cubic spline (Monaghan-Lattanzio M4):
 *                 W = 1/(pi h^3) (1 - 3/2 q^2 + 3/4 q^3)   q < 1
 *                                1/4 (2 - q)^3              1 <= q < 2
 *   quadratic (Johnson, Stryk and Beissel):
 *                 W = 5/(4 pi h^3) (3/16 q^2 - 3/4 q + 3/4)
 *   Gaussian truncated at d = 2h (the listing's w(q) = exp(-q^2) - exp(-(d/h)^2)):
 *                 W = C (exp(-q^2) - exp(-4)),
 *                 1/C = 4 pi h^3 (sqrt(pi)/4 erf(2) - 11/3 exp(-4))
 * The quadratic kernel's F = 15/(32 pi h^5) (1 - 2/q) is unbounded at r = 0;
 * the Gaussian's F does not vanish at r = 2h (W does). */
static double gaussian_norm(double h)
{
    const double e4 = exp(-4.0);
    return 1.0 / (4.0 * M_PI * h * h * h * (0.25 * sqrt(M_PI) * erf(2.0) - 11.0 / 3.0 * e4));
}

double orc_kernel_W(int kind, double r, double h)
{
    const double q = r / h;
    if (q >= 2.0) return 0.0;
    const double h3 = h * h * h;
    switch (kind) {
    case ORC_WENDLAND: {
        const double a = 1.0 - 0.5 * q;
        return 21.0 / (16.0 * M_PI * h3) * a * a * a * a * (2.0 * q + 1.0);
    }
    case ORC_CUBIC_SPLINE:
        if (q < 1.0) return (1.0 - 1.5 * q * q + 0.75 * q * q * q) / (M_PI * h3);
        return 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q) / (M_PI * h3);
    case ORC_QUADRATIC:
        /* 3/16 q^2 - 3/4 q + 3/4 = 3/16 (2 - q)^2, factored for accuracy near q = 2 */
        return 5.0 / (4.0 * M_PI * h3) * 0.1875 * (2.0 - q) * (2.0 - q);
    case ORC_GAUSSIAN:
        return gaussian_norm(h) * (exp(-q * q) - exp(-4.0));
    }
    return NAN;
}

/* F = (1/r) dW/dr, derived from W above. */
double orc_kernel_F(int kind, double r, double h)
{
    const double q = r / h;
    if (q >= 2.0) return 0.0;
    const double h5 = h * h * h * h * h;
    switch (kind) {
    case ORC_WENDLAND: {
        const double b = q - 2.0;
        return 105.0 / (128.0 * M_PI * h5) * b * b * b;
    }
    case ORC_CUBIC_SPLINE:
        /* dW/dq = (-3q + 9/4 q^2) and -3/4 (2 - q)^2, over pi h^3; F = dW/dq / (q h^2) */
        if (q < 1.0) return (-3.0 + 2.25 * q) / (M_PI * h5);
        return -0.75 * (2.0 - q) * (2.0 - q) / (q * M_PI * h5);
    case ORC_QUADRATIC:
        /* dW/dq = 5/(4 pi h^3) (3/8 q - 3/4) */
        return 15.0 / (32.0 * M_PI * h5) * (1.0 - 2.0 / q);
    case ORC_GAUSSIAN:
        return -2.0 * gaussian_norm(h) / (h * h) * exp(-q * q);
    }
    return NAN;
}

/* dF/dr, the derivative of the function above (for the reverse pass). */
double orc_kernel_dF(int kind, double r, double h)
{
    const double q = r / h;
    if (q >= 2.0) return 0.0;
    const double h6 = h * h * h * h * h * h;
    switch (kind) {
    case ORC_WENDLAND: {
        const double b = q - 2.0;
        return 3.0 * 105.0 / (128.0 * M_PI * h6) * b * b;
    }
    case ORC_CUBIC_SPLINE:
        if (q < 1.0) return 2.25 / (M_PI * h6);
        return 0.75 * (4.0 - q * q) / (q * q * M_PI * h6);
    case ORC_QUADRATIC:
        return 15.0 / (16.0 * M_PI * h6) / (q * q);
    case ORC_GAUSSIAN:
        return 4.0 * gaussian_norm(h) / (h * h * h) * q * exp(-q * q);
    }
    return NAN;
}

double orc_wendland_W(double r, double h) { return orc_kernel_W(ORC_WENDLAND, r, h); }

double orc_wendland_F(double r, double h) { return orc_kernel_F(ORC_WENDLAND, r, h); }

/* Cole's equation of state P = B ((rho/rho0)^gamma - 1), B = rho0 c0^2 / gamma,
 * and the sound speed c = sqrt(dP/drho) = c0 (rho/rho0)^((gamma-1)/2). */
double orc_pressure(const orc_params *p, double rho)
{
    const double B = p->rho0 * p->c0 * p->c0 / p->gamma;
    return B * (pow(rho / p->rho0, p->gamma) - 1.0);
}

double orc_sound_speed(const orc_params *p, double rho)
{
    return p->c0 * pow(rho / p->rho0, 0.5 * (p->gamma - 1.0));
}

/* separation x_i - x_j from the cell-relative encoding, in double */
static inline void separation(const orc_grid *g, int32_t cell_i, int32_t cell_j,
                              const double *oi, const double *oj, double x[3])
{
    int32_t ci[3], cj[3];
    cell_coords(g, cell_i, ci);
    cell_coords(g, cell_j, cj);
    for (int d = 0; d < 3; ++d) {
        int k = ci[d] - cj[d];
        if ((g->periodic >> d) & 1u) {
            const int nd = g->n[d];
            while (2 * k > nd) k -= nd;
            while (2 * k < -nd) k += nd;
        }
        x[d] = (double)k * (double)g->cs[d] + (oi[d] - oj[d]);
    }
}

/* ------------------------------------------------------------------------
 * Time derivatives (the "forces").  For central particle i and every
 * listed neighbour j with r_ij < 2h, golden-rule formulation (eq.
 * mass-cont-sph1, eq. ns-sph1):
 *   Drho_i/Dt = sum_j m_j (u_ij . x_ij) F_ij
 *   a_i       = -sum_j m_j (P_i/rho_i^2 + P_j/rho_j^2 + Pi_ij) x_ij F_ij + L_i
 * or the Landrini-Morris formulation (eq. mass-cont-sph2, eq. ns-sph2):
 *   Drho_i/Dt = sum_j (rho_i/rho_j) m_j (u_ij . x_ij) F_ij
 *   a_i       = -sum_j m_j ((P_i + P_j)/(rho_i rho_j) + Pi_ij) x_ij F_ij + L_i
 * with Monaghan's artificial viscosity
 *   Pi_ij     = -alpha h cbar (u_ij . x_ij) / (rhobar (r^2 + eps h^2)) if u_ij.x_ij < 0
 * and the laminar term L_i of section "Minimizing complexity", weight
 * m_j/(rho_i rho_j) and mu_bar = 2 rho_i rho_j nu/(rho_i + rho_j) (the
 * harmonic mean of mu = rho nu):
 *   Morris:     L_i = sum_j 4 nu m_j / (rho_i + rho_j) F_ij u_ij
 *   Monaghan K: L_i = K sum_j 4 nu m_j / (rho_i + rho_j) F_ij (u_ij . x_ij) / (r^2 + eps h^2) x_ij
 * and, with delta > 0, for a fluid i and fluid j the density diffusion of
 * Molteni and Colagrossi (named among the dissipative terms of section "A
 * lightning introduction to the method" and the options of "The SPH in
 * GPUSPH", used by the dam break of "Clang: the better compiler?" and the
 * wave basin of "An industrial test case"; the formula is that
 * publication's, the paper does not print it):
 *   Drho_i/Dt += -2 delta h c0 sum_j (rho_j - rho_i) F_ij r^2 / (r^2 + eps h^2) m_j / rho_j
 * Gravity is not included (the integrator adds it to fluid particles).
 * With the quadratic kernel a pair at r = 0 contributes nothing (its F is
 * unbounded there).
 *
 * Also returned, per particle and component, the sum of the magnitudes of
 * the pair terms (every signed factor replaced by its absolute value, the dot
 * product by the sum of absolute products): the scale against which the
 * float32 result is compared.  n_inter receives the number of (i, j) pairs
 * with r < 2h.
 * ------------------------------------------------------------------------ */
/* Derivatives of one particle i from its lists (fl_row, bl_row with nfi,
 * nbi entries): a[3], drho, the magnitude scales sa[3], sdr; returns the
 * number of pairs with r < 2h. */
static int forces_of(const orc_params *p, const orc_grid *g, int i, const int32_t *cell, const double *off,
                     const double *mass, const double *vel, const double *rho, const uint32_t *info, int nfi,
                     int nbi,
                     const int32_t *fl_row, const int32_t *bl_row, double a[3], double sa[3], double *dr_out,
                     double *sdr_out)
{
    const double h = p->h, h2 = h * h, two_h = 2.0 * h;
    double dr = 0.0, sdr = 0.0;
    int inter = 0;
    for (int d = 0; d < 3; ++d) a[d] = sa[d] = 0.0;
    if (cell[i] >= 0) {
        const double rhoi = rho[i];
        const double Pi = orc_pressure(p, rhoi);
        const double pi = Pi / (rhoi * rhoi);
        const double ci = orc_sound_speed(p, rhoi);
        const int central_fluid = (info[i] >> 30) == 0u;
        const int total = nfi + nbi;
        for (int k = 0; k < total; ++k) {
            const int j = k < nfi ? fl_row[k] : bl_row[k - nfi];
            double x[3];
            separation(g, cell[i], cell[j], off + 3 * (size_t)i, off + 3 * (size_t)j, x);
            const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            const double r = sqrt(r2);
            if (!(r < two_h)) continue;
            ++inter;
            if (p->kernel == ORC_QUADRATIC && r == 0.0) continue;
            const double F = orc_kernel_F(p->kernel, r, h);
            const double mj = mass[j];
            const double rhoj = rho[j];
            const double Pj = orc_pressure(p, rhoj);
            double u[3], ux = 0.0, uxabs = 0.0;
            for (int d = 0; d < 3; ++d) {
                u[d] = vel[3 * (size_t)i + d] - vel[3 * (size_t)j + d];
                ux += u[d] * x[d];
                uxabs += fabs(u[d] * x[d]);
            }
            /* pressure factor and continuity weight of the formulation */
            double pres, spres, wc;
            if (p->formulation == 1) {
                pres = (Pi + Pj) / (rhoi * rhoj);
                spres = (fabs(Pi) + fabs(Pj)) / (rhoi * rhoj);
                wc = rhoi / rhoj;
            } else {
                pres = pi + Pj / (rhoj * rhoj);
                spres = fabs(pi) + fabs(Pj / (rhoj * rhoj));
                wc = 1.0;
            }
            dr += wc * mj * ux * F;
            sdr += wc * mj * uxabs * fabs(F);
            if (p->delta != 0.0 && central_fluid && k < nfi) {
                /* density diffusion between fluid particles (Molteni and
                 * Colagrossi): delta h c0 sum_j psi_ij . grad_i W_ij V_j with
                 * psi_ij = 2 (rho_j - rho_i) x_ji / (r^2 + eps h^2) and
                 * grad_i W_ij = F x_ij, so psi . grad W = -2 (rho_j - rho_i) F r^2 / (r^2 + eps h^2) */
                const double dd = -2.0 * p->delta * h * p->c0 * (rhoj - rhoi) * F * r2 /
                                  (r2 + p->eps_visc * h2) * mj / rhoj;
                dr += dd;
                sdr += fabs(dd);
            }
            const double cbar = 0.5 * (ci + orc_sound_speed(p, rhoj));
            const double rhobar = 0.5 * (rhoi + rhoj);
            const double visc_den = rhobar * (r2 + p->eps_visc * h2);
            double Pi_ij = 0.0;
            if (ux < 0.0) Pi_ij = -p->alpha * h * cbar * ux / visc_den;
            const double Pi_abs = p->alpha * h * cbar * uxabs / visc_den;
            const double coef = -mj * (pres + Pi_ij) * F;
            const double scoef = mj * (spres + Pi_abs) * fabs(F);
            for (int d = 0; d < 3; ++d) {
                a[d] += coef * x[d];
                sa[d] += scoef * fabs(x[d]);
            }
            if (p->visc_model == 1) {
                const double lam = 4.0 * p->nu * mj / (rhoi + rhoj) * F;
                for (int d = 0; d < 3; ++d) {
                    a[d] += lam * u[d];
                    sa[d] += fabs(lam * u[d]);
                }
            } else if (p->visc_model == 2) {
                const double lk = ORC_MONAGHAN_K * 4.0 * p->nu * mj / (rhoi + rhoj) * F / (r2 + p->eps_visc * h2);
                for (int d = 0; d < 3; ++d) {
                    a[d] += lk * ux * x[d];
                    sa[d] += fabs(lk) * uxabs * fabs(x[d]);
                }
            }
        }
    }
    *dr_out = dr;
    *sdr_out = sdr;
    return inter;
}

void orc_forces(const orc_params *p, const orc_grid *g, int n,
                const int32_t *cell, const double *off, const double *mass,
                const double *vel, const double *rho, const uint32_t *info,
                const int32_t *nf, const int32_t *nb, const int32_t *fl, const int32_t *bl,
                int max_neibs, double *acc, double *drho, double *s_acc, double *s_drho,
                int64_t *n_inter)
{
    int64_t inter = 0;
#pragma omp parallel for schedule(static) reduction(+ : inter)
    for (int i = 0; i < n; ++i)
        inter += forces_of(p, g, i, cell, off, mass, vel, rho, info, nf[i], nb[i], fl + (size_t)i * max_neibs,
                           bl + (size_t)i * max_neibs, acc + 3 * (size_t)i, s_acc + 3 * (size_t)i, drho + i,
                           s_drho + i);
    if (n_inter) *n_inter = inter;
}

/* The same for particles rows[0..nrows) with row-indexed lists (as produced
 * by orc_neighbors_rows) and row-indexed outputs. */
void orc_forces_rows(const orc_params *p, const orc_grid *g, const int32_t *cell, const double *off,
                     const double *mass, const double *vel, const double *rho, const uint32_t *info,
                     const int32_t *rows, int nrows,
                     const int32_t *nf, const int32_t *nb, const int32_t *fl, const int32_t *bl, int max_neibs,
                     double *acc, double *drho, double *s_acc, double *s_drho)
{
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrows; ++r)
        (void)forces_of(p, g, rows[r], cell, off, mass, vel, rho, info, nf[r], nb[r], fl + (size_t)r * max_neibs,
                        bl + (size_t)r * max_neibs, acc + 3 * (size_t)r, s_acc + 3 * (size_t)r, drho + r,
                        s_drho + r);
}

/* Number of listed pairs whose float32 squared separation (evaluated as in
 * the neighbour predicate) is below fl32(2h)^2: the interaction count the
 * GPU uses for its masking decision.  One particle: */
static int64_t count_of(const orc_grid *g, float h, int i, const int32_t *cell, const float *pos4, int nfi,
                        int nbi, const int32_t *fl_row, const int32_t *bl_row)
{
    const float two_h = 2.0f * h;
    const float lim = two_h * two_h;
    int64_t cnt = 0;
    if (cell[i] < 0) return 0;
    int32_t ci[3];
    cell_coords(g, cell[i], ci);
    const int total = nfi + nbi;
    for (int k = 0; k < total; ++k) {
        const int j = k < nfi ? fl_row[k] : bl_row[k - nfi];
        int32_t cj[3];
        cell_coords(g, cell[j], cj);
        float x[3];
        for (int d = 0; d < 3; ++d) {
            int kd = ci[d] - cj[d];
            if ((g->periodic >> d) & 1u) {
                if (kd > 1) kd -= g->n[d];
                if (kd < -1) kd += g->n[d];
            }
            const float t1 = pos4[4 * (size_t)i + d] - pos4[4 * (size_t)j + d];
            const float t2 = (float)kd * g->cs[d];
            x[d] = t2 + t1;
        }
        const float xx = x[0] * x[0];
        const float yy = x[1] * x[1];
        const float zz = x[2] * x[2];
        const float s = xx + yy;
        const float r2 = s + zz;
        if (r2 < lim) ++cnt;
    }
    return cnt;
}

int64_t orc_count_interactions_f32(const orc_grid *g, float h, int n, const int32_t *cell,
                                   const float *pos4, const int32_t *nf, const int32_t *nb,
                                   const int32_t *fl, const int32_t *bl, int max_neibs)
{
    int64_t cnt = 0;
#pragma omp parallel for schedule(static) reduction(+ : cnt)
    for (int i = 0; i < n; ++i)
        cnt += count_of(g, h, i, cell, pos4, nf[i], nb[i], fl + (size_t)i * max_neibs, bl + (size_t)i * max_neibs);
    return cnt;
}

/* The same over particles rows[0..nrows) with row-indexed lists. */
int64_t orc_count_interactions_rows(const orc_grid *g, float h, const int32_t *cell, const float *pos4,
                                    const int32_t *rows, int nrows, const int32_t *nf, const int32_t *nb,
                                    const int32_t *fl, const int32_t *bl, int max_neibs)
{
    int64_t cnt = 0;
#pragma omp parallel for schedule(static) reduction(+ : cnt)
    for (int r = 0; r < nrows; ++r)
        cnt += count_of(g, h, rows[r], cell, pos4, nf[r], nb[r], fl + (size_t)r * max_neibs,
                        bl + (size_t)r * max_neibs);
    return cnt;
}

/* ------------------------------------------------------------------------
 * Explicit midpoint predictor / corrector.
 *   stage 0: y* = y^n + dt/2 f(y^n)
 *   stage 1: y^{n+1} = y^n + dt f(y*)   (positions advance with u*)
 * f = (u, a + g, Drho/Dt) for fluid; boundary particles only advance rho.
 * vel_star is the stage-0 result (used by stage 1 only).
 * ------------------------------------------------------------------------ */
void orc_integrate(const orc_params *p, int stage, double dt, int n,
                   const int32_t *cell, const uint32_t *info,
                   const double *off_n, const double *vel_n, const double *rho_n,
                   const double *vel_star, const double *acc, const double *drho,
                   double *off_out, double *vel_out, double *rho_out)
{
    const double tau = stage == 0 ? 0.5 * dt : dt;
    const double *uadv = stage == 0 ? vel_n : vel_star;
    for (int i = 0; i < n; ++i) {
        const int fluid = ptype(info[i]) != ORC_BOUNDARY && cell[i] >= 0;
        for (int d = 0; d < 3; ++d) {
            const size_t q = 3 * (size_t)i + d;
            if (fluid) {
                off_out[q] = off_n[q] + tau * uadv[q];
                vel_out[q] = vel_n[q] + tau * (acc[q] + p->g[d]);
            } else {
                off_out[q] = off_n[q];
                vel_out[q] = vel_n[q];
            }
        }
        rho_out[i] = cell[i] >= 0 ? rho_n[i] + tau * drho[i] : rho_n[i];
    }
}

/* dt = CFL min(h / max c, sqrt(h / max |a + g|) [, 0.125 h^2 / nu]) over fluid. */
double orc_dt(const orc_params *p, int n, const int32_t *cell, const uint32_t *info,
              const double *rho, const double *acc)
{
    double cmax = 0.0, amax = 0.0;
    for (int i = 0; i < n; ++i) {
        if (cell[i] < 0 || ptype(info[i]) == ORC_BOUNDARY) continue;
        const double c = orc_sound_speed(p, rho[i]);
        if (c > cmax) cmax = c;
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double v = acc[3 * (size_t)i + d] + p->g[d];
            s += v * v;
        }
        const double a = sqrt(s);
        if (a > amax) amax = a;
    }
    double dt = INFINITY;
    if (cmax > 0.0) dt = p->h / cmax;
    if (amax > 0.0) { const double t = sqrt(p->h / amax); if (t < dt) dt = t; }
    if (p->nu > 0.0) { const double t = 0.125 * p->h * p->h / p->nu; if (t < dt) dt = t; }
    return p->cfl * dt;
}

/* ------------------------------------------------------------------------
 * Reverse (adjoint) of orc_forces with the lists held fixed.
 *
 * Forward pair term of central c and neighbour n (r < 2h), x = x_c - x_n,
 * u = u_c - u_n, w = u . x:
 *   a_c += G x + Lm u + Lk x,   Drho_c += Wc m_n F w,
 *   G  = -m_n (S_p + Pi) F,
 *   S_p = P_c/rho_c^2 + P_n/rho_n^2, Wc = 1              (golden rule)
 *   S_p = (P_c + P_n)/(rho_c rho_n), Wc = rho_c/rho_n    (Landrini-Morris)
 *   Pi = K_a min(w, 0) / (r^2 + eps h^2),  K_a = -alpha h (c_c + c_n)/(rho_c + rho_n),
 *   Lm = 4 nu m_n F/(rho_c + rho_n)                        (Morris)
 *   Lk = K 4 nu m_n F w/((rho_c + rho_n)(r^2 + eps h^2))  (Monaghan K form),
 * plus the density diffusion of orc_forces.  Given the upstream adjoints
 * abar_c (3) and dbar_c of every central, the derivative of
 * T = abar_c . a_pair + dbar_c Drho_pair with respect to x, u, rho_c, rho_n
 * and (alpha, c0, nu) is formed and scattered: +x/+u to the central, -x/-u
 * to the neighbour.  The switch of Pi at w = 0 takes the derivative of the
 * active branch (zero at w = 0).
 * Results are ADDED to go [n,3], gu [n,3], grho [n] and gparams[3].
 * ------------------------------------------------------------------------ */
void orc_forces_reverse(const orc_params *p, const orc_grid *g, int n,
                        const int32_t *cell, const double *off, const double *mass,
                        const double *vel, const double *rho, const uint32_t *info,
                        const int32_t *nf, const int32_t *nb, const int32_t *fl, const int32_t *bl,
                        int max_neibs, const double *abar, const double *dbar,
                        double *go, double *gu, double *grho, double *gparams)
{
    const double h = p->h, two_h = 2.0 * h, eh2 = p->eps_visc * h * h;
    const int form2 = p->formulation == 1;
    double galpha = 0.0, gc0 = 0.0, gnu = 0.0;
    for (int c = 0; c < n; ++c) {
        if (cell[c] < 0) continue;
        const double rc = rho[c];
        const double Pc = orc_pressure(p, rc);
        const double pc = Pc / (rc * rc);
        const double cc = orc_sound_speed(p, rc);
        /* dP/drho = c^2; d(P/rho^2)/drho = c^2/rho^2 - 2P/rho^3; dc/drho = (gamma-1)/2 c/rho */
        const double dpc = cc * cc / (rc * rc) - 2.0 * Pc / (rc * rc * rc);
        const double dcc = 0.5 * (p->gamma - 1.0) * cc / rc;
        const double *ab = abar + 3 * (size_t)c;
        const double db = dbar[c];
        const int total = nf[c] + nb[c];
        const int central_fluid = ptype(info[c]) != ORC_BOUNDARY;
        for (int k = 0; k < total; ++k) {
            const int m = k < nf[c] ? fl[(size_t)c * max_neibs + k]
                                    : bl[(size_t)c * max_neibs + (k - nf[c])];
            double x[3], u[3];
            separation(g, cell[c], cell[m], off + 3 * (size_t)c, off + 3 * (size_t)m, x);
            const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            const double r = sqrt(r2);
            if (!(r < two_h)) continue;
            if (p->kernel == ORC_QUADRATIC && r == 0.0) continue;
            for (int d = 0; d < 3; ++d) u[d] = vel[3 * (size_t)c + d] - vel[3 * (size_t)m + d];
            const double w = u[0] * x[0] + u[1] * x[1] + u[2] * x[2];
            const double F = orc_kernel_F(p->kernel, r, h);
            const double dFdr = orc_kernel_dF(p->kernel, r, h);
            const double mn = mass[m];
            const double rn = rho[m];
            const double Pn = orc_pressure(p, rn);
            const double pn = Pn / (rn * rn);
            const double cn = orc_sound_speed(p, rn);
            const double dpn = cn * cn / (rn * rn) - 2.0 * Pn / (rn * rn * rn);
            const double dcn = 0.5 * (p->gamma - 1.0) * cn / rn;
            const double rs = rc + rn;
            const double dd = r2 + eh2;
            const int act = w < 0.0;
            const double mw = act ? w : 0.0;
            const double K = -p->alpha * h * (cc + cn) / rs;
            const double Pi = K * mw / dd;
            /* pressure factor, its rho derivatives, continuity weight */
            double Sp, dSp_drc, dSp_drn, Wc, dWc_drc, dWc_drn;
            if (form2) {
                Sp = (Pc + Pn) / (rc * rn);
                dSp_drc = cc * cc / (rc * rn) - Sp / rc;
                dSp_drn = cn * cn / (rc * rn) - Sp / rn;
                Wc = rc / rn;
                dWc_drc = 1.0 / rn;
                dWc_drn = -rc / (rn * rn);
            } else {
                Sp = pc + pn;
                dSp_drc = dpc;
                dSp_drn = dpn;
                Wc = 1.0;
                dWc_drc = dWc_drn = 0.0;
            }
            const double S = Sp + Pi;
            const double G = -mn * S * F;
            const double Lm = p->visc_model == 1 ? 4.0 * p->nu * mn * F / rs : 0.0;
            const double kk = p->visc_model == 2 ? ORC_MONAGHAN_K * 4.0 * p->nu * mn / rs : 0.0;
            const double Lk = kk * F * w / dd;
            const double A = ab[0] * x[0] + ab[1] * x[1] + ab[2] * x[2];
            const double Bu = ab[0] * u[0] + ab[1] * u[1] + ab[2] * u[2];
            double gx[3], gv[3];
            for (int d = 0; d < 3; ++d) {
                const double dFdx = dFdr * x[d] / r;
                const double dPidx = act ? K * (u[d] / dd - 2.0 * w * x[d] / (dd * dd)) : 0.0;
                const double dPidu = act ? K * x[d] / dd : 0.0;
                const double dGdx = -mn * (S * dFdx + F * dPidx);
                const double dGdu = -mn * F * dPidu;
                const double dLdx = p->visc_model == 1 ? 4.0 * p->nu * mn * dFdx / rs : 0.0;
                const double dLkdx = kk * (dFdx * w / dd + F * u[d] / dd - 2.0 * F * w * x[d] / (dd * dd));
                const double dLkdu = kk * F * x[d] / dd;
                gx[d] = (G + Lk) * ab[d] + A * (dGdx + dLkdx) + Bu * dLdx + db * Wc * mn * (F * u[d] + w * dFdx);
                gv[d] = Lm * ab[d] + A * (dGdu + dLkdu) + db * Wc * mn * F * x[d];
            }
            const double dPi_drc = act ? -p->alpha * h * mw / dd * (dcc / rs - (cc + cn) / (rs * rs)) : 0.0;
            const double dPi_drn = act ? -p->alpha * h * mw / dd * (dcn / rs - (cc + cn) / (rs * rs)) : 0.0;
            const double dL_drho = p->visc_model == 1 ? -4.0 * p->nu * mn * F / (rs * rs) : 0.0;
            const double dLk_drho = -Lk / rs;
            const double grc = A * (-mn * F * (dSp_drc + dPi_drc) + dLk_drho) + Bu * dL_drho +
                               db * dWc_drc * mn * w * F;
            const double grn = A * (-mn * F * (dSp_drn + dPi_drn) + dLk_drho) + Bu * dL_drho +
                               db * dWc_drn * mn * w * F;
            for (int d = 0; d < 3; ++d) {
                go[3 * (size_t)c + d] += gx[d];
                go[3 * (size_t)m + d] -= gx[d];
                gu[3 * (size_t)c + d] += gv[d];
                gu[3 * (size_t)m + d] -= gv[d];
            }
            grho[c] += grc;
            grho[m] += grn;
            /* Pi is proportional to alpha and to c0; the pressure factor to c0^2 */
            const double Pi_over_alpha = -h * (cc + cn) / rs * mw / dd;
            galpha += A * (-mn * F) * Pi_over_alpha;
            gc0 += A * (-mn * F) * (2.0 * Sp + Pi) / p->c0;
            if (p->visc_model == 1) gnu += Bu * 4.0 * mn * F / rs;
            if (p->visc_model == 2) gnu += A * ORC_MONAGHAN_K * 4.0 * mn / rs * F * w / dd;
            if (p->delta != 0.0 && central_fluid && k < nf[c]) {
                /* density diffusion, term = cD m_n (rho_c - rho_n)/rho_n Gd(r),
                 * Gd = F r^2 / (r^2 + eps h^2), cD = 2 delta h c0 */
                const double cD = 2.0 * p->delta * h * p->c0;
                const double Gd = F * r2 / dd;
                const double dGd_r = dFdr / r * r2 / dd + 2.0 * F * eh2 / (dd * dd); /* Gd'(r) / r */
                const double ratio = (rc - rn) / rn;
                for (int d = 0; d < 3; ++d) {
                    const double t = db * cD * mn * ratio * dGd_r * x[d];
                    go[3 * (size_t)c + d] += t;
                    go[3 * (size_t)m + d] -= t;
                }
                grho[c] += db * cD * mn * Gd / rn;
                grho[m] += db * cD * mn * Gd * (-rc / (rn * rn));
                gc0 += db * cD * mn * ratio * Gd / p->c0;
            }
        }
    }
    gparams[0] += galpha;
    gparams[1] += gc0;
    gparams[2] += gnu;
}

/* Magnitude scales of orc_forces_reverse, for error gates: the reverse pass
 * evaluated with every factor replaced by its absolute value (sums of
 * products become sums of absolute products, u.x becomes sum |u_d x_d|), on
 * the same pairs and active branches, scattered to the central and the
 * neighbour alike.  A float evaluation of the reverse in any order has an
 * error of a few units of rounding times these scales.  Results are ADDED to
 * so [n,3], su [n,3], srho [n] and sparams[3]. */
void orc_forces_reverse_scales(const orc_params *p, const orc_grid *g, int n,
                               const int32_t *cell, const double *off, const double *mass,
                               const double *vel, const double *rho, const uint32_t *info,
                               const int32_t *nf, const int32_t *nb, const int32_t *fl, const int32_t *bl,
                               int max_neibs, const double *abar, const double *dbar,
                               double *so, double *su, double *srho, double *sparams)
{
    const double h = p->h, two_h = 2.0 * h, eh2 = p->eps_visc * h * h;
    const int form2 = p->formulation == 1;
    double salpha = 0.0, sc0 = 0.0, snu = 0.0;
    for (int c = 0; c < n; ++c) {
        if (cell[c] < 0) continue;
        const double rc = rho[c];
        const double Pc = orc_pressure(p, rc);
        const double cc = orc_sound_speed(p, rc);
        const double dpc = cc * cc / (rc * rc) + 2.0 * fabs(Pc) / (rc * rc * rc);
        const double dcc = 0.5 * (p->gamma - 1.0) * cc / rc;
        const double *ab = abar + 3 * (size_t)c;
        const double db = fabs(dbar[c]);
        const int total = nf[c] + nb[c];
        const int central_fluid = ptype(info[c]) != ORC_BOUNDARY;
        for (int k = 0; k < total; ++k) {
            const int m = k < nf[c] ? fl[(size_t)c * max_neibs + k]
                                    : bl[(size_t)c * max_neibs + (k - nf[c])];
            double x[3], u[3];
            separation(g, cell[c], cell[m], off + 3 * (size_t)c, off + 3 * (size_t)m, x);
            const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            const double r = sqrt(r2);
            if (!(r < two_h)) continue;
            if (p->kernel == ORC_QUADRATIC && r == 0.0) continue;
            double w = 0.0, wa = 0.0, A = 0.0, Bu = 0.0;
            for (int d = 0; d < 3; ++d) {
                u[d] = vel[3 * (size_t)c + d] - vel[3 * (size_t)m + d];
                w += u[d] * x[d];
                wa += fabs(u[d] * x[d]);
                A += fabs(ab[d] * x[d]);
                Bu += fabs(ab[d] * u[d]);
            }
            const double F = fabs(orc_kernel_F(p->kernel, r, h));
            const double dFdr = fabs(orc_kernel_dF(p->kernel, r, h));
            const double mn = mass[m];
            const double rn = rho[m];
            const double Pn = orc_pressure(p, rn);
            const double cn = orc_sound_speed(p, rn);
            const double dpn = cn * cn / (rn * rn) + 2.0 * fabs(Pn) / (rn * rn * rn);
            const double dcn = 0.5 * (p->gamma - 1.0) * cn / rn;
            const double rs = rc + rn;
            const double dd = r2 + eh2;
            const int act = w < 0.0;
            const double K = p->alpha * h * (cc + cn) / rs;
            const double Pi = act ? K * wa / dd : 0.0;
            double Sp, dSp_drc, dSp_drn, Wc, dWc_drc, dWc_drn;
            if (form2) {
                Sp = (fabs(Pc) + fabs(Pn)) / (rc * rn);
                dSp_drc = cc * cc / (rc * rn) + Sp / rc;
                dSp_drn = cn * cn / (rc * rn) + Sp / rn;
                Wc = rc / rn;
                dWc_drc = 1.0 / rn;
                dWc_drn = rc / (rn * rn);
            } else {
                Sp = fabs(Pc) / (rc * rc) + fabs(Pn) / (rn * rn);
                dSp_drc = dpc;
                dSp_drn = dpn;
                Wc = 1.0;
                dWc_drc = dWc_drn = 0.0;
            }
            const double S = Sp + Pi;
            const double G = mn * S * F;
            const double Lm = p->visc_model == 1 ? 4.0 * p->nu * mn * F / rs : 0.0;
            const double kk = p->visc_model == 2 ? ORC_MONAGHAN_K * 4.0 * p->nu * mn / rs : 0.0;
            const double Lk = kk * F * wa / dd;
            double sx[3], sv[3];
            for (int d = 0; d < 3; ++d) {
                const double ax = fabs(x[d]), au = fabs(u[d]), aab = fabs(ab[d]);
                const double dFdx = dFdr * ax / r;
                const double dPidx = act ? K * (au / dd + 2.0 * wa * ax / (dd * dd)) : 0.0;
                const double dPidu = act ? K * ax / dd : 0.0;
                const double dGdx = mn * (S * dFdx + F * dPidx);
                const double dGdu = mn * F * dPidu;
                const double dLdx = p->visc_model == 1 ? 4.0 * p->nu * mn * dFdx / rs : 0.0;
                const double dLkdx = kk * (dFdx * wa / dd + F * au / dd + 2.0 * F * wa * ax / (dd * dd));
                const double dLkdu = kk * F * ax / dd;
                sx[d] = (G + Lk) * aab + A * (dGdx + dLkdx) + Bu * dLdx + db * Wc * mn * (F * au + wa * dFdx);
                sv[d] = Lm * aab + A * (dGdu + dLkdu) + db * Wc * mn * F * ax;
            }
            const double dPi_drc = act ? p->alpha * h * wa / dd * (dcc / rs + (cc + cn) / (rs * rs)) : 0.0;
            const double dPi_drn = act ? p->alpha * h * wa / dd * (dcn / rs + (cc + cn) / (rs * rs)) : 0.0;
            const double dL_drho = p->visc_model == 1 ? 4.0 * p->nu * mn * F / (rs * rs) : 0.0;
            const double dLk_drho = Lk / rs;
            const double src = A * (mn * F * (dSp_drc + dPi_drc) + dLk_drho) + Bu * dL_drho + db * dWc_drc * mn * wa * F;
            const double srn = A * (mn * F * (dSp_drn + dPi_drn) + dLk_drho) + Bu * dL_drho + db * dWc_drn * mn * wa * F;
            for (int d = 0; d < 3; ++d) {
                so[3 * (size_t)c + d] += sx[d];
                so[3 * (size_t)m + d] += sx[d];
                su[3 * (size_t)c + d] += sv[d];
                su[3 * (size_t)m + d] += sv[d];
            }
            srho[c] += src;
            srho[m] += srn;
            salpha += act ? A * mn * F * h * (cc + cn) / rs * wa / dd : 0.0;
            sc0 += A * mn * F * (2.0 * Sp + Pi) / p->c0;
            if (p->visc_model == 1) snu += Bu * 4.0 * mn * F / rs;
            if (p->visc_model == 2) snu += A * ORC_MONAGHAN_K * 4.0 * mn / rs * F * wa / dd;
            if (p->delta != 0.0 && central_fluid && k < nf[c]) {
                const double cD = 2.0 * p->delta * h * p->c0;
                const double Gd = F * r2 / dd;
                const double dGd_r = dFdr / r * r2 / dd + 2.0 * F * eh2 / (dd * dd);
                const double ratio = fabs(rc - rn) / rn;
                for (int d = 0; d < 3; ++d) {
                    const double t = db * cD * mn * ratio * dGd_r * fabs(x[d]);
                    so[3 * (size_t)c + d] += t;
                    so[3 * (size_t)m + d] += t;
                }
                srho[c] += db * cD * mn * Gd / rn;
                srho[m] += db * cD * mn * Gd * rc / (rn * rn);
                sc0 += db * cD * mn * ratio * Gd / p->c0;
            }
        }
    }
    sparams[0] += salpha;
    sparams[1] += sc0;
    sparams[2] += snu;
}

/* Reverse of orc_integrate.  Given the adjoint of the stage output
 * (go_out, gu_out, grho_out), return the adjoint of the stage inputs:
 *   stage 0 (y* = y + tau f(y), tau = dt/2):
 *       go_n = go_out, gu_n = gu_out + tau go_out (fluid), grho_n = grho_out,
 *       abar = tau gu_out (fluid), dbar = tau grho_out;
 *   stage 1 (y^{n+1} = y^n + dt (u*, a* + g, D*)):
 *       go_n = go_out, gu_n = gu_out, grho_n = grho_out,
 *       gu_star = dt go_out (fluid), abar = dt gu_out (fluid), dbar = dt grho_out.
 * The derivative contributions through abar/dbar are added by the caller via
 * orc_forces_reverse.  Outputs are overwritten. */
void orc_integrate_reverse(int stage, double dt, int n, const int32_t *cell, const uint32_t *info,
                           const double *go_out, const double *gu_out, const double *grho_out,
                           double *go_n, double *gu_n, double *grho_n, double *gu_star,
                           double *abar, double *dbar)
{
    const double tau = stage == 0 ? 0.5 * dt : dt;
    for (int i = 0; i < n; ++i) {
        const int fluid = ptype(info[i]) != ORC_BOUNDARY && cell[i] >= 0;
        for (int d = 0; d < 3; ++d) {
            const size_t q = 3 * (size_t)i + d;
            go_n[q] = go_out[q];
            if (stage == 0) {
                gu_n[q] = gu_out[q] + (fluid ? tau * go_out[q] : 0.0);
            } else {
                gu_n[q] = gu_out[q];
                if (gu_star) gu_star[q] = fluid ? dt * go_out[q] : 0.0;
            }
            abar[q] = fluid ? tau * gu_out[q] : 0.0;
        }
        grho_n[i] = grho_out[i];
        dbar[i] = cell[i] >= 0 ? tau * grho_out[i] : 0.0;
    }
}
