/*
 * soc_oracle.c -- FP64 CPU oracle for the SOC Monte Carlo hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see soc_oracle.h).  Plain C99 + optional
 * OpenMP over independent photon packages.  Every quantity is computed in
 * double precision; leaf lookup is a brute-force descent from the root at
 * every step, so this file never uses the neighbour stepping of the GPU
 * library.  Paper: Juvela 2019, arXiv:1812.06632 (section numbers cited at
 * each function).
 */
#include "soc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018, cgs. */
#define ORC_H     6.62607015e-27     /* erg s */
#define ORC_K     1.380649e-16       /* erg / K */
#define ORC_C     2.99792458e10      /* cm / s */
#define ORC_PI    3.14159265358979323846
#define ORC_EPS_PUSH 1e-9            /* lookup push along u, root units */
#define ORC_WFLOOR   1e-12           /* weight floor relative to W0 */

/* ------------------------------------------------------------------ */
/* Philox4x32-10, Salmon, Moraes, Dror & Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11: ten rounds of two 32x32->64 multiplies with
 * the published multipliers and Weyl key increments. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double orc_u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

/* One stream per package: counter = (block, package id, frequency index,
 * iteration<<8 | source class), key = (seed low word, seed high word). */
typedef struct { uint32_t ctr[4], key[2], buf[4]; int used; } stream_t;

static void stream_init(stream_t *s, uint64_t seed, uint32_t iteration, uint32_t cls,
                        uint32_t freq_index, uint32_t pid)
{
    s->ctr[0] = 0; s->ctr[1] = pid; s->ctr[2] = freq_index; s->ctr[3] = (iteration << 8) | (cls & 0xffu);
    s->key[0] = (uint32_t)seed; s->key[1] = (uint32_t)(seed >> 32);
    orc_philox4x32_10(s->ctr, s->key, s->buf);
    s->used = 0;
}

static double stream_next(stream_t *s)
{
    if (s->used == 4) {
        s->ctr[0] += 1;
        orc_philox4x32_10(s->ctr, s->key, s->buf);
        s->used = 0;
    }
    return orc_u01(s->buf[s->used++]);
}

void orc_uniforms(uint64_t seed, uint32_t iteration, uint32_t cls, uint32_t freq_index,
                  uint32_t package_id, int32_t n, double *out)
{
    stream_t s;
    stream_init(&s, seed, iteration, cls, freq_index, package_id);
    for (int32_t i = 0; i < n; ++i) out[i] = stream_next(&s);
}

/* ------------------------------------------------------------------ */
/* Planck law B_nu(T) = (2 h nu^3 / c^2) / (exp(h nu / k T) - 1). */
double orc_planck(double nu, double T)
{
    if (!(T > 0.0)) return 0.0;
    double x = ORC_H * nu / (ORC_K * T);
    double pre = 2.0 * ORC_H * nu * nu * nu / (ORC_C * ORC_C);
    if (x > 700.0) return pre * exp(-x);
    return pre / expm1(x);
}

/* Absorbed power per H atom of grains at temperature T in equilibrium,
 * 4 pi sum_k w_k sigma_abs(nu_k) B_nu_k(T): the left side of the
 * energy balance that the temperature kernel inverts (Sect. 2.1.1). */
double orc_gamma(const orc_freq *f, int32_t K, double T)
{
    double s = 0.0;
    for (int32_t k = 0; k < K; ++k) s += f[k].w_nu * f[k].sigma_abs * orc_planck(f[k].nu, T);
    return 4.0 * ORC_PI * s;
}

/* ------------------------------------------------------------------ */
/* Grid (Sect. 2.1.1): root cells first (x fastest), then each level; a
 * refined cell stores -(index of first child); octets are consecutive with
 * child octant o = ix + 2 iy + 4 iz. */
static inline int32_t word_i(const orc_grid *g, int64_t c) { return (int32_t)g->words[c]; }
static inline double word_f(const orc_grid *g, int64_t c)
{
    float v; uint32_t w = g->words[c];
    memcpy(&v, &w, 4);
    return (double)v;
}

static int cell_level(const orc_grid *g, int64_t c)
{
    for (int L = 0; L < g->nlevels; ++L)
        if (c >= g->level_offset[L] && c < g->level_offset[L + 1]) return L;
    return -1;
}

int64_t orc_leaf(const orc_grid *g, const double p[3], double lo[3], double *size)
{
    if (!(p[0] >= 0.0 && p[0] < g->nx && p[1] >= 0.0 && p[1] < g->ny && p[2] >= 0.0 && p[2] < g->nz))
        return -1;
    int64_t ix = (int64_t)floor(p[0]), iy = (int64_t)floor(p[1]), iz = (int64_t)floor(p[2]);
    int64_t c = ix + (int64_t)g->nx * (iy + (int64_t)g->ny * iz);
    double l0 = (double)ix, l1 = (double)iy, l2 = (double)iz, sz = 1.0;
    while (word_i(g, c) < 0) {
        int64_t first = -(int64_t)word_i(g, c);
        sz *= 0.5;
        int ox = p[0] >= l0 + sz, oy = p[1] >= l1 + sz, oz = p[2] >= l2 + sz;
        l0 += ox * sz; l1 += oy * sz; l2 += oz * sz;
        c = first + ox + 2 * oy + 4 * oz;
    }
    lo[0] = l0; lo[1] = l1; lo[2] = l2; *size = sz;
    return c;
}

int32_t orc_validate_grid(const orc_grid *g)
{
    if (!g || !g->words || !g->level_offset) return -1;
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->nlevels < 1) return -1;
    if (!(g->root_cell_cm > 0.0)) return -1;
    int64_t nroot = (int64_t)g->nx * g->ny * g->nz;
    if (g->level_offset[0] != 0 || g->level_offset[1] != nroot) return -2;
    for (int L = 1; L <= g->nlevels; ++L) {
        if (g->level_offset[L] < g->level_offset[L - 1]) return -2;
        if (L >= 2 && (g->level_offset[L] - g->level_offset[L - 1]) % 8 != 0) return -2;
    }
    if (g->level_offset[g->nlevels] != g->ncells) return -2;
    char *seen = (char *)calloc((size_t)(g->ncells / 8 + 1), 1);
    if (!seen) return -3;
    int32_t rc = 0;
    for (int64_t c = 0; c < g->ncells && rc == 0; ++c) {
        int32_t w = word_i(g, c);
        if (w < 0) {
            int L = cell_level(g, c);
            int64_t first = -(int64_t)w;
            if (L + 1 >= g->nlevels) { rc = -4; break; }
            int64_t a = g->level_offset[L + 1], b = g->level_offset[L + 2];
            if (first < a || first + 8 > b || (first - a) % 8 != 0) { rc = -4; break; }
            int64_t oct = (first - nroot) / 8;
            if (seen[oct]) { rc = -4; break; }
            seen[oct] = 1;
        } else {
            double v = word_f(g, c);
            if (!isfinite(v) || v < 0.0) { rc = -5; break; }
        }
    }
    if (rc == 0) {
        int64_t noct = (g->ncells - nroot) / 8;
        for (int64_t o = 0; o < noct; ++o)
            if (!seen[o]) { rc = -4; break; }
    }
    free(seen);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Henyey-Greenstein scattering (analytic inversion of the HG cumulative
 * distribution) followed by the exact rotation of the direction about the
 * old one by polar angle acos(mu) and azimuth phi (the z-axis formula is
 * used only when the old direction is the z axis itself). */
static void scatter_dir(double g, double xi_mu, double xi_phi, double u[3])
{
    double mu;
    if (fabs(g) < 1e-4) {
        mu = 2.0 * xi_mu - 1.0;
    } else {
        double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * xi_mu);
        mu = (1.0 + g * g - s * s) / (2.0 * g);
    }
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = 2.0 * ORC_PI * xi_phi;
    double cp = cos(phi), sp = sin(phi);
    double ux = u[0], uy = u[1], uz = u[2], n0, n1, n2;
    double t2 = ux * ux + uy * uy;   /* squared transverse length of the old direction */
    if (t2 < 1e-30) {
        n0 = st * cp;
        n1 = st * sp;
        n2 = (uz >= 0.0 ? 1.0 : -1.0) * mu;
    } else {
        double t = sqrt(t2);
        n0 = st * (ux * uz * cp - uy * sp) / t + ux * mu;
        n1 = st * (uy * uz * cp + ux * sp) / t + uy * mu;
        n2 = -st * cp * t + uz * mu;
    }
    double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    u[0] = n0 / nn; u[1] = n1 / nn; u[2] = n2 / nn;
}

void orc_hg_scatter(double g, const double u0[3], int32_t n, const double *xi, double *out3n)
{
    for (int32_t i = 0; i < n; ++i) {
        double u[3] = {u0[0], u0[1], u0[2]};
        scatter_dir(g, xi[2 * i], xi[2 * i + 1], u);
        out3n[3 * i] = u[0]; out3n[3 * i + 1] = u[1]; out3n[3 * i + 2] = u[2];
    }
}

static void iso_dir(double xi_mu, double xi_phi, double u[3])
{
    double mu = 2.0 * xi_mu - 1.0;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = 2.0 * ORC_PI * xi_phi;
    u[0] = st * cos(phi); u[1] = st * sin(phi); u[2] = mu;
}

/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t steps, scatterings, runaway;
    double escaped, path;
} pk_tally;

/* Transport of one package from (p,u) with weight W0 and remaining free
 * path tau in scattering optical depth: the per-cell loop of Sect. 2.1.1.
 * In each leaf the distance to the exit face is compared with the
 * distance to the next scattering; the segment deposits W (1 - e^{-k_abs d})
 * in the leaf; the package crosses, scatters (HG), escapes the box, falls
 * under the weight floor or hits the step cap. */
static void transport(const orc_grid *g, const orc_freq *f, double p[3], double u[3], double W0,
                      double tau, stream_t *rs, int64_t cap, double *absorbed, int64_t *hits, pk_tally *t,
                      orc_segment *seg, int32_t max_seg, int32_t *nseg, int64_t origin, double *self_abs)
{
    double W = W0;
    const double s_cm = g->root_cell_cm;
    for (;;) {
        double q[3] = {p[0] + ORC_EPS_PUSH * u[0], p[1] + ORC_EPS_PUSH * u[1], p[2] + ORC_EPS_PUSH * u[2]};
        double lo[3], size;
        int64_t c = orc_leaf(g, q, lo, &size);
        if (c < 0) { t->escaped += W; return; }
        double dexit = INFINITY;
        for (int i = 0; i < 3; ++i) {
            double d = INFINITY;
            if (u[i] > 0.0) d = (lo[i] + size - p[i]) / u[i];
            else if (u[i] < 0.0) d = (lo[i] - p[i]) / u[i];
            if (d < 0.0) d = 0.0;
            if (d < dexit) dexit = d;
        }
        double n = word_f(g, c);
        double ks = f->sigma_sca * n * s_cm, ka = f->sigma_abs * n * s_cm;
        int ev;
        double d;
        if (ks > 0.0 && ks * dexit >= tau) {
            d = tau / ks;
            if (d > dexit) d = dexit;
            ev = ORC_SCATTER;
        } else {
            d = dexit;
            tau -= ks * dexit;
            ev = ORC_CROSS;
        }
        /* deposits of a dust package in its own emitting cell are counted
         * apart for diagonal ALI */
        double *dst = (self_abs && c == origin) ? self_abs : absorbed;
        double dep = W * (-expm1(-ka * d));
        if (dst && dep != 0.0) dst[c] += dep;
        if (hits && dep != 0.0) hits[c] += 1;
        W -= dep;
        p[0] += d * u[0]; p[1] += d * u[1]; p[2] += d * u[2];
        t->steps++;
        t->path += d;
        if (ev == ORC_CROSS) {
            double q2[3] = {p[0] + ORC_EPS_PUSH * u[0], p[1] + ORC_EPS_PUSH * u[1], p[2] + ORC_EPS_PUSH * u[2]};
            double lo2[3], sz2;
            if (orc_leaf(g, q2, lo2, &sz2) < 0) ev = ORC_ESCAPE;
        }
        if (ev != ORC_ESCAPE && fabs(W) < ORC_WFLOOR * fabs(W0)) {
            if (dst) dst[c] += W;
            W = 0.0;
            ev = ORC_FLOOR;
        } else if (ev != ORC_ESCAPE && (int64_t)t->steps >= cap) {
            if (dst) dst[c] += W;
            W = 0.0;
            ev = ORC_RUNAWAY;
            t->runaway++;
        }
        if (seg && nseg && *nseg < max_seg) {
            seg[*nseg].cell = c; seg[*nseg].ds = d; seg[*nseg].event = ev;
        }
        if (nseg) (*nseg)++;
        if (ev == ORC_ESCAPE) { t->escaped += W; return; }
        if (ev == ORC_FLOOR || ev == ORC_RUNAWAY) return;
        if (ev == ORC_SCATTER) {
            double xm = stream_next(rs), xp = stream_next(rs);
            scatter_dir(f->g, xm, xp, u);
            tau = -log(stream_next(rs));
            t->scatterings++;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Per-frequency source setup: energies of the source classes (Sect. 2.2,
 * 3.1, 3.2).  Background: pi I_bg w A_box entering through the box faces.
 * Point source: L_nu w.  Dust cell c: 4 pi sigma_abs n_c V_c B_nu(T_c) w. */
typedef struct {
    const orc_grid *g;
    const orc_freq *f;
    const orc_sources *s;
    uint64_t seed;
    uint32_t iteration, freq_index;
    int64_t cap;
    double E_bg, W_bg;
    double *L;          /* dust luminosity per cell, or its difference to the reference
                           (mode 2); NULL if no dust */
    double *incl;       /* inclusive cumulative sum of the expected package counts
                           (modes 1, 2; in units of |L| when there is no cap) */
    double S;           /* sum of |L| */
    double X_total;     /* capped: expected package total, sum of the capped counts */
    int64_t last_pos;   /* last cell with L > 0 */
    int64_t *leaves;    /* leaf cells in index order */
    int64_t nleaves;
    uint64_t per_leaf;
    double u_sys;       /* systematic offset of the weighted draw */
    double *cell_lo;    /* lower corner of every cell, root units (dust only) */
    uint64_t n_total;
} sim_ctx;

static double cell_volume(const orc_grid *g, int64_t c)
{
    int L = cell_level(g, c);
    double s = g->root_cell_cm * ldexp(1.0, -L);
    return s * s * s;
}

static double box_area_root(const orc_grid *g)
{
    return 2.0 * ((double)g->ny * g->nz + (double)g->nx * g->nz + (double)g->nx * g->ny);
}

/* Dust emission per cell at one frequency (Sect. 3.2): 4 pi sigma_abs n V
 * B_nu(T) w in every leaf, 0 in refined cells. */
static void dust_lum(const orc_grid *g, const orc_freq *f, const float *T, double *L)
{
    for (int64_t c = 0; c < g->ncells; ++c) {
        double Lc = 0.0;
        if (word_i(g, c) >= 0) {
            double n = word_f(g, c);
            Lc = 4.0 * ORC_PI * f->sigma_abs * n * cell_volume(g, c) * orc_planck(f->nu, (double)T[c]) * f->w_nu;
        }
        L[c] = Lc;
    }
}

/* Expected number of packages of cell c in the weighted modes: its share
 * N |L_c| / S of the N packages, at most the cap (Sect. 3.2). */
static double expected_count(const sim_ctx *X, int64_t c)
{
    double x = (double)X->s->n_dust * fabs(X->L[c]) / X->S;
    if (X->s->dust_cap > 0.0 && x > X->s->dust_cap) x = X->s->dust_cap;
    return x;
}

int32_t orc_dust_luminosity(const orc_grid *g, const orc_freq *f, const float *T, double *L)
{
    if (!g || !f || !T || !L) return -1;
    if (orc_validate_grid(g) != 0) return -4;
    dust_lum(g, f, T, L);
    return 0;
}

static int32_t sim_setup(sim_ctx *X)
{
    const orc_grid *g = X->g;
    const orc_sources *s = X->s;
    const orc_freq *f = X->f;
    double s2 = g->root_cell_cm * g->root_cell_cm;
    X->E_bg = ORC_PI * s->I_bg_nu * f->w_nu * box_area_root(g) * s2;
    X->W_bg = s->n_bg ? X->E_bg / (double)s->n_bg : 0.0;
    X->L = NULL; X->incl = NULL; X->leaves = NULL; X->cell_lo = NULL; X->S = 0.0; X->nleaves = 0; X->last_pos = -1;
    X->per_leaf = 0; X->u_sys = 0.5;
    if (s->T && s->n_dust) {
        X->L = (double *)malloc(sizeof(double) * (size_t)g->ncells);
        X->incl = (double *)malloc(sizeof(double) * (size_t)g->ncells);
        if (!X->L || !X->incl) return -3;
        dust_lum(g, f, s->T, X->L);
        if (s->dust_mode == 2 && s->L_ref)
            for (int64_t c = 0; c < g->ncells; ++c) X->L[c] -= s->L_ref[c];
        /* selection weight |L|; with a cap, the expected count of cell c is
         * min(N |L_c| / S, cap) and the cumulative sum is in package units */
        double acc = 0.0;
        for (int64_t c = 0; c < g->ncells; ++c) {
            acc += fabs(X->L[c]);
            X->incl[c] = acc;
            if (X->L[c] != 0.0) X->last_pos = c;
        }
        X->S = acc;
        if (s->dust_mode != 0 && s->dust_cap > 0.0 && acc > 0.0) {
            double xacc = 0.0;
            for (int64_t c = 0; c < g->ncells; ++c) {
                xacc += expected_count(X, c);
                X->incl[c] = xacc;
            }
            X->X_total = xacc;
        }
        /* lower corners: roots from their indices, children from parents
         * (children always follow their parent in the cell vector) */
        X->cell_lo = (double *)malloc(sizeof(double) * 3 * (size_t)g->ncells);
        if (!X->cell_lo) return -3;
        for (int64_t c = 0; c < g->level_offset[1]; ++c) {
            X->cell_lo[3 * c] = (double)(c % g->nx);
            X->cell_lo[3 * c + 1] = (double)((c / g->nx) % g->ny);
            X->cell_lo[3 * c + 2] = (double)(c / ((int64_t)g->nx * g->ny));
        }
        for (int64_t c = 0; c < g->ncells; ++c) {
            if (word_i(g, c) >= 0) continue;
            int64_t first = -(int64_t)word_i(g, c);
            double half = ldexp(1.0, -(cell_level(g, c) + 1));
            for (int o = 0; o < 8; ++o) {
                X->cell_lo[3 * (first + o)] = X->cell_lo[3 * c] + (o & 1) * half;
                X->cell_lo[3 * (first + o) + 1] = X->cell_lo[3 * c + 1] + ((o >> 1) & 1) * half;
                X->cell_lo[3 * (first + o) + 2] = X->cell_lo[3 * c + 2] + ((o >> 2) & 1) * half;
            }
        }
        if (s->dust_mode == 0) {
            int64_t nl = 0;
            for (int64_t c = 0; c < g->ncells; ++c) nl += word_i(g, c) >= 0;
            X->leaves = (int64_t *)malloc(sizeof(int64_t) * (size_t)nl);
            if (!X->leaves) return -3;
            nl = 0;
            for (int64_t c = 0; c < g->ncells; ++c)
                if (word_i(g, c) >= 0) X->leaves[nl++] = c;
            X->nleaves = nl;
            if (s->n_dust % (uint64_t)nl != 0) return -1;
            X->per_leaf = s->n_dust / (uint64_t)nl;
        } else {
            stream_t rs;
            stream_init(&rs, X->seed, X->iteration, ORC_CLASS_DUST, X->freq_index, 0xFFFFFFFFu);
            X->u_sys = stream_next(&rs);
        }
    }
    X->n_total = s->n_bg + (uint64_t)s->n_ps * s->n_ps_pk + ((s->T && s->n_dust) ? s->n_dust : 0);
    return 0;
}

static void sim_free(sim_ctx *X)
{
    free(X->L); free(X->incl); free(X->leaves); free(X->cell_lo);
}

/* Weighted dust emission: package j of N takes the cell whose cumulative
 * interval contains x_j = (j + u) S / N, in units of |L| (systematic
 * sampling: cell c receives floor or ceil of N |L_c| / S packages).  With
 * a cap the intervals are the capped expected counts and x_j = j + u;
 * positions past their total emit nothing (-1). */
static int64_t weighted_cell(const sim_ctx *X, uint64_t j)
{
    double x;
    if (X->s->dust_cap > 0.0) {
        x = (double)j + X->u_sys;
        if (x >= X->X_total) return -1;
    } else {
        x = (((double)j + X->u_sys) * X->S) / (double)X->s->n_dust;
    }
    int64_t lo = 0, hi = X->g->ncells;  /* first c with incl[c] > x */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (X->incl[mid] > x) hi = mid; else lo = mid + 1;
    }
    if (lo >= X->g->ncells) lo = X->last_pos;
    return lo;
}

/* Emission of global package gid (class order bg | ps0..psN-1 | dust):
 * position p, direction u, energy W0 and the package's random stream.
 * origin receives the emitting cell of a dust package (-1 otherwise) and
 * cls its class.  Returns 0 for a package that carries no energy. */
static int emit_package(const sim_ctx *X, uint64_t gid, double p[3], double u[3], double *W0_out, stream_t *rs_out,
                        int64_t *origin_out, uint32_t *cls_out)
{
    int64_t origin = -1;
    const orc_grid *g = X->g;
    const orc_sources *s = X->s;
    double W0;
    stream_t rs;
    uint64_t nbg = s->n_bg, nps = (uint64_t)s->n_ps * s->n_ps_pk;
    if (gid < nbg) {
        uint32_t pid = (uint32_t)gid;
        stream_init(&rs, X->seed, X->iteration, ORC_CLASS_BG, X->freq_index, pid);
        *cls_out = ORC_CLASS_BG;
        W0 = X->W_bg;
        if (!(W0 > 0.0)) return 0;
        double N[3] = {(double)g->nx, (double)g->ny, (double)g->nz};
        double area[6] = {N[1] * N[2], N[1] * N[2], N[0] * N[2], N[0] * N[2], N[0] * N[1], N[0] * N[1]};
        double tot = area[0] + area[1] + area[2] + area[3] + area[4] + area[5];
        double x0 = stream_next(&rs), x1 = stream_next(&rs), x2 = stream_next(&rs);
        double x3 = stream_next(&rs), x4 = stream_next(&rs);
        double tt = x0 * tot, cum = 0.0;
        int face = 5;
        for (int k = 0; k < 6; ++k) { cum += area[k]; if (tt < cum) { face = k; break; } }
        int a = face / 2, neg = (face % 2) == 0;
        int b = a == 0 ? 1 : 0, cc = a == 2 ? 1 : 2;
        p[a] = neg ? 0.0 : N[a];
        p[b] = x1 * N[b];
        p[cc] = x2 * N[cc];
        double mu = sqrt(x3);
        double st = sqrt(fmax(0.0, 1.0 - mu * mu));
        double phi = 2.0 * ORC_PI * x4;
        u[a] = neg ? mu : -mu;
        u[b] = st * cos(phi);
        u[cc] = st * sin(phi);
    } else if (gid < nbg + nps) {
        uint64_t k = gid - nbg;
        int32_t src = (int32_t)(k / s->n_ps_pk);
        uint32_t pid = (uint32_t)(k % s->n_ps_pk);
        stream_init(&rs, X->seed, X->iteration, ORC_CLASS_PS0 + (uint32_t)src, X->freq_index, pid);
        *cls_out = ORC_CLASS_PS0 + (uint32_t)src;
        W0 = s->ps_L_nu[src] * X->f->w_nu / (double)s->n_ps_pk;
        if (!(W0 > 0.0)) return 0;
        p[0] = s->ps_pos[3 * src]; p[1] = s->ps_pos[3 * src + 1]; p[2] = s->ps_pos[3 * src + 2];
        double x0 = stream_next(&rs), x1 = stream_next(&rs);
        iso_dir(x0, x1, u);
    } else {
        uint64_t j = gid - nbg - nps;
        stream_init(&rs, X->seed, X->iteration, ORC_CLASS_DUST, X->freq_index, (uint32_t)j);
        *cls_out = ORC_CLASS_DUST;
        int64_t c;
        if (s->dust_mode == 0) {
            c = X->leaves[j / X->per_leaf];
            W0 = X->L[c] / (double)X->per_leaf;
        } else {
            /* each package of cell c carries L_c over the cell's expected
             * count, so the packages of c sum to L_c on average; in mode 2
             * L_c is the signed difference to the reference emission */
            if (!(X->S > 0.0)) return 0;
            c = weighted_cell(X, j);
            if (c < 0) return 0;
            W0 = X->L[c] / expected_count(X, c);
        }
        if (!(fabs(W0) > 0.0)) return 0;
        origin = c;
        double size = ldexp(1.0, -cell_level(g, c));
        const double *lo = X->cell_lo + 3 * c;
        double x0 = stream_next(&rs), x1 = stream_next(&rs), x2 = stream_next(&rs);
        double x3 = stream_next(&rs), x4 = stream_next(&rs);
        p[0] = lo[0] + x0 * size; p[1] = lo[1] + x1 * size; p[2] = lo[2] + x2 * size;
        iso_dir(x3, x4, u);
    }
    *W0_out = W0;
    *rs_out = rs;
    *origin_out = origin;
    return 1;
}

/* Emission of global package gid and its transport.  Returns the initial
 * weight W0 (0 for a package that carries no energy). */
static double run_package(const sim_ctx *X, uint64_t gid, double *absorbed, int64_t *hits, pk_tally *t,
                          orc_segment *seg, int32_t max_seg, int32_t *nseg, double *self_abs, double *emitted)
{
    double p[3], u[3], W0;
    stream_t rs;
    int64_t origin;
    uint32_t cls;
    if (!emit_package(X, gid, p, u, &W0, &rs, &origin, &cls)) return 0.0;
    if (origin >= 0 && self_abs && emitted) emitted[origin] += W0;
    double tau = -log(stream_next(&rs));
    transport(X->g, X->f, p, u, W0, tau, &rs, X->cap, absorbed, hits, t, seg, max_seg, nseg, origin,
              self_abs && emitted ? self_abs : NULL);
    return W0;
}

static int32_t check_inputs(const orc_grid *g, const orc_freq *f, const orc_sources *s);

/* ---- scattered light ---- */

/* Optical depth (scattering only, or extinction) from p along direction o
 * to the box boundary, leaf by leaf from a brute-force lookup. */
static double ray_tau(const orc_grid *g, const orc_freq *f, const double p0[3], const double o[3], int ext)
{
    double p[3] = {p0[0], p0[1], p0[2]}, tau = 0.0;
    const double s_cm = g->root_cell_cm;
    const double k_unit = (ext ? f->sigma_abs + f->sigma_sca : f->sigma_sca) * s_cm;
    for (int guard = 0; guard < 100000000; ++guard) {
        double q[3] = {p[0] + ORC_EPS_PUSH * o[0], p[1] + ORC_EPS_PUSH * o[1], p[2] + ORC_EPS_PUSH * o[2]};
        double lo[3], size;
        int64_t c = orc_leaf(g, q, lo, &size);
        if (c < 0) break;
        double d = INFINITY;
        for (int i = 0; i < 3; ++i) {
            double di = INFINITY;
            if (o[i] > 0.0) di = (lo[i] + size - p[i]) / o[i];
            else if (o[i] < 0.0) di = (lo[i] - p[i]) / o[i];
            if (di < 0.0) di = 0.0;
            if (di < d) d = di;
        }
        tau += k_unit * word_f(g, c) * d;
        p[0] += d * o[0]; p[1] += d * o[1]; p[2] += d * o[2];
    }
    return tau;
}

/* Henyey-Greenstein phase function normalised over the sphere. */
static double hg_phase(double g, double mu)
{
    if (fabs(g) < 1e-4) return 1.0 / (4.0 * ORC_PI);
    double d = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * ORC_PI * d * sqrt(d));
}

typedef struct {
    int axis, neg, npx, npy;
    double o[3], psz, scale;   /* scale: 1 / (A_pix w_nu) */
} peel_geom;

static int64_t peel_pixel(const peel_geom *G, const double p[3])
{
    int b = G->axis == 0 ? 1 : 0, c = G->axis == 2 ? 1 : 2;
    int64_t i = (int64_t)floor(p[b] / G->psz), j = (int64_t)floor(p[c] / G->psz);
    if (i < 0) i = 0;
    if (i >= G->npx) i = G->npx - 1;
    if (j < 0) j = 0;
    if (j >= G->npy) j = G->npy - 1;
    return j * G->npx + i;
}

/* One package of the scattered-light run: optional forced first
 * scattering, then the per-cell loop of transport() without tallies,
 * peeling off every scattering. */
static void peel_package(const sim_ctx *X, uint64_t gid, const orc_scatter_params *sp, const peel_geom *G,
                         double *image, pk_tally *t, double *W0_out)
{
    const orc_grid *g = X->g;
    const orc_freq *f = X->f;
    double p[3], u[3], W0;
    stream_t rs;
    int64_t origin;
    uint32_t cls;
    *W0_out = 0.0;
    if (!emit_package(X, gid, p, u, &W0, &rs, &origin, &cls)) return;
    *W0_out = W0;
    if (sp->direct && cls >= ORC_CLASS_PS0)
        image[peel_pixel(G, p)] += W0 / (4.0 * ORC_PI) * exp(-ray_tau(g, f, p, G->o, 1)) * G->scale;
    double xi = stream_next(&rs);
    double tau, W = W0;
    if (sp->forced) {
        double q = -expm1(-ray_tau(g, f, p, u, 0));   /* chance to scatter before leaving */
        if (!(q > 0.0)) return;
        W *= q;
        tau = -log1p(-xi * q);
    } else {
        tau = -log(xi);
    }
    const double s_cm = g->root_cell_cm;
    int nscat = 0;
    for (;;) {
        double q[3] = {p[0] + ORC_EPS_PUSH * u[0], p[1] + ORC_EPS_PUSH * u[1], p[2] + ORC_EPS_PUSH * u[2]};
        double lo[3], size;
        int64_t c = orc_leaf(g, q, lo, &size);
        if (c < 0) { t->escaped += W; return; }
        double dexit = INFINITY;
        for (int i = 0; i < 3; ++i) {
            double d = INFINITY;
            if (u[i] > 0.0) d = (lo[i] + size - p[i]) / u[i];
            else if (u[i] < 0.0) d = (lo[i] - p[i]) / u[i];
            if (d < 0.0) d = 0.0;
            if (d < dexit) dexit = d;
        }
        double n = word_f(g, c);
        double ks = f->sigma_sca * n * s_cm, ka = f->sigma_abs * n * s_cm;
        int scat = 0;
        double d;
        if (ks > 0.0 && ks * dexit >= tau) {
            d = tau / ks;
            if (d > dexit) d = dexit;
            scat = 1;
        } else {
            d = dexit;
            tau -= ks * dexit;
        }
        W *= exp(-ka * d);
        p[0] += d * u[0]; p[1] += d * u[1]; p[2] += d * u[2];
        t->steps++;
        if (W < ORC_WFLOOR * W0) return;
        if ((int64_t)t->steps >= X->cap) { t->runaway++; return; }
        if (!scat) continue;
        /* peel off towards the observer, then scatter */
        double mu = u[0] * G->o[0] + u[1] * G->o[1] + u[2] * G->o[2];
        image[peel_pixel(G, p)] += W * hg_phase(f->g, mu) * exp(-ray_tau(g, f, p, G->o, 1)) * G->scale;
        t->scatterings++;
        if (sp->max_scatter > 0 && ++nscat >= sp->max_scatter) return;
        double xm = stream_next(&rs), xp = stream_next(&rs);
        scatter_dir(f->g, xm, xp, u);
        tau = -log(stream_next(&rs));
    }
}

int32_t orc_scatter_map(const orc_grid *g, const orc_freq *f, const orc_sources *s, uint64_t seed,
                        uint32_t iteration, uint32_t freq_index, const orc_scatter_params *sp,
                        int64_t step_cap, int32_t nthreads, double *image, orc_stats *stats)
{
    int32_t rc = check_inputs(g, f, s);
    if (rc) return rc;
    if (!sp || !image || (s->T && s->n_dust) || (sp->axis & 3) > 2 || sp->max_scatter < 0) return -1;
    if (!(f->w_nu > 0.0)) return -1;
    sim_ctx X;
    memset(&X, 0, sizeof X);
    X.g = g; X.f = f; X.s = s; X.seed = seed; X.iteration = iteration; X.freq_index = freq_index;
    X.cap = step_cap > 0 ? step_cap : 10000000;
    rc = sim_setup(&X);
    if (rc) { sim_free(&X); return rc; }
    peel_geom G;
    memset(&G, 0, sizeof G);
    G.axis = sp->axis & 3;
    G.neg = (sp->axis & 4) != 0;
    G.o[G.axis] = G.neg ? -1.0 : 1.0;
    int32_t N[3] = {g->nx, g->ny, g->nz};
    int b = G.axis == 0 ? 1 : 0, c = G.axis == 2 ? 1 : 2;
    int fine = 1 << (g->nlevels - 1);
    G.npx = N[b] * fine;
    G.npy = N[c] * fine;
    G.psz = 1.0 / fine;
    double pix_cm = g->root_cell_cm * G.psz;
    G.scale = 1.0 / (pix_cm * pix_cm * f->w_nu);
    int64_t npix = (int64_t)G.npx * G.npy;
    orc_stats tot;
    memset(&tot, 0, sizeof tot);
    int failed = 0;
    if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *priv = (double *)calloc((size_t)npix, sizeof(double));
        orc_stats loc;
        memset(&loc, 0, sizeof loc);
        if (!priv) failed = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (int64_t gid = 0; gid < (int64_t)X.n_total; ++gid) {
            if (!priv) continue;
            pk_tally t;
            memset(&t, 0, sizeof t);
            double W0;
            peel_package(&X, (uint64_t)gid, sp, &G, priv, &t, &W0);
            loc.packages++;
            loc.cell_steps += t.steps;
            loc.scatterings += t.scatterings;
            loc.runaways += t.runaway;
            loc.e_emitted += W0;
            loc.e_escaped += t.escaped;
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            if (priv)
                for (int64_t k = 0; k < npix; ++k) image[k] += priv[k];
            tot.packages += loc.packages; tot.cell_steps += loc.cell_steps;
            tot.scatterings += loc.scatterings; tot.runaways += loc.runaways;
            tot.e_emitted += loc.e_emitted; tot.e_escaped += loc.e_escaped;
        }
        free(priv);
    }
    sim_free(&X);
    if (failed) return -3;
    if (stats) *stats = tot;
    return 0;
}

static int32_t check_inputs(const orc_grid *g, const orc_freq *f, const orc_sources *s)
{
    if (!g || !f || !s) return -1;
    if (!(f->sigma_abs >= 0.0) || !(f->sigma_sca >= 0.0) || !(fabs(f->g) < 1.0)) return -1;
    if (s->n_ps > 0 && (!s->ps_pos || !s->ps_L_nu)) return -1;
    if (s->n_ps > 253) return -1;
    if (s->T && s->n_dust && (s->dust_mode < 0 || s->dust_mode > 2)) return -1;
    if (!(s->dust_cap >= 0.0)) return -1;
    for (int32_t i = 0; i < s->n_ps; ++i) {
        double q[3] = {s->ps_pos[3 * i], s->ps_pos[3 * i + 1], s->ps_pos[3 * i + 2]}, lo[3], sz;
        if (orc_leaf(g, q, lo, &sz) < 0) return -1;
    }
    return orc_validate_grid(g) == 0 ? 0 : -4;
}

int32_t orc_simulate_frequency(const orc_grid *g, const orc_freq *f, const orc_sources *s,
                               uint64_t seed, uint32_t iteration, uint32_t freq_index,
                               int64_t step_cap, int32_t nthreads,
                               double *absorbed, orc_stats *stats, double *path_len, int64_t *hits)
{
    int32_t rc = check_inputs(g, f, s);
    if (rc) return rc;
    sim_ctx X;
    memset(&X, 0, sizeof X);
    X.g = g; X.f = f; X.s = s; X.seed = seed; X.iteration = iteration; X.freq_index = freq_index;
    X.cap = step_cap > 0 ? step_cap : 10000000;
    rc = sim_setup(&X);
    if (rc) { sim_free(&X); return rc; }
    orc_stats tot;
    memset(&tot, 0, sizeof tot);
    int64_t ncells = g->ncells;
    uint64_t NT = X.n_total;
    if (nthreads < 1) nthreads = 1;
    int failed = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *priv = (double *)calloc((size_t)ncells, sizeof(double));
        int64_t *phits = hits ? (int64_t *)calloc((size_t)ncells, sizeof(int64_t)) : NULL;
        const int ali = s->ali_self && s->ali_emitted;
        double *pself = ali ? (double *)calloc((size_t)ncells, sizeof(double)) : NULL;
        double *pemit = ali ? (double *)calloc((size_t)ncells, sizeof(double)) : NULL;
        orc_stats loc;
        memset(&loc, 0, sizeof loc);
        if (!priv || (hits && !phits) || (ali && (!pself || !pemit))) failed = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (int64_t gid = 0; gid < (int64_t)NT; ++gid) {
            if (!priv || (hits && !phits) || (ali && (!pself || !pemit))) continue;
            pk_tally t;
            memset(&t, 0, sizeof t);
            double W0 = run_package(&X, (uint64_t)gid, priv, phits, &t, NULL, 0, NULL, pself, pemit);
            loc.packages++;
            loc.cell_steps += t.steps;
            loc.scatterings += t.scatterings;
            loc.runaways += t.runaway;
            loc.e_emitted += W0;
            loc.e_escaped += t.escaped;
            if (path_len) path_len[gid] = t.path;
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            if (priv) {
                for (int64_t c = 0; c < ncells; ++c) absorbed[c] += priv[c];
                double a = 0.0;
                for (int64_t c = 0; c < ncells; ++c) a += priv[c];
                if (pself) {
                    for (int64_t c = 0; c < ncells; ++c) a += pself[c];
                    for (int64_t c = 0; c < ncells; ++c) s->ali_self[c] += pself[c];
                }
                if (pemit)
                    for (int64_t c = 0; c < ncells; ++c) s->ali_emitted[c] += pemit[c];
                loc.e_absorbed = a;
            }
            if (phits)
                for (int64_t c = 0; c < ncells; ++c) hits[c] += phits[c];
            tot.packages += loc.packages; tot.cell_steps += loc.cell_steps;
            tot.scatterings += loc.scatterings; tot.runaways += loc.runaways;
            tot.e_emitted += loc.e_emitted; tot.e_escaped += loc.e_escaped; tot.e_absorbed += loc.e_absorbed;
        }
        free(priv);
        free(phits);
        free(pself);
        free(pemit);
    }
    sim_free(&X);
    if (failed) return -3;
    if (stats) *stats = tot;
    return 0;
}

int32_t orc_trace_package(const orc_grid *g, const orc_freq *f, const orc_sources *s,
                          uint64_t seed, uint32_t iteration, uint32_t freq_index,
                          uint32_t cls, uint32_t package_id, int64_t step_cap,
                          orc_segment *out, int32_t max_seg, int32_t *n_seg)
{
    int32_t rc = check_inputs(g, f, s);
    if (rc) return rc;
    sim_ctx X;
    memset(&X, 0, sizeof X);
    X.g = g; X.f = f; X.s = s; X.seed = seed; X.iteration = iteration; X.freq_index = freq_index;
    X.cap = step_cap > 0 ? step_cap : 10000000;
    rc = sim_setup(&X);
    if (rc) { sim_free(&X); return rc; }
    uint64_t gid;
    if (cls == ORC_CLASS_BG) {
        if (package_id >= s->n_bg) { sim_free(&X); return -1; }
        gid = package_id;
    } else if (cls == ORC_CLASS_DUST) {
        if (!s->T || package_id >= s->n_dust) { sim_free(&X); return -1; }
        gid = s->n_bg + (uint64_t)s->n_ps * s->n_ps_pk + package_id;
    } else {
        uint32_t src = cls - ORC_CLASS_PS0;
        if ((int32_t)src >= s->n_ps || package_id >= s->n_ps_pk) { sim_free(&X); return -1; }
        gid = s->n_bg + (uint64_t)src * s->n_ps_pk + package_id;
    }
    pk_tally t;
    memset(&t, 0, sizeof t);
    *n_seg = 0;
    run_package(&X, gid, NULL, NULL, &t, out, max_seg, n_seg, NULL, NULL);
    sim_free(&X);
    return 0;
}

int32_t orc_trace_from(const orc_grid *g, const orc_freq *f, const double p0[3], const double u0[3],
                       double W0, double tau0, uint64_t seed, uint32_t package_id, int64_t step_cap,
                       double *absorbed, orc_segment *out, int32_t max_seg, int32_t *n_seg,
                       double *w_escaped)
{
    if (orc_validate_grid(g) != 0) return -4;
    stream_t rs;
    stream_init(&rs, seed, 0, ORC_CLASS_BG, 0, package_id);
    double p[3] = {p0[0], p0[1], p0[2]}, u[3] = {u0[0], u0[1], u0[2]};
    pk_tally t;
    memset(&t, 0, sizeof t);
    int32_t ns = 0;
    transport(g, f, p, u, W0, tau0, &rs, step_cap > 0 ? step_cap : 10000000, absorbed, NULL, &t, out, max_seg, &ns,
              -1, NULL);
    if (n_seg) *n_seg = ns;
    if (w_escaped) *w_escaped = t.escaped;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Equilibrium temperature (Sect. 2.1.1): per leaf, solve
 * Gamma(T) = A_c / (n_c V_c) by bisection on [T_floor, T_max].  Empty and
 * refined cells get T = 0; unhit cells and out-of-range values are clamped
 * to the interval and counted (the constant temperature given to unhit
 * cells, Sect. 3.2). */
static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

static int32_t update_temperature(const orc_grid *g, const orc_freq *emit, int32_t K, double T_floor,
                                  double T_max, const double *absorbed, const double *self_abs,
                                  const double *emitted, const float *T_old, float *T_new,
                                  orc_temp_stats *stats);

int32_t orc_update_temperature(const orc_grid *g, const orc_freq *emit, int32_t K,
                               double T_floor, double T_max,
                               const double *absorbed, const float *T_old, float *T_new,
                               orc_temp_stats *stats)
{
    return update_temperature(g, emit, K, T_floor, T_max, absorbed, NULL, NULL, T_old, T_new, stats);
}

int32_t orc_update_temperature_ali(const orc_grid *g, const orc_freq *emit, int32_t K,
                                   double T_floor, double T_max, const double *absorbed,
                                   const double *self_abs, const double *emitted,
                                   const float *T_old, float *T_new, orc_temp_stats *stats)
{
    if (!self_abs || !emitted) return -1;
    return update_temperature(g, emit, K, T_floor, T_max, absorbed, self_abs, emitted, T_old, T_new, stats);
}

static int32_t update_temperature(const orc_grid *g, const orc_freq *emit, int32_t K, double T_floor,
                                  double T_max, const double *absorbed, const double *self_abs,
                                  const double *emitted, const float *T_old, float *T_new,
                                  orc_temp_stats *stats)
{
    if (orc_validate_grid(g) != 0) return -4;
    if (!(T_floor > 0.0) || !(T_max > T_floor) || K < 1) return -1;
    double G_lo = orc_gamma(emit, K, T_floor), G_hi = orc_gamma(emit, K, T_max);
    int64_t n = g->ncells, cnt = 0, nrel = 0;
    uint64_t clamped = 0;
    double sumT = 0.0, sumrel = 0.0;
    double *vals = (double *)malloc(sizeof(double) * (size_t)n);
    if (!vals) return -3;
    for (int64_t c = 0; c < n; ++c) {
        double T = 0.0;
        if (word_i(g, c) >= 0 && word_f(g, c) > 0.0) {
            double y = absorbed[c] / (word_f(g, c) * cell_volume(g, c));
            if (self_abs) {
                /* escape probability of the cell's own emission */
                double esc = emitted[c] > 0.0 ? 1.0 - self_abs[c] / emitted[c] : 1.0;
                if (esc < 1e-6) esc = 1e-6;
                y /= esc;
            }
            if (!(y > G_lo)) { T = T_floor; clamped++; }
            else if (y >= G_hi) { T = T_max; clamped++; }
            else {
                double a = T_floor, b = T_max;
                for (int it = 0; it < 200 && b - a > 1e-10; ++it) {
                    double m = 0.5 * (a + b);
                    if (orc_gamma(emit, K, m) < y) a = m; else b = m;
                }
                T = 0.5 * (a + b);
            }
            vals[cnt++] = T;
            sumT += T;
            if (T_old && T_old[c] > 0.0f) {
                sumrel += fabs(T - (double)T_old[c]) / (double)T_old[c];
                nrel++;
            }
        }
        T_new[c] = (float)T;
    }
    if (stats) {
        stats->clamped = clamped;
        stats->mean_T = cnt ? sumT / (double)cnt : 0.0;
        stats->mean_rel_change = nrel ? sumrel / (double)nrel : NAN;
        if (cnt) {
            qsort(vals, (size_t)cnt, sizeof(double), cmp_desc);
            int64_t k = (int64_t)ceil(0.05 * (double)cnt);
            if (k < 1) k = 1;
            double s = 0.0;
            for (int64_t i = 0; i < k; ++i) s += vals[i];
            stats->hot5_mean_T = s / (double)k;
        } else {
            stats->hot5_mean_T = 0.0;
        }
    }
    free(vals);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Emission map (Sect. 2.1.1 map kernel; pixel = smallest cell, Sect. 3.2):
 * I = sum over segments of S_c (1 - e^{-dtau}) e^{-tau_front}, with
 * S_c = (sigma_abs / sigma_ext) B_nu(T_c) and dtau = sigma_ext n_c ds. */
int32_t orc_map(const orc_grid *g, const orc_freq *f, const float *T, int32_t axis,
                double *image, int32_t *npx, int32_t *npy)
{
    if (orc_validate_grid(g) != 0) return -4;
    int a = axis & 3, neg = (axis >> 2) & 1;
    if (a > 2) return -1;
    int b = a == 0 ? 1 : 0, cc = a == 2 ? 1 : 2;
    int N[3] = {g->nx, g->ny, g->nz};
    int64_t scale = (int64_t)1 << (g->nlevels - 1);
    int32_t nb = (int32_t)(N[b] * scale), nc = (int32_t)(N[cc] * scale);
    if (npx) *npx = nb;
    if (npy) *npy = nc;
    if (!image) return 0;
    double sext = f->sigma_abs + f->sigma_sca;
    double psz = 1.0 / (double)scale;
    for (int32_t j = 0; j < nc; ++j)
        for (int32_t i = 0; i < nb; ++i) {
            double I = 0.0, tau = 0.0;
            double p[3];
            p[b] = (i + 0.5) * psz;
            p[cc] = (j + 0.5) * psz;
            double x = neg ? 0.0 : (double)N[a];
            if (sext > 0.0) {
                for (;;) {
                    if (neg ? (x >= N[a]) : (x <= 0.0)) break;
                    p[a] = neg ? x + 0.5 * ORC_EPS_PUSH : x - 0.5 * ORC_EPS_PUSH;
                    double lo[3], sz;
                    int64_t c = orc_leaf(g, p, lo, &sz);
                    if (c < 0) break;
                    double xn = neg ? lo[a] + sz : lo[a];
                    double ds = fabs(xn - x);
                    double n = word_f(g, c);
                    if (n > 0.0) {
                        double dt = sext * n * ds * g->root_cell_cm;
                        double S = (f->sigma_abs / sext) * orc_planck(f->nu, (double)T[c]);
                        I += S * (-expm1(-dt)) * exp(-tau);
                        tau += dt;
                    }
                    x = xn;
                }
            }
            image[(int64_t)j * nb + i] = I;
        }
    return 0;
}
