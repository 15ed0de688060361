/*
 * soc_oracle.h -- FP64 CPU oracle for the SOC Monte Carlo hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can compare the GPU
 * library against a plain, slow, obviously correct implementation.  No
 * product code may link, load or call it.  It shares no code, header,
 * table or constant with the GPU library (its physical constants, Philox
 * generator, Henyey-Greenstein draw, rotation, leaf lookup and temperature
 * solver are all written here from their published definitions).
 *
 * What it computes follows Juvela, "SOC program for dust continuum
 * radiative transfer" (A&A 2019, arXiv:1812.06632):
 *   - Sect. 2.1.1 (Basic program): hierarchical grid stored as one density
 *     vector with negative links to the first child of each octet; photon
 *     packages simulated one frequency at a time; absorbed energy counted
 *     per cell and integrated over frequency for equilibrium grains;
 *     separate kernels for the temperature solve and for maps.
 *   - Sect. 2.2 and 3.1: isotropic external field, blackbody point sources
 *     in empty cells.
 *   - Sect. 3.2: dust re-emission with an equal number of packages per cell
 *     (uniform) or with package numbers proportional to cell luminosity
 *     (weighted), optionally with a cap on the packages of one cell.
 *   - Sect. 2.1.2 (reference field): an iteration simulates only the
 *     difference between the current dust emission and a reference
 *     emission, with packages of either sign.
 *   - Sect. 2.1.2, 4.1 (ALI with a diagonal operator): the part of a cell's
 *     emission that it absorbs itself is counted apart, and the temperature
 *     update solves that cell's own emission-absorption cycle exactly.
 * The paper prints no equations; the estimator and sampling rules below are
 * the textbook Monte Carlo readings recorded in the design notes:
 *   continuous absorption along each segment, free paths drawn in
 *   scattering optical depth, analytic Henyey-Greenstein scattering,
 *   cosine-weighted inward emission from the box faces, weight floor 1e-12
 *   with the remainder deposited, and a step cap that deposits the rest.
 *
 * Units: cgs.  Positions are in root-cell units inside the box
 * [0,nx) x [0,ny) x [0,nz).  Densities are in H cm^-3, cross sections in
 * cm^2 per H, intensities in erg s^-1 cm^-2 Hz^-1 sr^-1, luminosities in
 * erg s^-1 Hz^-1, absorbed energy in erg s^-1 per cell (already multiplied
 * by the frequency quadrature weight w_nu).
 *
 * Parity status of each function is stated in its comment.
 */
#ifndef SOC_ORACLE_H
#define SOC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One 32-bit word per cell: an FP32 density >= 0, or (as int32) the negated
 * global index of the first cell of the child octet (Sect. 2.1.1). */
typedef struct {
    int32_t nx, ny, nz, nlevels;
    int64_t ncells;
    const int64_t *level_offset;   /* nlevels+1 entries, first cell of each level */
    double root_cell_cm;           /* edge of a root cell in cm */
    const uint32_t *words;         /* ncells words */
} orc_grid;

typedef struct { double nu, w_nu, sigma_abs, sigma_sca, g; } orc_freq;

typedef struct {
    double I_bg_nu;            /* isotropic external intensity at nu */
    int32_t n_ps;              /* number of point sources */
    const double *ps_pos;      /* 3*n_ps, root units */
    const double *ps_L_nu;     /* n_ps, erg s^-1 Hz^-1 */
    const float *T;            /* per-cell dust temperature; NULL = no dust emission */
    uint64_t n_bg;             /* background packages */
    uint64_t n_ps_pk;          /* packages per point source */
    uint64_t n_dust;           /* dust-emission packages */
    int32_t dust_mode;         /* 0 = equal count per leaf, 1 = luminosity weighted,
                                  2 = correction to a reference emission (below) */
    const double *L_ref;       /* dust_mode 2: reference emission of each cell at this
                                  frequency (erg s^-1, already times w_nu); NULL = zero */
    double dust_cap;           /* modes 1 and 2: expected packages per cell at most this
                                  many (0 = no cap); the excess is not re-assigned */
    double *ali_self;          /* diagonal ALI (optional, +=, ncells): what dust packages
                                  deposit in the cell that emitted them goes here instead
                                  of into `absorbed` */
    double *ali_emitted;       /* with ali_self: the initial weight of every dust package,
                                  added to its emitting cell */
} orc_sources;

typedef struct {
    uint64_t packages, cell_steps, scatterings, runaways;
    double e_emitted, e_absorbed, e_escaped;
} orc_stats;

/* Segment end events. */
enum { ORC_CROSS = 0, ORC_SCATTER = 1, ORC_ESCAPE = 2, ORC_FLOOR = 3, ORC_RUNAWAY = 4 };
/* Source classes (Philox counter word 3 = iteration<<8 | class). */
enum { ORC_CLASS_BG = 0, ORC_CLASS_DUST = 1, ORC_CLASS_PS0 = 2 };

typedef struct { int64_t cell; double ds; int32_t event; } orc_segment;

/* ---- random numbers: Philox4x32-10 (Salmon et al. 2011, SC'11) ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Uniform in (0,1): ((x >> 9) + 0.5) * 2^-23 -- an odd multiple of 2^-24,
 * exactly representable in FP32 and FP64. */
double orc_u01(uint32_t x);
/* n consecutive uniforms of one package stream (for statistical pins). */
void orc_uniforms(uint64_t seed, uint32_t iteration, uint32_t cls, uint32_t freq_index,
                  uint32_t package_id, int32_t n, double *out);

/* ---- physics helpers ---- */
double orc_planck(double nu, double T);                       /* B_nu(T) */
double orc_gamma(const orc_freq *f, int32_t K, double T);      /* 4 pi sum_k w_k sigma_abs,k B(T) */
int64_t orc_leaf(const orc_grid *g, const double p[3], double lo[3], double *size);
int32_t orc_validate_grid(const orc_grid *g);                  /* 0 ok, <0 malformed */

/* Henyey-Greenstein draw + rotation for statistical pins: n new directions
 * from u0 using pairs of uniforms (xi_mu, xi_phi) from `xi` (2n values). */
void orc_hg_scatter(double g, const double u0[3], int32_t n, const double *xi, double *out3n);

/* Dust emission of every cell at one frequency, 4 pi sigma_abs n V B_nu(T) w
 * (0 in refined and empty cells), into L (ncells). */
int32_t orc_dust_luminosity(const orc_grid *g, const orc_freq *f, const float *T, double *L);

/* ---- the Monte Carlo pass at one frequency ---- */
/* absorbed (+=) must hold ncells doubles.  path_len (optional) receives the
 * total path length in root units of each package, in class order
 * [bg | ps0 | ps1 ... | dust].  hits (optional, +=) counts the segments that
 * deposited energy in each cell.  Returns 0 or a negative error. */
int32_t orc_simulate_frequency(const orc_grid *g, const orc_freq *f, const orc_sources *s,
                               uint64_t seed, uint32_t iteration, uint32_t freq_index,
                               int64_t step_cap, int32_t nthreads,
                               double *absorbed, orc_stats *stats, double *path_len, int64_t *hits);

/* Segments of one package (class, package id within that class). */
int32_t orc_trace_package(const orc_grid *g, const orc_freq *f, const orc_sources *s,
                          uint64_t seed, uint32_t iteration, uint32_t freq_index,
                          uint32_t cls, uint32_t package_id, int64_t step_cap,
                          orc_segment *out, int32_t max_seg, int32_t *n_seg);

/* Trace from an explicit state with a given initial free path tau0 (in
 * scattering optical depth); later free paths come from the stream of
 * (seed, package_id).  Deposits into absorbed (may be NULL).  Returns the
 * escaped weight through *w_escaped. */
int32_t orc_trace_from(const orc_grid *g, const orc_freq *f, const double p0[3], const double u0[3],
                       double W0, double tau0, uint64_t seed, uint32_t package_id, int64_t step_cap,
                       double *absorbed, orc_segment *out, int32_t max_seg, int32_t *n_seg,
                       double *w_escaped);

/* ---- scattered light (Sect. 2.1.1: separate runs with forced first
 * scattering and peel-off) ---- */
typedef struct {
    int32_t axis;          /* observer along root axis axis & 3, on the positive side; bit 2: negative side */
    int32_t forced;        /* 1: every package scatters at least once inside the box (weight times
                              1 - exp(-tau_esc), free path from the truncated exponential) */
    int32_t max_scatter;   /* 0: all scatterings; k: stop a package after its k-th (peeled) scattering */
    int32_t direct;        /* 1: add the attenuated direct light of the point sources */
} orc_scatter_params;

/* Image of the light scattered towards a distant observer, by peel-off:
 * at every scattering a package of weight W at p, moving along u, adds
 * W Phi(u.o) exp(-tau_ext(p -> boundary along o)) / (A_pix w_nu) to the
 * pixel under p, Phi the normalised Henyey-Greenstein function (1/4pi for
 * |g| < 1e-4), o the direction towards the observer, tau_ext the
 * extinction optical depth (absorption + scattering).  Sources: external
 * field and point sources (no dust emission).  Pixels as orc_map: npy rows
 * of npx, the lower and higher of the other two axes, finest-cell size.
 * image (+=, npx*npy doubles) is in erg s^-1 cm^-2 Hz^-1 sr^-1.
 * Returns 0 or a negative error. */
int32_t orc_scatter_map(const orc_grid *g, const orc_freq *f, const orc_sources *s, uint64_t seed,
                        uint32_t iteration, uint32_t freq_index, const orc_scatter_params *sp,
                        int64_t step_cap, int32_t nthreads, double *image, orc_stats *stats);

/* ---- temperature update (equilibrium grains) ---- */

typedef struct { double mean_T, hot5_mean_T, mean_rel_change; uint64_t clamped; } orc_temp_stats;
int32_t orc_update_temperature(const orc_grid *g, const orc_freq *emit, int32_t K,
                               double T_floor, double T_max,
                               const double *absorbed, const float *T_old, float *T_new,
                               orc_temp_stats *stats);
/* Diagonal ALI: with beta_c = self_c / emitted_c (0 where the cell emitted
 * nothing; the escape probability 1 - beta_c is kept >= 1e-6), solve
 * Gamma(T_c) n_c V_c (1 - beta_c) = absorbed_c: the cell's emission equals
 * what it absorbs from elsewhere plus the fraction beta_c of its own
 * emission.  Otherwise as orc_update_temperature. */
int32_t orc_update_temperature_ali(const orc_grid *g, const orc_freq *emit, int32_t K,
                                   double T_floor, double T_max, const double *absorbed,
                                   const double *self_abs, const double *emitted,
                                   const float *T_old, float *T_new, orc_temp_stats *stats);

/* ---- emission map along a root-grid axis (axis 0..2, bit 2 = observer on
 * the negative side), pixel = finest cell; image is npy*npx doubles. ---- */
int32_t orc_map(const orc_grid *g, const orc_freq *f, const float *T, int32_t axis,
                double *image, int32_t *npx, int32_t *npy);

#ifdef __cplusplus
}
#endif
#endif
