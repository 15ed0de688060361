/*
 * soc.h -- C ABI of the SOC Monte Carlo dust radiative-transfer hot path on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow Juvela, "SOC program for dust continuum radiative
 * transfer" (A&A 2019, arXiv:1812.06632), Sect. 2.1.1 "Basic program": the
 * cloud is one vector of cells on a hierarchical (octree) grid, photon
 * packages are simulated one frequency at a time by a kernel that counts
 * the energy absorbed in each cell, a second kernel solves the equilibrium
 * dust temperature from the frequency-integrated absorbed energy, and a
 * third makes surface-brightness maps from that solution.
 *
 * Conventions shared by every call
 *  - Every call returns soc_status (0 = SOC_OK, < 0 = error).  No call
 *    aborts, exits or throws; on error the text of the failure is available
 *    from soc_last_error(ctx) until the next call on that context.
 *  - Pointers named d_* are device pointers (HIP device memory of the
 *    context's device, e.g. torch tensors' data_ptr()).  Other pointers are
 *    host pointers, read or written only during the call.
 *  - Large arrays are owned by the caller; a soc_grid borrows the caller's
 *    cell array for its lifetime.  The library allocates only private
 *    scratch, owned by the context (or grid) and freed by its destroy call.
 *  - Work is enqueued on the context's HIP stream and the call returns
 *    without waiting, unless it returns host results (statistics, traces),
 *    in which case it synchronises that stream before returning.
 *  - Units are cgs: cell size in cm, density in H cm^-3, cross sections in
 *    cm^2 per H, intensity in erg s^-1 cm^-2 Hz^-1 sr^-1, luminosity in
 *    erg s^-1 Hz^-1, absorbed energy in erg s^-1 per cell (already
 *    multiplied by the frequency quadrature weight), temperature in K.
 *    Positions are in root-cell units inside [0,nx) x [0,ny) x [0,nz).
 *  - Validation happens before any launch: NULL pointers, negative counts,
 *    negative or non-finite cross sections, |g| >= 1 -> SOC_EINVAL; a
 *    malformed grid -> SOC_EGRID; HIP failures -> SOC_EHIP.
 */
#ifndef SOC_H
#define SOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SOC_OK = 0,
    SOC_EINVAL = -1,   /* bad argument */
    SOC_ENOMEM = -2,   /* device or host allocation failed */
    SOC_EHIP = -3,     /* HIP runtime error */
    SOC_EGRID = -4,    /* malformed grid */
    SOC_ESTATE = -5    /* call not valid in the current state */
} soc_status;

typedef struct soc_ctx_s *soc_ctx;
typedef struct soc_grid_s *soc_grid;

/* ---------------------------------------------------------------- context */
/* Create a context bound to HIP device `hip_device` and the HIP stream
 * `hip_stream` (a hipStream_t; NULL = the device's null stream).  The
 * stream is borrowed, never destroyed by the library. */
soc_status soc_ctx_create(int32_t hip_device, void *hip_stream, soc_ctx *out);
void soc_ctx_destroy(soc_ctx ctx);
soc_status soc_ctx_set_stream(soc_ctx ctx, void *hip_stream);
/* Text of the last failure on this context ("" if none).  Valid until the
 * next call on the context. */
const char *soc_last_error(soc_ctx ctx);

/* Tunables of the Monte Carlo kernels (defaults in brackets). */
typedef enum {
    SOC_OPT_STEP_CAP = 0,        /* steps per package before it is stopped [10000000] */
    SOC_OPT_BLOCK = 1,           /* threads per workgroup of the MC kernel, multiple of 64 in 64..512 [128] */
    SOC_OPT_BLOCKS_PER_CU = 2,   /* persistent workgroups launched per compute unit [6] */
    SOC_OPT_REFILL_MIN = 3,      /* refill a wave once this many lanes are idle, 1..64 [16] */
    SOC_OPT_INNER_STEPS = 4,     /* cell steps between refill checks, 1..16 [1] */
    SOC_OPT_TIMING = 5,          /* 1 = time each MC launch with HIP events [0] */
    SOC_OPT_SCATTER_MIN = 6,     /* draw new directions once this many lanes of a wave wait for one, 1..64 [1] */
    SOC_OPT_XCD_COPIES = 7,      /* 1 = each wave adds into one of 16 private copies of the absorbed array
                                    (two per XCD: the hardware XCC id and the workgroup index's parity;
                                    context scratch of 16 x ncells doubles), summed into d_absorbed by one
                                    kernel after the launch: spreads the same-address adds of hot cells
                                    over 16 addresses.  With even root dimensions the copies hold the root
                                    cells in 2 x 2 x 2 bricks, so that a package's consecutive deposits
                                    often share one memory-side transaction.  Batches created while it is
                                    1 also tally their tiled arrays in a brick-ordered scratch [1] */
    SOC_OPT_CHUNK = 8,           /* package ids a wave takes from the global counter at a time, 64..65536
                                    (smaller: finer load balance between waves) [256] */
    SOC_OPT_BATCH_LDS_CELLS = 9, /* batches created afterwards: pairs whose grid has at most this many cells
                                    are taken whole by one workgroup, which keeps the grid's absorbed array
                                    in LDS (0 = never; at most what the device's LDS per workgroup holds)
                                    [13824 = 24^3, or less if the device holds less] */
    SOC_OPT_MULTI_SPREAD = 10    /* soc_simulate_frequencies: 1 = wave w starts its rotation over the
                                    frequencies at w mod K (the waves divide over the frequencies); 0 = every
                                    wave starts at the first, the next filling in as each ends [1] */
} soc_option;
soc_status soc_ctx_set_option(soc_ctx ctx, soc_option opt, int64_t value);
soc_status soc_ctx_get_option(soc_ctx ctx, soc_option opt, int64_t *value);
/* With SOC_OPT_TIMING on: total milliseconds and number of timed MC kernel
 * launches since the last reset (synchronises the stream). */
soc_status soc_ctx_mc_timing(soc_ctx ctx, double *total_ms, int64_t *launches, int32_t reset);

/* ---------------------------------------------------------------- grid */
/* Hierarchical grid of Sect. 2.1.1.  The cells form one vector: the root
 * grid first (x fastest, then y, then z), then every cell of level 2, then
 * level 3 and so on.  Each cell holds one 32-bit word: an FP32 density >= 0,
 * or, for a refined cell, the int32 value -(index of the first cell of its
 * child octet).  Octets are 8 consecutive cells with child octant
 * o = ix + 2 iy + 4 iz (i* = 1 for the upper half of the parent on that
 * axis).  nlevels == 1 is a regular grid. */
typedef struct {
    int32_t nx, ny, nz, nlevels;
    int64_t ncells;
    const int64_t *level_offset;   /* host, nlevels+1: first cell of each level, last = ncells */
    double root_cell_cm;           /* edge of a root cell in cm */
    const uint32_t *d_words;       /* device, ncells words, borrowed */
} soc_grid_desc;

/* Validate the grid on the device (links in range, octet-aligned, every
 * octet linked exactly once, densities finite and >= 0) and build the
 * reverse links of Sect. 2.1.1 (one parent index per non-root octet) and
 * the leaf list.  Synchronises the stream.  SOC_EGRID on a malformed grid. */
soc_status soc_build_grid(soc_ctx ctx, const soc_grid_desc *desc, soc_grid *out);
/* Frees the grid's private arrays; valid before or after its context is
 * destroyed. */
void soc_grid_destroy(soc_grid grid);
/* Number of leaf cells and (optional) device pointer to the reverse links
 * (int32 per non-root octet; NULL for a regular grid). */
soc_status soc_grid_info(soc_grid grid, int64_t *n_leaves, const int32_t **d_parent);

/* ---------------------------------------------------------------- simulation */
/* Dust properties at the simulated frequency (Sect. 2.1.1: the kernel only
 * needs the data of one frequency).  w_nu is the quadrature weight (Hz) by
 * which this frequency's energy enters the frequency integral. */
typedef struct {
    double nu, w_nu;               /* Hz, Hz */
    double sigma_abs, sigma_sca;   /* cm^2 per H */
    double g;                      /* Henyey-Greenstein asymmetry, |g| < 1 */
} soc_freq;

typedef struct { double x, y, z, L_nu; } soc_point_source;   /* root units; erg s^-1 Hz^-1 */

/* Radiation sources of one call (Sect. 2.2, 3.1, 3.2).
 *  - background: isotropic intensity I_bg_nu entering through the box
 *    faces, total energy pi I_bg w A_box, n_bg packages;
 *  - point sources: n_ps <= 32 isotropic sources, each with n_ps_pk
 *    packages and energy L_nu w;
 *  - dust emission at temperatures d_T (NULL = off): cell c emits
 *    L_c = 4 pi sigma_abs n_c V_c B_nu(T_c) w; dust_mode 0 sends the same
 *    number of packages from every leaf (n_dust must be a multiple of the
 *    leaf count), dust_mode 1 draws n_dust packages in proportion to the
 *    cell luminosity by systematic sampling (each cell gets the floor or
 *    the ceiling of its share N L_c / sum L, each package carries
 *    sum L / N);
 *  - dust_mode 2, the reference-field correction (Sect. 2.1.2): the
 *    packages carry only the difference dL_c = L_c - L_ref,c between the
 *    emission at d_T and the reference emission d_L_ref of this frequency
 *    (device, ncells FP64, erg s^-1 including w).  Cells are drawn in
 *    proportion to |dL_c| as in mode 1 and each package carries the sign
 *    of dL_c (negative packages deposit negative energy).  In the same call
 *    d_L_ref is blended towards the current emission, L_ref += ref_beta
 *    dL (ref_beta in [0, 1]; 0 leaves it unchanged; the packages use the
 *    reference as it was on entry).  The absorbed energies of the
 *    reference field itself are the caller's (see soc_reference_blend);
 *  - dust_cap > 0 (modes 1 and 2): the expected number of packages of one
 *    cell is limited to dust_cap (Sect. 3.2), min(N |dL_c| / S, dust_cap)
 *    with S = sum |dL|; a package of a capped cell carries |dL_c| /
 *    dust_cap, and the excess is not re-assigned to other cells (fewer
 *    than n_dust packages are emitted; the rest are counted but carry
 *    nothing).  0 = no cap;
 *  - diagonal ALI (Sect. 2.1.2, 4.1): with d_ali_self and d_ali_emitted
 *    (device, ncells FP64 each, accumulated +=), what a dust package
 *    deposits in the cell that emitted it -- on its way out, on returning
 *    after scatterings, the weight-floor remainder -- goes to d_ali_self
 *    instead of d_absorbed, and its initial weight is added to
 *    d_ali_emitted of that cell; other classes are unaffected.  The
 *    temperature solve soc_update_temperature_ali then uses them. */
typedef struct {
    double I_bg_nu;
    int32_t n_ps;
    const soc_point_source *ps;    /* host, n_ps entries */
    const float *d_T;              /* device, ncells temperatures, or NULL */
    uint64_t n_bg, n_ps_pk, n_dust;
    int32_t dust_mode;             /* 0 uniform, 1 weighted, 2 reference-field correction */
    double *d_L_ref;               /* dust_mode 2: device, ncells FP64 reference emission, updated in place */
    double ref_beta;               /* dust_mode 2: blend weight of this call's emission in d_L_ref */
    double dust_cap;               /* modes 1, 2: packages per cell at most (expected), 0 = no cap */
    double *d_ali_self;            /* diagonal ALI (both or neither; modes 0, 1): device FP64 ncells, += */
    double *d_ali_emitted;         /*   see below */
} soc_sources;

typedef struct {
    uint64_t packages, cell_steps, scatterings, runaways;
    double e_emitted, e_absorbed, e_escaped;   /* erg s^-1 */
} soc_sim_stats;

/* Monte Carlo pass at one frequency: emit every package, draw its free
 * path in scattering optical depth, step it cell by cell depositing
 * W (1 - exp(-k_abs d)) in each cell crossed, scatter it with the
 * Henyey-Greenstein function, until it leaves the box, falls below 1e-12
 * of its initial weight or reaches the step cap (the rest of its weight is
 * then deposited in its cell).  Deposits are added (+=) to d_absorbed
 * (FP64, ncells).  Random numbers come from Philox4x32-10 with counter
 * (block, package id, freq_index, iteration << 8 | class) and key = seed,
 * class 0 = background, 1 = dust, 2 + s = point source s, so each
 * package's numbers depend only on its identity.  If stats is non-NULL the
 * call synchronises and fills it with this call's totals. */
soc_status soc_simulate_frequency(soc_ctx ctx, soc_grid grid, const soc_freq *freq,
                                  const soc_sources *src, uint64_t seed, uint32_t iteration,
                                  uint32_t freq_index, double *d_absorbed, soc_sim_stats *stats);

/* The work of K soc_simulate_frequency calls on one grid -- frequency k
 * with freqs[k], srcs[k] and freq_indices[k], the same seed and iteration
 * -- in one persistent launch, all deposits added to d_absorbed: the
 * frequency-integrated absorbed energy the temperature kernel needs
 * (Sect. 2.1.1).  Every package has the random numbers it has in the
 * single call, so the counters are identical and d_absorbed equal up to
 * FP64 summation order.  Waves take the frequencies in a rotation and
 * move on when one has no ids left, so the tail of a launch comes only at
 * the end, not after every frequency.  Each frequency's setup (dust
 * luminosities, selection of cells) runs before the launch and keeps its
 * own package-to-cell list until then (context scratch: 4 B per weighted
 * dust package, plus 8 B per cell for frequencies whose kernel reads the
 * luminosities: dust modes 0 and 2 and capped emission).  The frequencies
 * in weighted mode 1 without a cap have their tables built together, a
 * few launches for all of them (context scratch: 8 B per cell and
 * frequency, when that comes to at most 16 GiB; one frequency at a time
 * otherwise); the package cells are the same either way.  The
 * diagonal-ALI tallies (Sect. 2.1.2) are taken as in
 * soc_simulate_frequency when every srcs[k] names the same d_ali_self and
 * d_ali_emitted (SOC_EINVAL when they differ between frequencies).
 * 1 <= K <= 4096.  Synchronises the stream before it starts (the argument
 * blocks are staged on the host); not allowed during graph capture. */
soc_status soc_simulate_frequencies(soc_ctx ctx, soc_grid grid, int32_t K, const soc_freq *freqs,
                                    const soc_sources *srcs, const uint32_t *freq_indices, uint64_t seed,
                                    uint32_t iteration, double *d_absorbed, soc_sim_stats *stats);

/* soc_simulate_frequency without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels, random
 * numbers and results (up to FP64 summation order) as
 * soc_simulate_frequency; the caller still owns d_absorbed and the other
 * device inputs.  Its scratch (refill counter, per-call statistics, the
 * dust-emission tables and the per-XCD private copies of the tallies) is a
 * fixed array of about 13 MB per device, held until the process ends, so:
 *  - grids of at most 32768 cells (all levels) and, in the weighted dust
 *    modes (1, 2), at most 2^20 dust packages per call; larger inputs
 *    return SOC_EINVAL with a message, before any launch;
 *  - every call on a device shares that device's array: calls that
 *    overlap on one device (several contexts or streams) race and must be
 *    serialised by the caller; each call clears what must start at zero;
 *  - the context's timing option is ignored (no events are created); the
 *    running totals of soc_read_stats include these calls;
 *  - stats, if non-NULL, is filled after a synchronisation (not allowed
 *    during graph capture: SOC_ESTATE).
 * Returns SOC_EHIP if the array's device address could not be resolved
 * when the context was created. */
soc_status soc_simulate_frequency_noalloc(soc_ctx ctx, soc_grid grid, const soc_freq *freq,
                                          const soc_sources *src, uint64_t seed, uint32_t iteration,
                                          uint32_t freq_index, double *d_absorbed, soc_sim_stats *stats);

/* Reference-field running mean (Sect. 2.1.2): d_ref += beta (d_x - d_ref)
 * over n FP64 device values, enqueued on the context's stream.  With the
 * weight beta = n_i / (sum of the package counts so far) of iteration i it
 * keeps the reference absorption the package-weighted mean of the
 * iterations' absorption estimates.  beta in [0, 1]; SOC_EINVAL otherwise. */
soc_status soc_reference_blend(soc_ctx ctx, int64_t n, double beta, const double *d_x, double *d_ref);

/* Statistics summed over every soc_simulate_frequency call on the context
 * since the last reset (synchronises). */
soc_status soc_read_stats(soc_ctx ctx, soc_sim_stats *out, int32_t reset);

/* Deterministic single-package mode: trace n packages of one class
 * (ids[i] within that class) with the same random numbers and the same
 * transport code as soc_simulate_frequency, recording up to max_seg
 * segments each.  precision 0 = the FP32 production arithmetic, 1 = the
 * same code in FP64.  out (host) holds n * max_seg segments; n_seg (host)
 * receives each package's full segment count (may exceed max_seg). */
typedef struct { int64_t cell; double ds; int32_t event; int32_t pad; } soc_segment;
enum { SOC_EV_CROSS = 0, SOC_EV_SCATTER = 1, SOC_EV_ESCAPE = 2, SOC_EV_FLOOR = 3, SOC_EV_RUNAWAY = 4 };
soc_status soc_trace_packages(soc_ctx ctx, soc_grid grid, const soc_freq *freq, const soc_sources *src,
                              uint64_t seed, uint32_t iteration, uint32_t freq_index, uint32_t cls,
                              const uint32_t *ids, int32_t n, int32_t precision,
                              soc_segment *out, int32_t max_seg, int32_t *n_seg);

/* ---------------------------------------------------------------- temperature */
/* Equilibrium temperature table (Sect. 2.1.1 temperature kernel): built on
 * the device from the K frequencies of the dust emission model (host
 * arrays nu, w_nu, sigma_abs) as Gamma(T) = 4 pi sum_k w_k sigma_abs,k
 * B_nu_k(T) on nT log-spaced temperatures in [T_floor, T_max], 16 <= nT <= 4096
 * (the table is staged in LDS by the temperature kernel). */
typedef struct soc_temp_table_s *soc_temp_table;
soc_status soc_temp_table_build(soc_ctx ctx, int32_t K, const double *nu, const double *w_nu,
                                const double *sigma_abs, double T_floor, double T_max, int32_t nT,
                                soc_temp_table *out);
void soc_temp_table_destroy(soc_temp_table t);   /* valid before or after its context is destroyed */

typedef struct {
    double mean_T;            /* over leaves with n > 0 */
    double hot5_mean_T;       /* mean over the hottest 5% (ceil) of those leaves */
    double mean_rel_change;   /* mean |T_new - T_old| / T_old over cells with T_old > 0 (NaN if none) */
    uint64_t clamped;         /* leaves clamped to T_floor (incl. unhit) or T_max */
} soc_temp_stats;

/* Solve Gamma(T_c) = A_c / (n_c V_c) for every leaf (inverse of the
 * tabulated log-log relation).  Empty and refined cells get T = 0; unhit
 * cells and values outside the table are clamped to [T_floor, T_max] and
 * counted.  d_T_old may equal d_T_new or be NULL (then no relative
 * change).  If stats is non-NULL the call synchronises and fills it (the
 * hottest-5% mean is found exactly from a coarse log-T histogram and a
 * fine histogram of the bin holding the threshold). */
soc_status soc_update_temperature(soc_ctx ctx, soc_grid grid, soc_temp_table table,
                                  const double *d_absorbed, const float *d_T_old, float *d_T_new,
                                  soc_temp_stats *stats);

/* Diagonal ALI (Sect. 2.1.2, 4.1): as soc_update_temperature, with each
 * cell's own absorption-emission cycle taken exactly.  beta_c =
 * d_ali_self / d_ali_emitted (0 where the cell emitted nothing) is the
 * fraction of its emission the cell absorbs itself, so its emission
 * equals d_absorbed (what reached it from elsewhere) plus beta_c times
 * itself: Gamma(T_c) n_c V_c (1 - beta_c) = d_absorbed_c.  The escape
 * probability 1 - beta_c is kept >= 1e-6.  Tallies as filled by
 * soc_simulate_frequency (device FP64, ncells each, read only). */
soc_status soc_update_temperature_ali(soc_ctx ctx, soc_grid grid, soc_temp_table table,
                                      const double *d_absorbed, const double *d_ali_self,
                                      const double *d_ali_emitted, const float *d_T_old, float *d_T_new,
                                      soc_temp_stats *stats);

/* The same statistics (mean_T, hot5_mean_T; mean_rel_change and clamped
 * are 0) of a given temperature field d_T (device FP32, ncells, read only)
 * over the leaves with n > 0 -- the convergence statistics of Sect. 3.3
 * for a field that did not come from a solve (a learned starting field).
 * The table supplies the log-T histogram range.  Synchronises. */
soc_status soc_temperature_stats(soc_ctx ctx, soc_grid grid, soc_temp_table table, const float *d_T,
                                 soc_temp_stats *stats);

/* ---------------------------------------------------------------- map */
/* Emission map (Sect. 2.1.1 map kernel, pixel = smallest cell, Sect. 3.2)
 * seen along root-grid axis `axis & 3` (0..2) from the positive side, or
 * from the negative side when bit 2 is set:
 * I = sum over cells on the ray of S_c (1 - exp(-dtau)) exp(-tau_front),
 * S_c = (sigma_abs / sigma_ext) B_nu(T_c), dtau = sigma_ext n_c ds.
 * d_image (device, FP32) has npy rows of npx pixels: npx spans the lower of
 * the two other axes, npy the higher, each N * 2^(nlevels-1) pixels. */
soc_status soc_map(soc_ctx ctx, soc_grid grid, const soc_freq *freq, const float *d_T, int32_t axis,
                   float *d_image, int32_t npx, int32_t npy);

/* ---------------------------------------------------------------- scattered light */
/* Image of scattered light (Sect. 2.1.1: scattered-light images come from
 * separate runs with forced first scattering and peel-off).  The external
 * field and point sources of `src` are simulated at one frequency (no dust
 * emission, no tallies; src->d_T must be NULL or n_dust 0).  At every
 * scattering a package of weight W at r, moving along u, adds
 *   W Phi(u . o) exp(-tau_ext) / (A_pix w_nu)
 * to the pixel under r: o the direction towards a distant observer on the
 * positive side of root axis axis & 3 (bit 2: negative side), Phi the
 * Henyey-Greenstein function normalised over the sphere (1/4pi for
 * |g| < 1e-4), tau_ext the extinction optical depth from r to the box
 * boundary along o, A_pix the pixel area.  forced != 0: each package first
 * keeps the fraction 1 - exp(-tau_esc) of its weight that scatters before
 * leaving the box (tau_esc the scattering optical depth ahead of it) and
 * draws its first free path from the exponential truncated at tau_esc.
 * direct != 0: point sources add their attenuated direct light W/(4pi)
 * exp(-tau_ext) to their pixel.  max_scatter > 0 stops a package after its
 * max_scatter-th scattering (0 = all orders).  d_image (device FP64, npy
 * rows of npx pixels laid out as soc_map's, erg s^-1 cm^-2 Hz^-1 sr^-1) is
 * accumulated (+=).  Random numbers as soc_simulate_frequency (forcing
 * reuses the uniform of the first free path).  stats (host, optional)
 * makes the call synchronise. */
typedef struct {
    int32_t axis;          /* 0..2, | 4 for an observer on the negative side */
    int32_t forced;        /* forced first scattering */
    int32_t max_scatter;   /* 0 = all orders */
    int32_t direct;        /* add the direct light of point sources */
} soc_scatter_params;
typedef struct {
    uint64_t packages, cell_steps, scatterings, ray_steps;   /* ray_steps: steps of the rays to the boundary */
    double e_emitted, e_escaped;
} soc_scatter_stats;
soc_status soc_scatter_map(soc_ctx ctx, soc_grid grid, const soc_freq *freq, const soc_sources *src, uint64_t seed,
                           uint32_t iteration, uint32_t freq_index, const soc_scatter_params *params,
                           double *d_image, int32_t npx, int32_t npy, soc_scatter_stats *stats);

/* ---------------------------------------------------------------- stochastic heating */
/* Stochastically heated grains (Sect. 2.1.1, Appendix A, "thermal continuous"
 * approximation).  A grain model: K frequencies nu (Hz, increasing) with
 * quadrature weights w (Hz), S grain sizes with abundances (grains per H),
 * absorption cross sections sigma[S][K] (cm^2 per grain) and enthalpy grids
 * U[S][N] (erg per grain, increasing) at temperatures T[S][N] (K); all host
 * arrays, copied.  K <= 128, 2 <= N <= 128, 1 <= S <= 4096.  The model is
 * tied to ctx.  Errors: SOC_EINVAL for sizes out of range, frequencies or
 * enthalpies that do not increase, non-positive temperatures, negative or
 * non-finite weights, abundances or cross sections (*out stays NULL);
 * SOC_ENOMEM when its device tables cannot be allocated. */
typedef struct soc_shg_model_s *soc_shg_model;
soc_status soc_shg_model_create(soc_ctx ctx, int32_t K, const double *nu, const double *w, int32_t S,
                                const double *abundance, const double *sigma, int32_t N, const double *U,
                                const double *T, soc_shg_model *out);
void soc_shg_model_destroy(soc_shg_model model);   /* valid before or after its context is destroyed */

/* Temperature distributions and emission of every leaf.  d_absorbed
 * (device FP64 [K][ncells]): the energy absorbed per second in each band
 * (erg/s per cell; the tallies of one soc_simulate_frequency call per
 * band, with the model's total cross section).  Size s takes the share
 * abundance_s sigma_sk / sum_s abundance_s sigma_sk of band k, divided among
 * abundance_s n_H V grains, as r_k = photons per grain per second.  A photon
 * raises a grain in bin i to U_i + h nu_k, split between the two bins
 * around it in proportion to the distance (a target above the top bin goes
 * to the top bin); a grain in bin i > 0 cools into bin i-1 at the rate
 * L(T_i)/(U_i - U_{i-1}), L(T) = 4 pi sum_k sigma_sk B_nu_k(T) w_k.  The
 * stationary populations P (sum 1) follow by forward substitution in FP64.
 * d_emission (device FP64 [K][ncells], overwritten): sum over sizes of the
 * grain count times 4 pi sigma_sk sum_i P_i B_nu_k(T_i), erg s^-1 Hz^-1 per
 * cell (0 in empty and refined cells).  d_P (device FP64
 * [ncells][S][N], optional): the populations.  Enqueued on ctx's stream.
 * Errors: SOC_EINVAL for NULL arguments or a grid or model of another
 * context; SOC_EHIP when the launch fails. */
soc_status soc_shg_solve(soc_ctx ctx, soc_grid grid, soc_shg_model model, const double *d_absorbed,
                         double *d_emission, double *d_P);

/* ---------------------------------------------------------------- batches */
/* Many independent Monte Carlo problems -- (cloud model, frequency) pairs
 * over regular grids of any size -- simulated by one persistent launch that
 * pulls tiles of package ids from a queue (the work of soc_simulate_frequency
 * for each pair, background and point sources).  Pair i uses the Philox key
 * (seed low word, seed high word XOR grids[pairs[i].grid] index), so its
 * random numbers equal those of a single soc_simulate_frequency call with
 * seed ^ ((uint64_t)grid << 32). */
typedef struct {
    int32_t grid;                  /* index into the grids given to soc_batch_create */
    uint32_t freq_index;           /* Philox counter word of this frequency */
    soc_freq freq;
    double I_bg_nu;
    uint64_t n_bg;
    int32_t n_ps;                  /* <= 32 */
    const soc_point_source *ps;    /* host, copied at creation */
    uint64_t n_ps_pk;
    double *d_absorbed;            /* device FP64 of the grid's ncells, accumulated (+=) */
} soc_batch_pair;

typedef struct soc_batch_s *soc_batch;
/* Copies the pair table and the tile queue (tiles of at most tile_packages
 * ids, ordered by decreasing estimated cost) to the device.  Pairs whose
 * grid has at most SOC_OPT_BATCH_LDS_CELLS cells (the option's value now)
 * are not tiled: each is one work item of a workgroup that tallies the
 * grid in LDS, taken before the tiles (same random numbers and results up
 * to FP64 summation order).  A batch with such pairs launches 512-lane
 * workgroups, one or two per compute unit as their LDS allows
 * (SOC_OPT_BLOCK and SOC_OPT_BLOCKS_PER_CU shape the other batches).
 * With SOC_OPT_XCD_COPIES 1 (now), an array that only tiled pairs of one
 * grid with even dimensions add into is tallied in a batch-owned scratch
 * copy in 2 x 2 x 2 brick order (one FP64 per cell of every such array),
 * which each soc_batch_run adds into the array after its launch and leaves
 * zero.  Synchronises.  soc_batch_info counts the LDS pairs among the
 * tiles. */
soc_status soc_batch_create(soc_ctx ctx, int32_t n_grids, const soc_grid *grids, int32_t n_pairs,
                            const soc_batch_pair *pairs, uint64_t seed, uint64_t tile_packages, soc_batch *out);
void soc_batch_destroy(soc_batch b);
soc_status soc_batch_info(soc_batch b, int32_t *n_tiles, uint64_t *n_packages);
/* One persistent launch over every tile.  iteration: the Philox iteration
 * word (bits 8..31 of counter word 3); SOC_ITER_ADVANCE instead adds one to
 * the value the previous run used (so that a captured graph advances on
 * every replay).  With stats non-NULL the call synchronises and returns
 * the totals of this run; pass NULL inside a graph capture. */
#define SOC_ITER_ADVANCE 0xFFFFFFFFu
soc_status soc_batch_run(soc_batch b, uint32_t iteration, soc_sim_stats *stats);

/* ---------------------------------------------------------------- ceilings */
/* Device micro-benchmarks for the roofline of the Monte Carlo kernel
 * (times one launch with HIP events, synchronises):
 *  which 0: FP64 atomic adds of 1.0, per_thread per thread, into d_buf
 *           (n doubles): mode 0 random addresses; mode 1 random addresses
 *           in one slice of n doubles per XCD, selected by the hardware XCC
 *           id, so d_buf must hold 8 n doubles; mode 2 each wave adds to
 *           the 64 consecutive doubles of one random 64-double block
 *           (n >= 64); mode 3 random addresses in a 4096-double LDS array
 *           per workgroup, folded into d_buf[0..4095] (n >= 4096);
 *           mode 4 random FP32 atomic adds into n floats; mode 5 random
 *           64-bit and mode 6 random 32-bit integer atomic adds of 1 into
 *           n words;
 *  which 1: dependent random 4-byte gathers over n words of d_buf;
 *  which 2: streaming copy of n bytes from d_buf to d_buf2.
 * ms receives the kernel time. */
soc_status soc_ubench(soc_ctx ctx, int32_t which, void *d_buf, void *d_buf2, uint64_t n, int32_t per_thread,
                      int32_t mode, int32_t blocks, int32_t threads, double *ms);

/* ---------------------------------------------------------------- graphs */
/* Capture the library calls issued on the context's stream between
 * soc_graph_begin and soc_graph_end into a HIP graph (stream capture,
 * relaxed mode) and replay it with soc_graph_launch.  The stream must not
 * be the null stream.  Calls that allocate or synchronise (statistics,
 * traces, grid or table construction) return SOC_ESTATE while capturing;
 * library scratch is reset with kernels, never memset nodes. */
typedef struct soc_graph_s *soc_graph;
soc_status soc_graph_begin(soc_ctx ctx);
soc_status soc_graph_end(soc_ctx ctx, soc_graph *out);
soc_status soc_graph_launch(soc_graph g);
void soc_graph_destroy(soc_graph g);

/* ---------------------------------------------------------------- surrogate */
/* Learned starting temperatures.  The paper speeds up the iteration by
 * starting it from a reference field (Sec. 2.1.2); here a 3-D
 * convolutional U-Net, trained on fields the plain method produced,
 * predicts the field the iteration starts from, and the plain iterations
 * that follow keep the result unbiased.
 *
 * Network: `levels` resolution levels with base * 2^l channels; each level
 * has two 3^3 convolutions (zero padding) with a leaky ReLU of slope 0.1; a
 * stride-2 2^3 convolution (+ leaky ReLU) goes down, a stride-2 transposed
 * 2^3 convolution (+ leaky ReLU) comes up and is concatenated after the
 * skip tensor of the level; a last 3^3 convolution without activation
 * gives `cout` channels.  BF16 activations and weights in the matrix-core
 * products, FP32 accumulation, FP32 master weights and Adam state.
 *
 * Parameters: one FP32 array, layer by layer in the order
 *   e0a e0b d0 e1a e1b d1 ... e{L-1}a e{L-1}b u{L-2} q{L-2}a q{L-2}b ... u0 q0a q0b out
 * (e encoder convolutions, d down, u up, q decoder convolutions), each as
 * weights w[kz][ky][kx][cin][cout] followed by biases b[cout].
 *
 * Tensors passed to the calls are device FP32, channels-last:
 * x[n][nz][ny][nx][cin], y[n][nz][ny][nx][cout].  The network owns its
 * parameters, optimiser state, activations and gradients (allocated at
 * creation for up to nmax samples); calls enqueue on the context's stream.
 * forward, backward and adam allocate nothing and may be captured in a
 * graph; calls with host buffers synchronise and return SOC_ESTATE while
 * capturing. */
typedef struct soc_unet_s *soc_unet;
typedef struct {
    int32_t cin, cout;     /* input and output channels (>= 1) */
    int32_t base, levels;  /* level-0 channels (a positive multiple of 16), 1 <= levels <= 6 */
    int32_t nmax;          /* largest batch */
    int32_t nz, ny, nx;    /* cells of one sample, each divisible by 2^(levels-1) */
} soc_unet_desc;
/* He-normal weights from seed, zero biases.  SOC_EINVAL on a bad shape. */
soc_status soc_unet_create(soc_ctx ctx, const soc_unet_desc *desc, uint64_t seed, soc_unet *out);
void soc_unet_destroy(soc_unet u);
soc_status soc_unet_param_count(soc_unet u, int64_t *count);
/* 2 x multiply-adds of one forward pass over n samples (unpadded shapes). */
soc_status soc_unet_flops(soc_unet u, int32_t n, int64_t *flops);
/* Host FP32 arrays of soc_unet_param_count elements. */
soc_status soc_unet_set_params(soc_ctx ctx, soc_unet u, const float *h_params);
soc_status soc_unet_get_params(soc_ctx ctx, soc_unet u, float *h_params);
soc_status soc_unet_get_grads(soc_ctx ctx, soc_unet u, float *h_grads);
/* y = net(x) for n <= nmax samples. */
soc_status soc_unet_forward(soc_ctx ctx, soc_unet u, int32_t n, const float *d_x, float *d_y);
/* Gradients of sum(dy * y) with respect to every parameter, for the
 * inputs of the last forward call; they replace the previous gradients. */
soc_status soc_unet_backward(soc_ctx ctx, soc_unet u, const float *d_dy);
/* Test hooks for per-layer parity (layers indexed in parameter order,
 * soc_unet_param_count's layout).  soc_unet_backward_to runs the backward
 * pass of soc_unet_backward up to and including layer stop_layer (its
 * weight gradient, and its backward-data pass where it has one) and
 * returns; gradients of the layers not reached are left as they were.
 * soc_unet_read copies one stored BF16 tensor of a layer to host FP32,
 * real channels only, [n][positions][channels] for the batch n of the last
 * forward (count must equal that size): which 0 its forward input, 1 its
 * forward output (SOC_EINVAL for the last layer, whose output is the
 * caller's FP32 array), 2 the output-side gradient its weight gradient and
 * backward-data pass consumed, 3 its backward-data result (leaky-ReLU slope
 * of the input and, for a down convolution, the skip gradient applied).
 * 2 and 3 are defined for the layer the last backward stopped at (later
 * layers of a full backward overwrite them).  Synchronises. */
soc_status soc_unet_backward_to(soc_ctx ctx, soc_unet u, const float *d_dy, int32_t stop_layer);
soc_status soc_unet_read(soc_ctx ctx, soc_unet u, int32_t layer, int32_t which, float *h_out, int64_t count);
/* Mean of (y - t)^2 over n samples x cells x cout into *loss (host; NULL:
 * no result and no synchronisation) and its gradient 2 (y - t) / count into
 * d_dy (NULL: not written). */
soc_status soc_unet_mse(soc_ctx ctx, soc_unet u, int32_t n, const float *d_y, const float *d_t, float *d_dy,
                        double *loss);
/* One Adam step (bias-corrected moments, step counts from 1) with the
 * current gradients; refreshes the BF16 weight copies. */
soc_status soc_unet_adam(soc_ctx ctx, soc_unet u, float lr, float beta1, float beta2, float eps, int32_t step);

/* The network's input and output on a regular cubic grid of n^3 cells
 * seen as S^3 blocks of b^3 cells (n = b S; SOC_EINVAL for octrees,
 * non-cubic grids or S not dividing n).  The plain method's first
 * iteration (constant sources only) gives T1, the temperatures the dust
 * iterations start from (Sect. 2.1.2, 3.3); the network predicts how far
 * the dust re-emission raises them.  All temperatures are in cells with
 * density 0 replaced by the table's T_floor, and below T_floor raised to
 * it.
 *
 * soc_surrogate_features writes d_features[S^3][4] (device FP32,
 * z-major like the grid, channels last): per block,
 *   0: log10(sigma_v <n> s + 1e-4) / 2, s the block edge in cm;
 *   1: log10(1 + sum_p L_p / (4 pi d_p^2) / F_ext) / 4, the unattenuated
 *      bolometric flux of the point sources against the external field's
 *      4 pi J, F_ext = 4 pi sum_k w_k I_k, L_p = sum_k w_k L_p,k;
 *   2: (log10 T_thin - 1.5) / 0.5, T_thin the equilibrium temperature in
 *      the unattenuated radiation field, from the table:
 *      Gamma(T_thin) = 4 pi (sum_k w_k sigma_k I_k
 *                            + sum_p sum_k w_k sigma_k L_p,k / (16 pi^2 d_p^2));
 *   3: (mean of log10 T1 over the block - 1.5) / 0.5;
 * d_p^2 = (|r - r_p|^2 + 1/4) s^2 between the block centre and source p.
 * Host inputs: K frequencies' w_nu, sigma_abs (cm^2 per H), I_bg; sigma_v
 * the 0.55 um extinction cross section; n_ps <= 32 sources at ps_pos
 * [n_ps][3] (root units) with ps_Lnu [n_ps][K]; d_T1 device FP32 ncells.
 *
 * Coarse arrays hold several channels: block i's value of channel c is
 * element [i * stride + c] (0 <= c < stride), so a network with several
 * outputs is read and trained in place.
 *
 * soc_surrogate_target writes channel `channel` of d_target (S^3 blocks):
 * the block mean of log10(T / T1) divided by scale > 0 (the training
 * target of the temperatures).  soc_surrogate_target_absorbed does the
 * same with the absorbed energies (device FP64 ncells each): the block
 * mean of log10(A / A1) over the cells with dust and A1, A > 0 (other
 * cells count 0), A1 the constant sources' absorption (Sect. 2.1.2: the
 * reference field's stored absorptions).
 *
 * soc_surrogate_apply writes d_T (ncells): with r channel `channel` of the
 * network output d_pred times scale plus offset, interpolated trilinearly
 * to the cell centres (fine cell j maps to coarse coordinate
 * (j + 1/2) / b - 1/2, clamped to [0, S - 1]), T = T1 10^r clamped to
 * [T_floor, T_max]; 0 in cells of density 0.  soc_surrogate_apply_absorbed
 * writes d_A = A1 10^r (scale only; 0 in cells of density 0).
 * All of them only enqueue work on the context's stream. */
soc_status soc_surrogate_features(soc_ctx ctx, soc_grid grid, soc_temp_table table, int32_t S, int32_t K,
                                  const double *w_nu, const double *sigma_abs, const double *I_bg, double sigma_v,
                                  int32_t n_ps, const double *ps_pos, const double *ps_Lnu, const float *d_T1,
                                  float *d_features);
soc_status soc_surrogate_target(soc_ctx ctx, soc_grid grid, soc_temp_table table, int32_t S, const float *d_T,
                                const float *d_T1, double scale, float *d_target, int32_t stride, int32_t channel);
soc_status soc_surrogate_target_absorbed(soc_ctx ctx, soc_grid grid, int32_t S, const double *d_A,
                                         const double *d_A1, double scale, float *d_target, int32_t stride,
                                         int32_t channel);
soc_status soc_surrogate_apply(soc_ctx ctx, soc_grid grid, soc_temp_table table, int32_t S, const float *d_pred,
                               int32_t stride, int32_t channel, double scale, double offset, const float *d_T1,
                               float *d_T);
soc_status soc_surrogate_apply_absorbed(soc_ctx ctx, soc_grid grid, int32_t S, const float *d_pred, int32_t stride,
                                        int32_t channel, double scale, const double *d_A1, double *d_A);

#ifdef __cplusplus
}
#endif
#endif /* SOC_H */
