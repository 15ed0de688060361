// soc_kernels.h -- argument blocks and launchers shared by the C-ABI host
// code (api.hip) and the kernel translation units.  Host-visible only; no
// device code here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace soc {

// Private copies of a tally for the Monte Carlo launches: two per XCD, so
// that the same-address adds of the hottest cells spread over 16 addresses
// (8 copies: 410 ms per benchmark iteration, 16: 387 ms, 32: 400 ms, the
// fold after each launch then costing more than it saves).
constexpr uint32_t kPrivPerXcd = 2;
constexpr uint32_t kPrivCopies = 8 * kPrivPerXcd;

// Source classes: the low byte of Philox counter word 3.
constexpr uint32_t kClassBg = 0;
constexpr uint32_t kClassDust = 1;
constexpr uint32_t kClassPs0 = 2;

// Segment end events (same values as SOC_EV_* in soc.h).
constexpr int kEvCross = 0;
constexpr int kEvScatter = 1;
constexpr int kEvEscape = 2;
constexpr int kEvFloor = 3;
constexpr int kEvRunaway = 4;

constexpr int kMaxPs = 32;
// LDS deposit ring per lane of the MC kernels: 16 entries, flushed as 16
// consecutive deposits of each of 4 packages per atomic instruction
// (198.5 ms per benchmark pass, against 207.0 ms with 8 entries)
constexpr int kDepSlots = 16;
constexpr int kRingStride = kDepSlots + 1;   // LDS entries per lane's ring (one pad entry)
constexpr int kMcMaxBlock = 512;  // MC workgroup size limit (LDS rings: 102 KB at 512)
constexpr int kMaxLevels = 16;

struct PsArg {
    double x, y, z;   // root units
    double W;         // energy per package
};

struct DevStats {
    unsigned long long packages, steps, scatterings, runaways;
    double emitted, absorbed, escaped;
};

// Everything one Monte Carlo launch needs, passed by value.
struct McArgs {
    // grid
    const uint32_t *words;
    const int32_t *parent;      // reverse links (octree only)
    int32_t nx, ny, nz, nlevels;
    int64_t ncells, nroot;
    int64_t level_offset[kMaxLevels + 1];
    // frequency: k = sigma * root_cell_cm per unit density per root unit
    float ks_f, ka_f, g_f;
    double ks_d, ka_d, g_d;
    // sources
    uint64_t n_bg, n_ps_pk, n_dust, n_total;
    int32_t n_ps, dust_mode;
    double W_bg;
    double face_cum[6];
    double face_tot;
    PsArg ps[kMaxPs];
    const double *dust_L;        // per-cell luminosity; its difference to the reference (mode 2)
    const double *dust_S;        // weighted modes: device scalar, sum over cells of |dust_L|
    double dust_cap;             // weighted modes: expected packages per cell at most this (0 = no cap)
    const int32_t *dust_cell;    // cell of every dust package (weighted modes; -1 = none)
    const int64_t *leaves;       // leaf list (octree, uniform mode); NULL = identity
    uint64_t per_leaf;
    // random numbers
    uint32_t key0, key1, freq_index, iteration;
    // transport
    int64_t step_cap;
    double *absorbed;
    double *priv;                // NULL, or kPrivCopies private copies of ncells (see priv_index)
    int32_t brick;               // 1: the private copies hold the root cells (even root dimensions)
                                 // in 2 x 2 x 2 bricks (brick_cell), folded back to the cell order
    double *ali_self;            // diagonal ALI (NULL = off): dust deposits in the emitting cell
    double *priv_self;           // NULL, or kPrivCopies private copies of ali_self
    // persistent scheduling
    unsigned long long *next_id;
    DevStats *st_call, *st_total;
    int32_t refill_min, inner_steps, chunk, scatter_min;
};

// Scattered-light image (peel-off).  The observer is along +/- axis; the
// image has npy rows of npx pixels of edge psz root units; scale is
// 1 / (A_pix w_nu).  totals: packages, steps, scatterings, ray-march steps,
// emitted and escaped energy (device doubles, +=).
struct PeelArgs {
    int32_t axis, npx, npy, forced, max_scatter, direct;
    float ox, oy, oz;
    double psz, scale;
    double *image;
    double *totals;
};

// Stochastically heated grains: model tables on the device (S sizes, K
// frequencies, N enthalpy bins).
constexpr int kShgMaxK = 128;
constexpr int kShgMaxN = 128;
struct ShgModelDev {
    int32_t S, K, N;
    const double *nu, *hnu, *inv_hnu;   // [K]
    const double *abundance;            // [S] grains per H
    const double *sigma;                // [S][K] cm^2 per grain
    const double *U, *T;                // [S][N]
    double *share;                      // [S][K] share of each size in the absorption of band k
    double *emit;                       // [S][N][K] 4 pi sigma B_nu(T_i)
    double *icool;                      // [S][N] inverse cooling rate from bin i to i-1: (U_i - U_i-1) / L(T_i)
    double *idu;                        // [S][N] 1 / (U_i - U_i-1), 0 at i = 0
    uint8_t *ks;                        // [S][ks stride] ks[j][i] (j, i < N): photons k < ks of bin i land below
                                        // bin j (K at j = N-1); 16-byte aligned, each size padded to 16 bytes
    int32_t *band;                      // [S] up[j][i] = 0 for j - i >= band
};
struct ShgArgs {
    ShgModelDev model;
    const uint32_t *words;
    int64_t ncells;
    int64_t level_offset[kMaxLevels + 1];
    int32_t nlevels;
    double root_cell_cm;
    const double *absorbed;             // [K][ncells]
    double *emission;                   // [K][ncells]
    double *P;                          // [ncells][S][N] or NULL
};
// bytes of one size's ks table, a multiple of 16 for vector copies
__host__ __device__ inline int shg_ks_stride(int N)
{
    return (N * N + 15) & ~15;
}
hipError_t launch_shg_prep(const ShgModelDev &m, const double *w, hipStream_t s);
hipError_t launch_shg(const ShgArgs &a, hipStream_t s);

struct SegmentDev {
    int64_t cell;
    double ds;
    int32_t event, pad;
};

struct TraceArgs {
    uint32_t cls;
    const uint32_t *ids;
    int32_t n, max_seg;
    SegmentDev *out;
    int32_t *nseg;
};

// Weight of a package of cell c in the weighted dust modes: L_c over the
// cell's expected count min(N |L_c| / S, cap), i.e. S / N (= WN) or, for a
// capped cell, |L_c| / cap, with the sign of L_c.
__device__ inline double weighted_package_weight(double WN, double cap, double Lc)
{
    const double m = cap > 0.0 ? fmax(WN, fabs(Lc) / cap) : WN;
    return copysign(m, Lc);
}

// ---- launchers (each returns the launch status) ----
// Regular-grid kernels when a.nlevels == 1, octree kernels otherwise.
hipError_t launch_mc(const McArgs &a, int blocks, int threads, hipStream_t s);
// Several frequencies of one grid in one launch: K argument blocks in
// device memory (each with its own package-id counter in next_id; tallies,
// private copies, statistics and schedule taken from args[0]).
struct MultiArgs {
    const McArgs *args;
    int32_t K;
    int32_t spread;   // 1: wave w starts at frequency w mod K; 0: every wave starts at 0
};
hipError_t launch_mc_multi(const MultiArgs &m, int nlevels, bool ali, int blocks, int threads, hipStream_t s);
hipError_t launch_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s);
hipError_t launch_trace(const McArgs &a, const TraceArgs &t, int precision, hipStream_t s);
hipError_t launch_peel(const McArgs &a, const PeelArgs &p, int blocks, hipStream_t s);

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
// absorbed[c] += sum_x priv[x n + c] over the kPrivCopies private copies, which are left zero.
// Add the private copies into absorbed and clear them; brick: their first
// nroot entries are the root cells of an nx x ny x nz root grid (even
// dimensions) in brick order.
hipError_t launch_fold_copies(double *absorbed, double *priv, int64_t n, int32_t brick, int32_t nx, int32_t ny,
                              int64_t nroot, hipStream_t s);

// dust emission setup
hipError_t launch_dust_luminosity(const uint32_t *words, int64_t ncells, const int64_t *level_offset,
                                  int32_t nlevels, double root_cell_cm, double nu, double sigma_abs,
                                  double w_nu, const float *T, double *L, hipStream_t s);
size_t scan_f64_scratch_elems(int64_t n);
hipError_t launch_scan_f64(const double *in, double *out, int64_t n, double *scratch, hipStream_t s);
// Correction emission: L = L(T) - L_ref into dL, |dL| into a, and
// L_ref += beta dL (no write when beta == 0).
hipError_t launch_dust_correction(const uint32_t *words, int64_t ncells, const int64_t *level_offset,
                                  int32_t nlevels, double root_cell_cm, double nu, double sigma_abs,
                                  double w_nu, const float *T, double *L_ref, double beta, double *dL, double *a,
                                  hipStream_t s);
// |L| into a.
hipError_t launch_abs_f64(const double *L, double *a, int64_t n, hipStream_t s);
// Capped expected counts: x_c = min(N a_c / S, cap) in place, S = *S_in
// (copied to *S_out first by every workgroup's first thread).
hipError_t launch_dust_cap(double *a, int64_t n, const double *S_in, double *S_out, uint64_t n_dust, double cap,
                           hipStream_t s);
// Systematic selection over an inclusive cumulative sum: package j takes
// the first cell whose cumulative value exceeds (j + u) S / N (units of
// the selection weight), or, in package units, j + u (cell -1 past the
// total).
hipError_t launch_dust_select(const double *incl, int64_t ncells, uint64_t n_dust, double u_sys, int32_t package_units,
                              int32_t *cell_out, hipStream_t s);
// One frequency of the batched weighted-mode setup (mode 1, no cap).
struct DustJob {
    const float *T;              // temperatures [ncells]
    double nu, sigma_abs, w_nu;  // the band
    double *incl;                // [ncells]: the luminosity, then its inclusive cumulative sum
    double *sums;                // scan scratch, scan_f64_scratch_elems(ncells) elements
    int32_t *cell;               // [n_dust] cell of every package
    uint64_t n_dust;
    double u_sys;                // systematic-sampling offset
};
// Luminosity, inclusive cumulative sum and package cells of njobs
// frequencies in five launches (d_jobs: device array of njobs jobs,
// max_dust = the largest n_dust); each row equals what
// launch_dust_luminosity, launch_scan_f64 and launch_dust_select give.
hipError_t launch_dust_setup_rows(const uint32_t *words, int64_t ncells, const int64_t *level_offset, int32_t nlevels,
                                  double root_cell_cm, const DustJob *d_jobs, int32_t njobs, uint64_t max_dust,
                                  hipStream_t s);
// Diagonal ALI: the dust energy each cell emits in this call, added to E.
// Weighted modes: from the cell of every package (non-decreasing, -1 past
// a capped total), one writer per cell; uniform mode: per_leaf packages of
// L_c / per_leaf in every leaf.
hipError_t launch_dust_emitted_weighted(const int32_t *cell, uint64_t n_dust, const double *dL, const double *S,
                                        int32_t mode, double cap, double *E, hipStream_t s);
hipError_t launch_dust_emitted_uniform(const int64_t *leaves, int64_t nleaves, const double *L, uint64_t per_leaf,
                                       double *E, hipStream_t s);
// ref += beta (x - ref) over n doubles.
hipError_t launch_blend(const double *x, double *ref, int64_t n, double beta, hipStream_t s);

// grid validation / reverse links / leaf list
hipError_t launch_validate_grid(const uint32_t *words, int64_t ncells, const int64_t *level_offset,
                                int32_t nlevels, int64_t nroot, int32_t *parent, int32_t *octet_count,
                                int32_t *flags, hipStream_t s);
hipError_t launch_check_octets(const int32_t *octet_count, int64_t noct, int32_t *flags, hipStream_t s);
size_t scan_i64_scratch_elems(int64_t n);
hipError_t launch_leaf_list(const uint32_t *words, int64_t ncells, int64_t *scan_tmp, int64_t *scratch,
                            int64_t *leaves, hipStream_t s);

// temperature
hipError_t launch_temp_table(const double *nu, const double *w, const double *sabs, int32_t K, double lnTf,
                             double dlnT, int32_t nT, double *lnG, hipStream_t s);
struct TempArgs {
    const uint32_t *words;
    int64_t ncells;
    int64_t level_offset[kMaxLevels + 1];
    int32_t nlevels;
    double root_cell_cm;
    const double *lnG;
    int32_t nT;
    double lnTf, dlnT, T_floor, T_max;
    const double *absorbed;
    const double *ali_self;      // diagonal ALI (NULL = off): self-absorbed and emitted dust energy
    const double *ali_emit;
    const float *T_old;
    float *T_new;
    int32_t given;               // 1: T_new holds a given field; statistics only, nothing written
    int32_t blocks;              // workgroups of the update and refine passes
    // statistics (part == NULL: not requested)
    double *part;                // blocks x 8 partial sums
    unsigned int *hist_part;     // blocks x kHistBins coarse ln T histograms
    unsigned int *hist_total;    // kHistBins
    double *meta;                // 8 values, see temp_stats_reduce_kernel
    unsigned int *fine_n;        // kHistBins fine bins inside the threshold bin
    double *fine_T;
};
// Learned starting temperatures (surrogate.hip): regular cubic grids of n^3
// cells, S^3 block averages of b^3 cells each (n = b S).
struct SurFeatArgs {
    const uint32_t *words;
    const float *T1;
    int32_t n, S, b, n_ps;
    double cell_cm, sigma_v, T_floor;
    const double *lnG;           // temperature table: ln Gamma on nT log-spaced T from lnTf, step dlnT
    int32_t nT;
    double lnTf, dlnT;
    double F_ext, Jbg;           // external field: 4 pi sum w I and sum w sigma I
    double px[kMaxPs], py[kMaxPs], pz[kMaxPs];   // point sources in coarse-cell units
    double Lbol[kMaxPs], Lw[kMaxPs];             // sum w L and sum w sigma L
    float *out;                  // [S^3][4]
};
struct SurMapArgs {
    const uint32_t *words;
    int32_t n, S, b;
    int32_t stride, channel;     // coarse arrays: block i at [i * stride + channel]
    int32_t absorbed;            // 0: temperatures (FP32), 1: absorbed energies (FP64)
    double T_floor, T_max, scale, offset;
    const float *T1, *T;         // temperatures of the constant sources and of the field
    const double *A1, *A;        // absorbed energies: the same
    float *coarse;               // target: output
    const float *pred;           // apply: network output
    float *T_out;                // apply: start temperatures
    double *A_out;               // apply: absorbed energies
};
hipError_t launch_sur_features(const SurFeatArgs &a, hipStream_t s);
hipError_t launch_sur_target(const SurMapArgs &a, hipStream_t s);
hipError_t launch_sur_apply(const SurMapArgs &a, hipStream_t s);

constexpr int kHistBins = 4096;
constexpr int kTempBlocks = 512;
hipError_t launch_temp_update(const TempArgs &a, hipStream_t s);
// Hottest-5% statistics after launch_temp_update (fine_n / fine_T zeroed).
hipError_t launch_temp_stats(const TempArgs &a, double *out4, hipStream_t s);

// ---- batched launch: many (model, frequency) pairs in one persistent launch
// One (model, frequency) pair: the grid, its absorbed array and the
// background / point sources of that frequency, as McArgs would hold them.
struct PairDev {
    const uint32_t *words;
    double *absorbed;
    const PsArg *ps;          // n_ps entries, device
    int32_t nx, ny, nz, n_ps;
    int64_t ncells;
    double *tally;            // tiles' deposits: the batch's brick-ordered scratch of this array, or absorbed
    int32_t brick, pad0;      // 1: tally is in 2 x 2 x 2 brick order (even dimensions)
    float ks_f, ka_f, g_f, pad;
    double W_bg, face_tot;
    double face_cum[6];
    uint64_t n_bg, n_ps_pk, n_total;
    uint32_t key0, key1, freq_index, pad2;
};

struct TileDev {
    int32_t pair;
    uint32_t begin, end;      // package ids [begin, end) of the pair
    int32_t pad;
};

struct BatchArgs {
    const PairDev *pairs;
    const TileDev *tiles;
    int32_t n_tiles;
    unsigned int *next_tile;
    const int32_t *lds_pairs;    // pairs a workgroup takes whole, tallied in LDS (small grids)
    int32_t n_lds_pairs;
    unsigned int *next_lds;
    const uint32_t *iteration;   // device word, read at launch
    int64_t step_cap;
    DevStats *st_call, *st_total;
    int32_t refill_min, inner_steps, scatter_min, chunk;
};

// The lean per-pair view the emission and step code read in the batched
// kernel (regular grids, background and point sources).
struct BatchView {
    const uint32_t *words;
    const int32_t *parent;
    int32_t nx, ny, nz, nlevels;
    int64_t ncells, nroot;
    const int64_t *level_offset;
    uint64_t n_bg, n_ps_pk, n_dust, n_total;
    int32_t n_ps, dust_mode;
    double W_bg;
    double face_cum[6];
    double face_tot;
    const PsArg *ps;
    const double *dust_L, *dust_S;
    double dust_cap;
    const int32_t *dust_cell;
    const int64_t *leaves;
    uint64_t per_leaf;
    uint32_t key0, key1, freq_index, iteration;
    int64_t step_cap;
};

// lds_cells: the largest grid of a.lds_pairs (the LDS tally's size)
hipError_t launch_mc_batch(const BatchArgs &a, int blocks, int threads, int64_t lds_cells, hipStream_t s);
// A brick-ordered tally of the batch and the array it is added to.
struct BrickFold {
    double *tally;
    double *absorbed;
    int32_t nx, ny;
    int64_t ncells;
};
// Add every brick-ordered tally into its array in cell order and clear it.
hipError_t launch_batch_fold(const BrickFold *folds, int32_t n, int64_t max_cells, hipStream_t s);
hipError_t launch_advance_iteration(uint32_t *it, int32_t mode, uint32_t value, hipStream_t s);

// micro-benchmarks: which 0 = random FP64 atomics (mode 0 shared, 1 per
// XCD slice; buf holds n doubles, or 8 n in mode 1), 1 = dependent random
// 4-byte gathers over n words (buf2: 1-word sink), 2 = copy of n bytes
// from buf to buf2.
hipError_t launch_ubench(int32_t which, void *buf, void *buf2, uint64_t n, int32_t per_thread, int32_t mode,
                         int blocks, int threads, hipStream_t s);

// map
struct MapArgs {
    const uint32_t *words;
    int32_t nx, ny, nz, nlevels;
    double root_cell_cm;
    int32_t axis, neg, npx, npy;
    double nu, sigma_abs, sigma_ext;
    const float *T;
    float *image;
};
hipError_t launch_map(const MapArgs &a, hipStream_t s);

}  // namespace soc
