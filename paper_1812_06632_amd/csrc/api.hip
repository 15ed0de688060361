// api.hip -- host implementation of the C ABI declared in include/soc.h.
//
// Each call validates its arguments before any launch, converts the
// physical inputs of one frequency into the per-launch argument block
// (McArgs) and enqueues the kernels on the context's stream.  The library
// owns only private scratch (statistics, the refill counter, dust-emission
// tables, trace buffers), grown on demand and freed with the context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <map>
#include <vector>

#include "soc.h"
#include "soc_device.h"
#include "soc_kernels.h"
#include "unet.h"

using namespace soc;

struct soc_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int num_cus = 256;
    int64_t step_cap = 10000000;
    // default schedule: 12 waves per compute unit, each refilled once 16 of
    // its lanes are idle.  12 waves is what the Monte Carlo kernels' 152-163
    // VGPRs allow per CU (3 per SIMD) and about what their deposit rings
    // allow in LDS (157 KB of 160).  The regular-grid benchmark iteration
    // takes the same time at 8, 10 or 12 waves (it waits on the memory-side
    // atomics); the octree pass, bound by the latency of its dependent
    // gathers, is 23% faster at 12 than at 8.
    int64_t block = 128;
    int64_t blocks_per_cu = 6;
    int64_t refill_min = 16;
    int64_t inner_steps = 1;
    int64_t timing = 0;
    int64_t chunk = 256;
    int64_t scatter_min = 1;
    int64_t xcd_copies = 1;
    int64_t multi_spread = 1;
    int64_t batch_lds_cells = 0;      // grids of at most this many cells: whole pairs tallied in LDS (set at creation)
    int64_t max_lds_cells = 0;        // the most the device's LDS per workgroup holds
    int64_t lds_per_cu = 65536;       // bytes of LDS per compute unit
    // scratch
    DevStats *d_stats = nullptr;              // [0] per call, [1] running total
    unsigned long long *d_counter = nullptr;
    double *d_tmp_out = nullptr;              // small result buffer (temperature stats)
    double *d_priv = nullptr;                 // kPrivCopies private copies of the absorbed array (zero between launches)
    int64_t cap_priv = 0;
    double *d_priv_self = nullptr;            // the same for the ALI self-absorption tally
    int64_t cap_priv_self = 0;
    double *d_peel = nullptr;                 // totals of a scattered-light run
    int64_t cap_peel = 0;
    double *d_L = nullptr, *d_incl = nullptr, *d_scan = nullptr;
    int64_t cap_L = 0, cap_incl = 0, cap_scan = 0;
    double *d_a = nullptr, *d_S = nullptr;   // selection weights / capped counts; sum of |L| (capped mode)
    int64_t cap_a = 0, cap_S = 0;
    int32_t *d_pkcell = nullptr;
    uint64_t cap_pk = 0;
    double *d_tpart = nullptr;           // temperature statistics scratch
    unsigned int *d_thist = nullptr;
    double *d_tmeta = nullptr;
    unsigned int *d_tfine_n = nullptr;
    double *d_tfine_T = nullptr;
    // soc_simulate_frequencies: per-frequency tables and argument blocks
    double *d_mL = nullptr, *d_mS = nullptr;
    int64_t cap_mL = 0, cap_mS = 0;
    int32_t *d_mpk = nullptr;
    int64_t cap_mpk = 0;
    McArgs *d_margs = nullptr;
    int64_t cap_margs = 0;
    unsigned long long *d_mcount = nullptr;
    int64_t cap_mcount = 0;
    std::vector<McArgs> h_margs;   // staging of the argument blocks (kept until the next call)
    // batched weighted-mode dust setup: one luminosity/cumulative row and
    // one scan scratch row per frequency, the jobs and their staging
    double *d_mincl = nullptr, *d_msums = nullptr;
    int64_t cap_mincl = 0, cap_msums = 0;
    DustJob *d_djobs = nullptr;
    int64_t cap_djobs = 0;
    std::vector<DustJob> h_djobs;
    std::vector<hipEvent_t> ev_start, ev_stop;
    bool capturing = false;
};

struct soc_batch_s {
    soc_ctx ctx = nullptr;
    int device = 0;
    int32_t n_tiles = 0;
    uint64_t n_packages = 0;
    PairDev *d_pairs = nullptr;
    TileDev *d_tiles = nullptr;
    PsArg *d_ps = nullptr;
    unsigned int *d_counter = nullptr;      // [0] next tile, [1] next LDS pair
    uint32_t *d_iteration = nullptr;
    int32_t *d_lds_pairs = nullptr;         // pairs of small grids, largest cost first
    int32_t n_lds_pairs = 0;
    int64_t lds_cells = 0;                  // the largest grid among them
    double *d_brick = nullptr;              // brick-ordered tallies of the tiled arrays (zero between runs)
    BrickFold *d_folds = nullptr;           // each tally and its array
    int32_t n_folds = 0;
    int64_t max_fold_cells = 0;
};

struct soc_graph_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct soc_grid_s {
    soc_ctx ctx = nullptr;   // identity check only; never dereferenced after creation
    int device = 0;
    int32_t nx = 0, ny = 0, nz = 0, nlevels = 0;
    int64_t ncells = 0, nroot = 0, nleaves = 0;
    std::vector<int64_t> level_offset;
    double root_cell_cm = 0.0;
    const uint32_t *d_words = nullptr;
    int32_t *d_parent = nullptr;
    int64_t *d_leaves = nullptr;
};

struct soc_temp_table_s {
    soc_ctx ctx = nullptr;   // identity check only; never dereferenced after creation
    int device = 0;
    int32_t nT = 0;
    double T_floor = 0.0, T_max = 0.0, lnTf = 0.0, dlnT = 0.0;
    double *d_lnG = nullptr;
};

struct soc_shg_model_s {
    soc_ctx ctx = nullptr;   // identity check only
    int device = 0;
    int32_t S = 0, K = 0, N = 0;
    double *d_buf = nullptr;   // every table in one allocation
    soc::ShgModelDev dev{};
};

namespace {

soc_status fail(soc_ctx c, soc_status s, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIPCHK(ctx, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail((ctx), SOC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
soc_status grow(soc_ctx c, T **p, int64_t &cap, int64_t need)
{
    if (need <= cap && *p) return SOC_OK;
    if (c->capturing) return fail(c, SOC_ESTATE, "scratch would grow during graph capture; run the call once before capturing");
    if (*p) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, SOC_EHIP, "sync before regrow: %s", hipGetErrorString(e));
        (void)hipFree(*p);
        *p = nullptr;
        cap = 0;
    }
    if (hipMalloc((void **)p, sizeof(T) * (size_t)(need > 0 ? need : 1)) != hipSuccess) {
        *p = nullptr;
        return fail(c, SOC_ENOMEM, "device allocation of %lld elements failed", (long long)need);
    }
    cap = need;
    return SOC_OK;
}

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

#define NOT_WHILE_CAPTURING(c)                                                                    \
    do {                                                                                          \
        if ((c)->capturing) return fail((c), SOC_ESTATE, "call not allowed during graph capture"); \
    } while (0)

soc_status check_freq(soc_ctx c, const soc_freq *f)
{
    if (!f) return fail(c, SOC_EINVAL, "freq is NULL");
    if (!(std::isfinite(f->nu) && f->nu > 0.0)) return fail(c, SOC_EINVAL, "nu must be finite and > 0");
    if (!finite_nonneg(f->w_nu)) return fail(c, SOC_EINVAL, "w_nu must be finite and >= 0");
    if (!finite_nonneg(f->sigma_abs) || !finite_nonneg(f->sigma_sca))
        return fail(c, SOC_EINVAL, "cross sections must be finite and >= 0");
    if (!(std::fabs(f->g) < 1.0)) return fail(c, SOC_EINVAL, "|g| must be < 1");
    return SOC_OK;
}

// Where the scratch of one call lives: the context's buffers, grown on
// demand (base == NULL), or fixed slices of the per-device no-allocation
// array at base (sizes checked against its limits).
struct ScratchSrc {
    char *base = nullptr;
    // set by soc_simulate_frequencies, where each frequency keeps its own
    // tables until the launch: the luminosities (when the kernel reads
    // them), the package-to-cell list and the total weight
    double *L = nullptr;
    int32_t *pk = nullptr;
    double *S = nullptr;
    // weighted mode without a cap: the luminosity row, its scan scratch and
    // the job that the caller's batched setup fills them from (the tables
    // are then not built here)
    DustJob *job = nullptr;
    double *incl = nullptr, *sums = nullptr;
};

// Largest total of the per-frequency luminosity rows that
// soc_simulate_frequencies builds together (16 GiB: 64 frequencies of a
// 256^3 grid take 8.6 GB).
constexpr int64_t kDustRowsMaxBytes = int64_t(16) << 30;

// Systematic-sampling offset of one frequency's weighted dust emission: the
// first uniform of the stream of package id 2^32-1 of the dust class.
double dust_offset(uint64_t seed, uint32_t iteration, uint32_t freq_index)
{
    uint32_t x0 = 0, x1 = 0xFFFFFFFFu, x2 = freq_index, x3 = (iteration << 8) | kClassDust;
    philox4x32_10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    return u01<double>(x0);
}

// Fixed slices of the no-allocation array (byte offsets, 256-aligned).
constexpr int64_t kNaMaxCells = 32768;           // 32^3 cells, every level included
constexpr int64_t kNaMaxDust = int64_t(1) << 20; // weighted dust packages per call
constexpr size_t na_round(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kNaStats = 0;                                              // 2 DevStats
constexpr size_t kNaCounter = kNaStats + na_round(2 * sizeof(DevStats));    // refill counter
constexpr size_t kNaS = kNaCounter + 256;                                   // capped dust total
constexpr size_t kNaL = kNaS + 256;
constexpr size_t kNaA = kNaL + na_round(sizeof(double) * kNaMaxCells);
constexpr size_t kNaIncl = kNaA + na_round(sizeof(double) * kNaMaxCells);
constexpr size_t kNaScan = kNaIncl + na_round(sizeof(double) * kNaMaxCells);
constexpr size_t kNaScanElems = 1024;   // >= scan_f64_scratch_elems(kNaMaxCells), checked at run time
constexpr size_t kNaPk = kNaScan + na_round(sizeof(double) * kNaScanElems);
constexpr size_t kNaPriv = kNaPk + na_round(sizeof(int32_t) * kNaMaxDust);
constexpr size_t kNaPrivSelf = kNaPriv + na_round(sizeof(double) * kPrivCopies * kNaMaxCells);
constexpr size_t kNaBytes = kNaPrivSelf + na_round(sizeof(double) * kPrivCopies * kNaMaxCells);

// A scratch buffer of `need` elements: the context's (grown) or the slice
// at byte offset `off` of the no-allocation array.
template <typename T>
soc_status take(soc_ctx c, const ScratchSrc &src, T **ctx_p, int64_t &ctx_cap, int64_t need, size_t off,
                int64_t max_need, T **out)
{
    if (!src.base) {
        soc_status st = grow(c, ctx_p, ctx_cap, need);
        *out = *ctx_p;
        return st;
    }
    if (need > max_need)
        return fail(c, SOC_EINVAL, "no-allocation call: %lld elements exceed its fixed scratch of %lld",
                    (long long)need, (long long)max_need);
    *out = (T *)(src.base + off);
    return SOC_OK;
}

// Per-frequency argument block shared by the production and trace kernels.
soc_status prepare(soc_ctx c, soc_grid g, const soc_freq *f, const soc_sources *s, uint64_t seed,
                   uint32_t iteration, uint32_t freq_index, double *d_absorbed, McArgs &A,
                   const ScratchSrc &src = ScratchSrc())
{
    soc_status st = check_freq(c, f);
    if (st) return st;
    if (!g) return fail(c, SOC_EINVAL, "grid is NULL");
    if (g->ctx != c) return fail(c, SOC_EINVAL, "grid belongs to another context");
    if (!s) return fail(c, SOC_EINVAL, "sources is NULL");
    if (!finite_nonneg(s->I_bg_nu)) return fail(c, SOC_EINVAL, "I_bg_nu must be finite and >= 0");
    if (s->n_ps < 0 || s->n_ps > kMaxPs) return fail(c, SOC_EINVAL, "n_ps must be in [0, %d]", kMaxPs);
    if (s->n_ps > 0 && !s->ps) return fail(c, SOC_EINVAL, "ps is NULL");
    if (s->d_T && (s->dust_mode < 0 || s->dust_mode > 2)) return fail(c, SOC_EINVAL, "dust_mode must be 0, 1 or 2");
    if (s->d_T && s->dust_mode == 2 && !s->d_L_ref) return fail(c, SOC_EINVAL, "dust_mode 2 needs d_L_ref");
    if (!(s->ref_beta >= 0.0 && s->ref_beta <= 1.0)) return fail(c, SOC_EINVAL, "ref_beta must be in [0, 1]");
    if (!finite_nonneg(s->dust_cap)) return fail(c, SOC_EINVAL, "dust_cap must be finite and >= 0");
    if ((s->d_ali_self == nullptr) != (s->d_ali_emitted == nullptr))
        return fail(c, SOC_EINVAL, "ALI needs both d_ali_self and d_ali_emitted");
    if (s->d_ali_self && s->d_T && s->dust_mode == 2)
        return fail(c, SOC_EINVAL, "ALI tallies apply to dust modes 0 and 1");
    if (s->d_T && s->dust_mode == 0 && s->dust_cap > 0.0)
        return fail(c, SOC_EINVAL, "dust_cap applies to the weighted modes (1, 2)");
    if (s->n_bg > 0xFFFFFFFFull || s->n_ps_pk > 0xFFFFFFFFull || s->n_dust > 0x7FFFFFFFull)
        return fail(c, SOC_EINVAL, "package counts exceed the 32-bit package id range");

    std::memset(&A, 0, sizeof A);
    A.words = g->d_words;
    A.parent = g->d_parent;
    A.nx = g->nx; A.ny = g->ny; A.nz = g->nz; A.nlevels = g->nlevels;
    A.ncells = g->ncells;
    A.nroot = g->nroot;
    for (int i = 0; i <= kMaxLevels; ++i)
        A.level_offset[i] = i <= g->nlevels ? g->level_offset[i] : g->ncells;
    const double s_cm = g->root_cell_cm;
    A.ks_d = f->sigma_sca * s_cm;
    A.ka_d = f->sigma_abs * s_cm;
    A.g_d = f->g;
    A.ks_f = (float)A.ks_d;
    A.ka_f = (float)A.ka_d;
    A.g_f = (float)f->g;

    // background: pi I w A_box through the faces, face chosen by area
    const double N0 = g->nx, N1 = g->ny, N2 = g->nz;
    const double area[6] = {N1 * N2, N1 * N2, N0 * N2, N0 * N2, N0 * N1, N0 * N1};
    double tot = 0.0;
    for (int k = 0; k < 6; ++k) tot += area[k];
    double cum = 0.0;
    for (int k = 0; k < 6; ++k) {
        cum += area[k];
        A.face_cum[k] = cum;
    }
    A.face_tot = tot;
    const double E_bg = M_PI * s->I_bg_nu * f->w_nu * tot * (s_cm * s_cm);
    A.n_bg = s->n_bg;
    A.W_bg = s->n_bg ? E_bg / (double)s->n_bg : 0.0;

    A.n_ps = s->n_ps;
    A.n_ps_pk = s->n_ps > 0 ? s->n_ps_pk : 0;
    for (int i = 0; i < s->n_ps; ++i) {
        const soc_point_source &q = s->ps[i];
        if (!(q.x >= 0.0 && q.x < N0 && q.y >= 0.0 && q.y < N1 && q.z >= 0.0 && q.z < N2))
            return fail(c, SOC_EINVAL, "point source %d lies outside the box", i);
        if (!finite_nonneg(q.L_nu)) return fail(c, SOC_EINVAL, "point source %d: L_nu must be finite and >= 0", i);
        A.ps[i].x = q.x; A.ps[i].y = q.y; A.ps[i].z = q.z;
        A.ps[i].W = A.n_ps_pk ? q.L_nu * f->w_nu / (double)A.n_ps_pk : 0.0;
    }

    // dust emission: per-cell luminosity (or its difference to the
    // reference), inclusive cumulative sum of the selection weights and,
    // for the weighted modes, the cell of every package
    A.n_dust = 0;
    A.dust_mode = s->dust_mode;
    const bool deferred = src.job && s->d_T && s->n_dust > 0 && s->dust_mode == 1 && !(s->dust_cap > 0.0);
    if (deferred) {
        A.n_dust = s->n_dust;
        DustJob &J = *src.job;
        J.T = s->d_T;
        J.nu = f->nu;
        J.sigma_abs = f->sigma_abs;
        J.w_nu = f->w_nu;
        J.incl = src.incl;
        J.sums = src.sums;
        J.cell = src.pk;
        J.n_dust = s->n_dust;
        J.u_sys = dust_offset(seed, iteration, freq_index);
        A.dust_L = src.incl;   // not read in this mode
        A.dust_S = src.incl + (g->ncells - 1);
        A.dust_cell = src.pk;
    } else if (s->d_T && s->n_dust > 0) {
        A.n_dust = s->n_dust;
        double *dL = src.L, *da = nullptr;
        if (!dL && (st = take(c, src, &c->d_L, c->cap_L, g->ncells, kNaL, kNaMaxCells, &dL))) return st;
        if (s->dust_mode == 2) {
            if ((st = take(c, src, &c->d_a, c->cap_a, g->ncells, kNaA, kNaMaxCells, &da))) return st;
            HIPCHK(c, launch_dust_correction(g->d_words, g->ncells, g->level_offset.data(), g->nlevels, s_cm, f->nu,
                                             f->sigma_abs, f->w_nu, s->d_T, s->d_L_ref, s->ref_beta, dL, da,
                                             c->stream));
        } else {
            HIPCHK(c, launch_dust_luminosity(g->d_words, g->ncells, g->level_offset.data(), g->nlevels, s_cm, f->nu,
                                             f->sigma_abs, f->w_nu, s->d_T, dL, c->stream));
        }
        A.dust_L = dL;
        if (s->dust_mode == 0) {
            if (s->n_dust % (uint64_t)g->nleaves != 0)
                return fail(c, SOC_EINVAL, "uniform dust mode needs n_dust to be a multiple of the %lld leaves",
                            (long long)g->nleaves);
            A.per_leaf = s->n_dust / (uint64_t)g->nleaves;
            A.leaves = g->d_leaves;
        } else {
            const bool capped = s->dust_cap > 0.0;
            if (capped && s->dust_mode == 1) {
                if ((st = take(c, src, &c->d_a, c->cap_a, g->ncells, kNaA, kNaMaxCells, &da))) return st;
                HIPCHK(c, launch_abs_f64(dL, da, g->ncells, c->stream));
            }
            const double *weight = s->dust_mode == 2 || capped ? da : dL;
            double *dincl = nullptr, *dscan = nullptr;
            if ((st = take(c, src, &c->d_incl, c->cap_incl, g->ncells, kNaIncl, kNaMaxCells, &dincl))) return st;
            if ((st = take(c, src, &c->d_scan, c->cap_scan, (int64_t)scan_f64_scratch_elems(g->ncells), kNaScan,
                           (int64_t)kNaScanElems, &dscan)))
                return st;
            HIPCHK(c, launch_scan_f64(weight, dincl, g->ncells, dscan, c->stream));
            A.dust_S = dincl + (g->ncells - 1);
            if (src.S && !capped) {   // the scan array is reused by the next frequency
                HIPCHK(c, launch_copy_f64(dincl + (g->ncells - 1), src.S, 1, c->stream));
                A.dust_S = src.S;
            }
            if (capped) {
                // expected counts min(N a / S, cap) replace the weights; their
                // cumulative sum (package units) replaces the first one
                double *dS = src.S;
                if (!dS && (st = take(c, src, &c->d_S, c->cap_S, 1, kNaS, 1, &dS))) return st;
                HIPCHK(c, launch_dust_cap(da, g->ncells, dincl + (g->ncells - 1), dS, s->n_dust,
                                          s->dust_cap, c->stream));
                HIPCHK(c, launch_scan_f64(da, dincl, g->ncells, dscan, c->stream));
                A.dust_S = dS;
                A.dust_cap = s->dust_cap;
            }
            int64_t cap_pk = (int64_t)c->cap_pk;
            int32_t *dpk = src.pk;
            if (!dpk && (st = take(c, src, &c->d_pkcell, cap_pk, (int64_t)s->n_dust, kNaPk, kNaMaxDust, &dpk)))
                return st;
            c->cap_pk = (uint64_t)cap_pk;
            const double u_sys = dust_offset(seed, iteration, freq_index);
            HIPCHK(c, launch_dust_select(dincl, g->ncells, s->n_dust, u_sys, capped ? 1 : 0, dpk, c->stream));
            A.dust_cell = dpk;
        }
    }
    A.n_total = A.n_bg + (uint64_t)A.n_ps * A.n_ps_pk + A.n_dust;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.freq_index = freq_index;
    A.iteration = iteration;
    A.step_cap = c->step_cap;
    A.absorbed = d_absorbed;
    A.ali_self = s->d_ali_self;
    if (s->d_ali_emitted && A.n_dust > 0 && !deferred) {
        // emitted dust energy per cell from the package assignment (no atomics)
        // (a deferred frequency's comes after the caller's batched setup)
        if (A.dust_mode == 0)
            HIPCHK(c, launch_dust_emitted_uniform(g->d_leaves, g->nleaves, A.dust_L, A.per_leaf, s->d_ali_emitted,
                                                  c->stream));
        else
            HIPCHK(c, launch_dust_emitted_weighted(A.dust_cell, A.n_dust, A.dust_L, A.dust_S, A.dust_mode, A.dust_cap,
                                                   s->d_ali_emitted, c->stream));
    }
    A.next_id = src.base ? (unsigned long long *)(src.base + kNaCounter) : c->d_counter;
    A.st_call = src.base ? (DevStats *)(src.base + kNaStats) : c->d_stats;
    A.st_total = c->d_stats + 1;
    A.refill_min = (int32_t)c->refill_min;
    A.inner_steps = (int32_t)c->inner_steps;
    A.chunk = (int32_t)c->chunk;
    A.scatter_min = (int32_t)c->scatter_min;
    return SOC_OK;
}

void to_public(const DevStats &d, soc_sim_stats *o)
{
    o->packages = d.packages;
    o->cell_steps = d.steps;
    o->scatterings = d.scatterings;
    o->runaways = d.runaways;
    o->e_emitted = d.emitted;
    o->e_absorbed = d.absorbed;
    o->e_escaped = d.escaped;
}

}  // namespace

// Scratch of soc_simulate_frequency_noalloc, one instance per device for the
// life of the process.  Host code never passes this name to a kernel: it
// resolves the device's own address once (soc_ctx_create, the device
// current) and uses that.
static __device__ __align__(256) char scratch[kNaBytes];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
char *g_na_base[kNaMaxDevices] = {};

// Address of the no-allocation array on the current device `dev`,
// resolved on the first call for that device.
hipError_t na_resolve(int dev)
{
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (g_na_base[dev]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_na_base[dev] = (char *)ptr;
    return hipSuccess;
}

char *na_base(int dev)
{
    if (dev < 0 || dev >= kNaMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_na_mu);
    return g_na_base[dev];
}

}  // namespace

extern "C" {

soc_status soc_ctx_create(int32_t hip_device, void *hip_stream, soc_ctx *out)
{
    if (!out) return SOC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SOC_EHIP;
    if (hip_device < 0 || hip_device >= ndev) return SOC_EINVAL;
    soc_ctx c = new (std::nothrow) soc_ctx_s;
    if (!c) return SOC_ENOMEM;
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(hip_device) != hipSuccess) { delete c; return SOC_EHIP; }
    if (na_resolve(hip_device) != hipSuccess) { delete c; return SOC_EHIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) != hipSuccess)
        lds_max = 65536;
    // room for the kernel's own static LDS words; at most 24^3 cells by default
    c->max_lds_cells = std::max<int64_t>(0, ((int64_t)lds_max - 256) / (int64_t)sizeof(double));
    int lds_cu = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, hip_device) == hipSuccess &&
        lds_cu > 0)
        c->lds_per_cu = lds_cu;
    c->batch_lds_cells = std::min<int64_t>(c->max_lds_cells, 13824);
    if (hipMalloc((void **)&c->d_stats, 2 * sizeof(DevStats)) != hipSuccess ||
        hipMalloc((void **)&c->d_counter, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void **)&c->d_tmp_out, 8 * sizeof(double)) != hipSuccess) {
        soc_ctx_destroy(c);
        return SOC_ENOMEM;
    }
    if (launch_fill_u64((unsigned long long *)c->d_stats, 0ull, 2 * (int64_t)(sizeof(DevStats) / 8), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        soc_ctx_destroy(c);
        return SOC_EHIP;
    }
    *out = c;
    return SOC_OK;
}

void soc_ctx_destroy(soc_ctx c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto e : c->ev_start) (void)hipEventDestroy(e);
    for (auto e : c->ev_stop) (void)hipEventDestroy(e);
    (void)hipFree(c->d_stats);
    (void)hipFree(c->d_counter);
    (void)hipFree(c->d_tmp_out);
    (void)hipFree(c->d_priv);
    (void)hipFree(c->d_priv_self);
    (void)hipFree(c->d_peel);
    (void)hipFree(c->d_L);
    (void)hipFree(c->d_incl);
    (void)hipFree(c->d_a);
    (void)hipFree(c->d_S);
    (void)hipFree(c->d_scan);
    (void)hipFree(c->d_pkcell);
    (void)hipFree(c->d_tpart);
    (void)hipFree(c->d_thist);
    (void)hipFree(c->d_tmeta);
    (void)hipFree(c->d_tfine_n);
    (void)hipFree(c->d_tfine_T);
    (void)hipFree(c->d_mL);
    (void)hipFree(c->d_mS);
    (void)hipFree(c->d_mpk);
    (void)hipFree(c->d_margs);
    (void)hipFree(c->d_mcount);
    (void)hipFree(c->d_mincl);
    (void)hipFree(c->d_msums);
    (void)hipFree(c->d_djobs);
    delete c;
}

soc_status soc_ctx_set_stream(soc_ctx c, void *hip_stream)
{
    if (!c) return SOC_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return SOC_OK;
}

const char *soc_last_error(soc_ctx c) { return c ? c->err.c_str() : "NULL context"; }

soc_status soc_ctx_set_option(soc_ctx c, soc_option opt, int64_t v)
{
    if (!c) return SOC_EINVAL;
    switch (opt) {
    case SOC_OPT_STEP_CAP:
        if (v < 1) return fail(c, SOC_EINVAL, "step cap must be >= 1");
        c->step_cap = v;
        return SOC_OK;
    case SOC_OPT_BLOCK:
        if (v < 64 || v > kMcMaxBlock || v % 64)
            return fail(c, SOC_EINVAL, "block must be a multiple of 64 in [64,%d]", kMcMaxBlock);
        c->block = v;
        return SOC_OK;
    case SOC_OPT_BLOCKS_PER_CU:
        if (v < 1 || v > 64) return fail(c, SOC_EINVAL, "blocks per CU must be in [1,64]");
        c->blocks_per_cu = v;
        return SOC_OK;
    case SOC_OPT_REFILL_MIN:
        if (v < 1 || v > 64) return fail(c, SOC_EINVAL, "refill threshold must be in [1,64]");
        c->refill_min = v;
        return SOC_OK;
    case SOC_OPT_INNER_STEPS:
        if (v < 1 || v > kDepSlots) return fail(c, SOC_EINVAL, "inner steps must be in [1,%d]", kDepSlots);
        c->inner_steps = v;
        return SOC_OK;
    case SOC_OPT_TIMING:
        c->timing = v ? 1 : 0;
        return SOC_OK;
    case SOC_OPT_SCATTER_MIN:
        if (v < 1 || v > 64) return fail(c, SOC_EINVAL, "scatter threshold must be in [1,64]");
        c->scatter_min = v;
        return SOC_OK;
    case SOC_OPT_XCD_COPIES:
        c->xcd_copies = v ? 1 : 0;
        return SOC_OK;
    case SOC_OPT_CHUNK:   // >= 64: one grant must cover every idle lane of a wave
        if (v < 64 || v > 65536) return fail(c, SOC_EINVAL, "chunk must be in [64,65536]");
        c->chunk = v;
        return SOC_OK;
    case SOC_OPT_MULTI_SPREAD:
        c->multi_spread = v ? 1 : 0;
        return SOC_OK;
    case SOC_OPT_BATCH_LDS_CELLS:
        if (v < 0 || v > c->max_lds_cells)
            return fail(c, SOC_EINVAL, "batch LDS cells must be in [0,%lld] on this device", (long long)c->max_lds_cells);
        c->batch_lds_cells = v;
        return SOC_OK;
    }
    return fail(c, SOC_EINVAL, "unknown option %d", (int)opt);
}

soc_status soc_ctx_get_option(soc_ctx c, soc_option opt, int64_t *v)
{
    if (!c || !v) return SOC_EINVAL;
    switch (opt) {
    case SOC_OPT_STEP_CAP: *v = c->step_cap; return SOC_OK;
    case SOC_OPT_BLOCK: *v = c->block; return SOC_OK;
    case SOC_OPT_BLOCKS_PER_CU: *v = c->blocks_per_cu; return SOC_OK;
    case SOC_OPT_REFILL_MIN: *v = c->refill_min; return SOC_OK;
    case SOC_OPT_INNER_STEPS: *v = c->inner_steps; return SOC_OK;
    case SOC_OPT_TIMING: *v = c->timing; return SOC_OK;
    case SOC_OPT_SCATTER_MIN: *v = c->scatter_min; return SOC_OK;
    case SOC_OPT_XCD_COPIES: *v = c->xcd_copies; return SOC_OK;
    case SOC_OPT_CHUNK: *v = c->chunk; return SOC_OK;
    case SOC_OPT_BATCH_LDS_CELLS: *v = c->batch_lds_cells; return SOC_OK;
    case SOC_OPT_MULTI_SPREAD: *v = c->multi_spread; return SOC_OK;
    }
    return fail(c, SOC_EINVAL, "unknown option %d", (int)opt);
}

soc_status soc_ctx_mc_timing(soc_ctx c, double *total_ms, int64_t *launches, int32_t reset)
{
    if (!c) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (size_t i = 0; i < c->ev_start.size(); ++i) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)c->ev_start.size();
    if (reset) {
        for (auto e : c->ev_start) (void)hipEventDestroy(e);
        for (auto e : c->ev_stop) (void)hipEventDestroy(e);
        c->ev_start.clear();
        c->ev_stop.clear();
    }
    return SOC_OK;
}

soc_status soc_build_grid(soc_ctx c, const soc_grid_desc *d, soc_grid *out)
{
    if (!c) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    if (!d || !out) return fail(c, SOC_EINVAL, "desc/out is NULL");
    *out = nullptr;
    if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0) return fail(c, SOC_EINVAL, "grid dimensions must be > 0");
    if (d->nlevels < 1 || d->nlevels > kMaxLevels) return fail(c, SOC_EINVAL, "nlevels must be in [1,%d]", kMaxLevels);
    if (!d->level_offset || !d->d_words) return fail(c, SOC_EINVAL, "level_offset/d_words is NULL");
    if (!(std::isfinite(d->root_cell_cm) && d->root_cell_cm > 0.0)) return fail(c, SOC_EINVAL, "root_cell_cm must be > 0");
    const int64_t nroot = (int64_t)d->nx * d->ny * d->nz;
    if (d->ncells > 0x7FFFFFFFll) return fail(c, SOC_EINVAL, "more than 2^31-1 cells");
    if (d->level_offset[0] != 0 || d->level_offset[1] != nroot || d->level_offset[d->nlevels] != d->ncells)
        return fail(c, SOC_EGRID, "level offsets inconsistent with the root grid and ncells");
    for (int L = 1; L <= d->nlevels; ++L) {
        if (d->level_offset[L] < d->level_offset[L - 1]) return fail(c, SOC_EGRID, "level offsets decrease");
        if (L >= 2 && (d->level_offset[L] - d->level_offset[L - 1]) % 8)
            return fail(c, SOC_EGRID, "level %d is not a whole number of octets", L);
    }
    HIPCHK(c, hipSetDevice(c->device));
    soc_grid g = new (std::nothrow) soc_grid_s;
    if (!g) return fail(c, SOC_ENOMEM, "host allocation failed");
    g->ctx = c;
    g->device = c->device;
    g->nx = d->nx; g->ny = d->ny; g->nz = d->nz; g->nlevels = d->nlevels;
    g->ncells = d->ncells;
    g->nroot = nroot;
    g->level_offset.assign(d->level_offset, d->level_offset + d->nlevels + 1);
    g->root_cell_cm = d->root_cell_cm;
    g->d_words = d->d_words;
    const int64_t noct = (d->ncells - nroot) / 8;
    int32_t *d_count = nullptr, *d_flags = nullptr;
    int64_t *d_tmp = nullptr, *d_scr = nullptr;
    auto cleanup = [&](soc_status s) {
        (void)hipFree(d_count); (void)hipFree(d_flags); (void)hipFree(d_tmp); (void)hipFree(d_scr);
        if (s != SOC_OK) soc_grid_destroy(g);
        return s;
    };
    if (hipMalloc((void **)&d_flags, sizeof(int32_t)) != hipSuccess) return cleanup(fail(c, SOC_ENOMEM, "alloc"));
    if (noct > 0) {
        if (hipMalloc((void **)&g->d_parent, sizeof(int32_t) * noct) != hipSuccess ||
            hipMalloc((void **)&d_count, sizeof(int32_t) * noct) != hipSuccess)
            return cleanup(fail(c, SOC_ENOMEM, "alloc of reverse links failed"));
        if (launch_fill_i32(d_count, 0, noct, c->stream) != hipSuccess ||
            launch_fill_i32(g->d_parent, -1, noct, c->stream) != hipSuccess)
            return cleanup(fail(c, SOC_EHIP, "fill failed"));
    }
    if (launch_fill_i32(d_flags, 0, 1, c->stream) != hipSuccess) return cleanup(fail(c, SOC_EHIP, "fill failed"));
    if (launch_validate_grid(d->d_words, d->ncells, d->level_offset, d->nlevels, nroot, g->d_parent, d_count, d_flags,
                             c->stream) != hipSuccess ||
        launch_check_octets(d_count, noct, d_flags, c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "grid validation launch failed: %s", hipGetErrorString(hipGetLastError())));
    int32_t flags = 0;
    if (hipMemcpyAsync(&flags, d_flags, sizeof flags, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "grid validation failed: %s", hipGetErrorString(hipGetLastError())));
    if (flags) {
        return cleanup(fail(c, SOC_EGRID, "malformed grid:%s%s%s", (flags & 1) ? " bad link" : "",
                            (flags & 2) ? " bad density" : "", (flags & 4) ? " octet not linked exactly once" : ""));
    }
    if (d->nlevels == 1) {
        g->nleaves = d->ncells;
    } else {
        const size_t ns = scan_i64_scratch_elems(d->ncells);
        if (hipMalloc((void **)&g->d_leaves, sizeof(int64_t) * d->ncells) != hipSuccess ||
            hipMalloc((void **)&d_tmp, sizeof(int64_t) * d->ncells) != hipSuccess ||
            hipMalloc((void **)&d_scr, sizeof(int64_t) * ns) != hipSuccess)
            return cleanup(fail(c, SOC_ENOMEM, "alloc of leaf list failed"));
        if (launch_leaf_list(d->d_words, d->ncells, d_tmp, d_scr, g->d_leaves, c->stream) != hipSuccess)
            return cleanup(fail(c, SOC_EHIP, "leaf list launch failed"));
        int64_t last_pos = 0;
        uint32_t last_word = 0;
        if (hipMemcpyAsync(&last_pos, d_tmp + d->ncells - 1, sizeof last_pos, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipMemcpyAsync(&last_word, d->d_words + d->ncells - 1, sizeof last_word, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return cleanup(fail(c, SOC_EHIP, "leaf count readback failed"));
        g->nleaves = last_pos + (((int32_t)last_word >= 0) ? 1 : 0);
    }
    *out = g;
    return cleanup(SOC_OK);
}

void soc_grid_destroy(soc_grid g)
{
    if (!g) return;
    // hipFree waits for work that uses the memory; the context may already
    // be gone, so only the device id recorded at creation is used
    (void)hipSetDevice(g->device);
    (void)hipFree(g->d_parent);
    (void)hipFree(g->d_leaves);
    delete g;
}

soc_status soc_grid_info(soc_grid g, int64_t *n_leaves, const int32_t **d_parent)
{
    if (!g) return SOC_EINVAL;
    if (n_leaves) *n_leaves = g->nleaves;
    if (d_parent) *d_parent = g->d_parent;
    return SOC_OK;
}

// The root cells of a grid with even root dimensions (every cell of such a
// regular grid) are kept in 2 x 2 x 2 bricks in the private copies, so that
// neighbouring cells share 64-byte lines.
static int32_t brick_copies(const soc_grid g)
{
    return g->nx % 2 == 0 && g->ny % 2 == 0 && g->nz % 2 == 0 ? 1 : 0;
}

soc_status soc_simulate_frequency(soc_ctx c, soc_grid g, const soc_freq *f, const soc_sources *s, uint64_t seed,
                                  uint32_t iteration, uint32_t freq_index, double *d_absorbed, soc_sim_stats *stats)
{
    if (!c) return SOC_EINVAL;
    if (!d_absorbed) return fail(c, SOC_EINVAL, "d_absorbed is NULL");
    HIPCHK(c, hipSetDevice(c->device));
    if (c->capturing && (stats || c->timing)) return fail(c, SOC_ESTATE, "statistics/timing not allowed during graph capture");
    McArgs A;
    soc_status st = prepare(c, g, f, s, seed, iteration, freq_index, d_absorbed, A);
    if (st) return st;
    if (c->xcd_copies) {
        if (c->cap_priv < (int64_t)kPrivCopies * g->ncells) {   // new copies start zero; every fold leaves them zero
            st = grow(c, &c->d_priv, c->cap_priv, (int64_t)kPrivCopies * g->ncells);
            if (st) return st;
            HIPCHK(c, launch_fill_f64(c->d_priv, 0.0, c->cap_priv, c->stream));
        }
        A.priv = c->d_priv;
        A.brick = brick_copies(g);
        if (A.ali_self) {
            if (c->cap_priv_self < (int64_t)kPrivCopies * g->ncells) {
                st = grow(c, &c->d_priv_self, c->cap_priv_self, (int64_t)kPrivCopies * g->ncells);
                if (st) return st;
                HIPCHK(c, launch_fill_f64(c->d_priv_self, 0.0, c->cap_priv_self, c->stream));
            }
            A.priv_self = c->d_priv_self;
        }
    }
    HIPCHK(c, launch_fill_u64((unsigned long long *)c->d_stats, 0ull, (int64_t)(sizeof(DevStats) / 8), c->stream));
    HIPCHK(c, launch_fill_u64(c->d_counter, 0ull, 1, c->stream));
    const int blocks = (int)(c->num_cus * c->blocks_per_cu);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    HIPCHK(c, launch_mc(A, blocks, (int)c->block, c->stream));
    if (c->timing) {
        HIPCHK(c, hipEventRecord(e1, c->stream));
        c->ev_start.push_back(e0);
        c->ev_stop.push_back(e1);
    }
    if (A.priv) HIPCHK(c, launch_fold_copies(d_absorbed, A.priv, g->ncells, A.brick, g->nx, g->ny, g->nroot, c->stream));
    if (A.priv_self)
        HIPCHK(c, launch_fold_copies(A.ali_self, A.priv_self, g->ncells, A.brick, g->nx, g->ny, g->nroot, c->stream));
    if (stats) {
        DevStats h;
        HIPCHK(c, hipMemcpyAsync(&h, c->d_stats, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        to_public(h, stats);
    }
    return SOC_OK;
}

soc_status soc_simulate_frequencies(soc_ctx c, soc_grid g, int32_t K, const soc_freq *freqs, const soc_sources *srcs,
                                    const uint32_t *freq_indices, uint64_t seed, uint32_t iteration,
                                    double *d_absorbed, soc_sim_stats *stats)
{
    if (!c) return SOC_EINVAL;
    if (!d_absorbed) return fail(c, SOC_EINVAL, "d_absorbed is NULL");
    if (!g) return fail(c, SOC_EINVAL, "grid is NULL");
    if (K < 1 || K > 4096) return fail(c, SOC_EINVAL, "K must be in [1, 4096]");
    if (!freqs || !srcs || !freq_indices) return fail(c, SOC_EINVAL, "freqs, srcs and freq_indices must be given");
    NOT_WHILE_CAPTURING(c);
    int64_t nL = 0, npk = 0, njobs = 0;
    uint64_t max_dust = 0;
    const auto batched = [](const soc_sources &q) {
        return q.d_T && q.n_dust > 0 && q.dust_mode == 1 && !(q.dust_cap > 0.0);
    };
    for (int32_t k = 0; k < K; ++k) {
        const soc_sources &q = srcs[k];
        if (q.d_ali_self != srcs[0].d_ali_self || q.d_ali_emitted != srcs[0].d_ali_emitted)
            return fail(c, SOC_EINVAL, "frequency %d: every frequency of the call must use the same ALI tallies", k);
        if (q.d_T && q.n_dust > 0) {
            if (q.dust_mode == 0 || q.dust_mode == 2 || q.dust_cap > 0.0) nL += g->ncells;   // the kernel reads L
            if (q.dust_mode != 0) npk += (int64_t)q.n_dust;
        }
        if (batched(q)) {
            ++njobs;
            max_dust = std::max<uint64_t>(max_dust, q.n_dust);
        }
    }
    // the weighted-mode tables of all frequencies are built together when
    // their rows fit in kDustRowsMaxBytes; otherwise one frequency at a time
    const int64_t scan_elems = (int64_t)scan_f64_scratch_elems(g->ncells);
    if ((double)njobs * (double)g->ncells * sizeof(double) > (double)kDustRowsMaxBytes) njobs = 0;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));   // the previous call's staging copy has been consumed
    soc_status st;
    if ((st = grow(c, &c->d_mL, c->cap_mL, std::max<int64_t>(nL, 1)))) return st;
    if ((st = grow(c, &c->d_mpk, c->cap_mpk, std::max<int64_t>(npk, 1)))) return st;
    if ((st = grow(c, &c->d_mS, c->cap_mS, K))) return st;
    if ((st = grow(c, &c->d_margs, c->cap_margs, K))) return st;
    if ((st = grow(c, &c->d_mcount, c->cap_mcount, K))) return st;
    if (njobs > 0) {
        if ((st = grow(c, &c->d_mincl, c->cap_mincl, njobs * g->ncells))) return st;
        if ((st = grow(c, &c->d_msums, c->cap_msums, njobs * scan_elems))) return st;
        if ((st = grow(c, &c->d_djobs, c->cap_djobs, njobs))) return st;
    }
    c->h_margs.resize(K);
    c->h_djobs.assign((size_t)njobs, DustJob{});
    int64_t oL = 0, opk = 0, j = 0;
    for (int32_t k = 0; k < K; ++k) {
        const soc_sources &q = srcs[k];
        ScratchSrc src;
        if (njobs > 0 && batched(q)) {
            src.job = &c->h_djobs[(size_t)j];
            src.incl = c->d_mincl + j * g->ncells;
            src.sums = c->d_msums + j * scan_elems;
            ++j;
        }
        const bool dust = q.d_T && q.n_dust > 0;
        if (dust && (q.dust_mode == 0 || q.dust_mode == 2 || q.dust_cap > 0.0)) {
            src.L = c->d_mL + oL;
            oL += g->ncells;
        }
        if (dust && q.dust_mode != 0) {
            src.pk = c->d_mpk + opk;
            opk += (int64_t)q.n_dust;
        }
        src.S = c->d_mS + k;
        McArgs &A = c->h_margs[k];
        if ((st = prepare(c, g, &freqs[k], &q, seed, iteration, freq_indices[k], d_absorbed, A, src)))
            return fail(c, st, "frequency %d: %s", k, c->err.c_str());
        A.next_id = c->d_mcount + k;
    }
    if (njobs > 0) {
        HIPCHK(c, hipMemcpyAsync(c->d_djobs, c->h_djobs.data(), sizeof(DustJob) * (size_t)njobs,
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, launch_dust_setup_rows(g->d_words, g->ncells, g->level_offset.data(), g->nlevels, g->root_cell_cm,
                                         c->d_djobs, (int32_t)njobs, max_dust, c->stream));
        if (srcs[0].d_ali_emitted) {
            for (int32_t k = 0; k < K; ++k) {
                const McArgs &A = c->h_margs[k];
                if (!batched(srcs[k])) continue;
                HIPCHK(c, launch_dust_emitted_weighted(A.dust_cell, A.n_dust, A.dust_L, A.dust_S, A.dust_mode,
                                                       A.dust_cap, srcs[k].d_ali_emitted, c->stream));
            }
        }
    }
    if (c->xcd_copies) {
        if (c->cap_priv < (int64_t)kPrivCopies * g->ncells) {   // new copies start zero; every fold leaves them zero
            if ((st = grow(c, &c->d_priv, c->cap_priv, (int64_t)kPrivCopies * g->ncells))) return st;
            HIPCHK(c, launch_fill_f64(c->d_priv, 0.0, c->cap_priv, c->stream));
        }
        for (auto &A : c->h_margs) {
            A.priv = c->d_priv;
            A.brick = brick_copies(g);
        }
        if (srcs[0].d_ali_self) {
            if (c->cap_priv_self < (int64_t)kPrivCopies * g->ncells) {
                if ((st = grow(c, &c->d_priv_self, c->cap_priv_self, (int64_t)kPrivCopies * g->ncells))) return st;
                HIPCHK(c, launch_fill_f64(c->d_priv_self, 0.0, c->cap_priv_self, c->stream));
            }
            for (auto &A : c->h_margs) A.priv_self = c->d_priv_self;
        }
    }
    HIPCHK(c, hipMemcpyAsync(c->d_margs, c->h_margs.data(), sizeof(McArgs) * (size_t)K, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, launch_fill_u64((unsigned long long *)c->d_stats, 0ull, (int64_t)(sizeof(DevStats) / 8), c->stream));
    HIPCHK(c, launch_fill_u64(c->d_mcount, 0ull, K, c->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    MultiArgs M;
    M.args = c->d_margs;
    M.K = K;
    M.spread = (int32_t)c->multi_spread;
    const bool ali = srcs[0].d_ali_self != nullptr;
    HIPCHK(c, launch_mc_multi(M, g->nlevels, ali, (int)(c->num_cus * c->blocks_per_cu), (int)c->block, c->stream));
    if (c->timing) {
        HIPCHK(c, hipEventRecord(e1, c->stream));
        c->ev_start.push_back(e0);
        c->ev_stop.push_back(e1);
    }
    if (c->xcd_copies)
        HIPCHK(c, launch_fold_copies(d_absorbed, c->d_priv, g->ncells, brick_copies(g), g->nx, g->ny, g->nroot, c->stream));
    if (c->xcd_copies && ali)
        HIPCHK(c, launch_fold_copies(srcs[0].d_ali_self, c->d_priv_self, g->ncells, brick_copies(g), g->nx, g->ny, g->nroot,
                                     c->stream));
    if (stats) {
        DevStats h;
        HIPCHK(c, hipMemcpyAsync(&h, c->d_stats, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        to_public(h, stats);
    }
    return SOC_OK;
}

soc_status soc_simulate_frequency_noalloc(soc_ctx c, soc_grid g, const soc_freq *f, const soc_sources *s,
                                          uint64_t seed, uint32_t iteration, uint32_t freq_index,
                                          double *d_absorbed, soc_sim_stats *stats)
{
    if (!c) return SOC_EINVAL;
    if (!d_absorbed) return fail(c, SOC_EINVAL, "d_absorbed is NULL");
    if (!g) return fail(c, SOC_EINVAL, "grid is NULL");
    if (g->ncells > kNaMaxCells)
        return fail(c, SOC_EINVAL, "no-allocation call: the grid's %lld cells exceed its limit of %lld",
                    (long long)g->ncells, (long long)kNaMaxCells);
    if (s && s->d_T && s->n_dust > 0 && s->dust_mode != 0 && s->n_dust > (uint64_t)kNaMaxDust)
        return fail(c, SOC_EINVAL, "no-allocation call: %llu weighted dust packages exceed its limit of %lld",
                    (unsigned long long)s->n_dust, (long long)kNaMaxDust);
    if (c->capturing && stats) return fail(c, SOC_ESTATE, "statistics not allowed during graph capture");
    HIPCHK(c, hipSetDevice(c->device));
    ScratchSrc src;
    src.base = na_base(c->device);
    if (!src.base) return fail(c, SOC_EHIP, "no-allocation scratch of device %d is not resolved", c->device);
    McArgs A;
    soc_status st = prepare(c, g, f, s, seed, iteration, freq_index, d_absorbed, A, src);
    if (st) return st;
    if (c->xcd_copies) {   // the array keeps the last call's contents: clear the copies this call uses
        A.priv = (double *)(src.base + kNaPriv);
        A.brick = brick_copies(g);
        HIPCHK(c, launch_fill_f64(A.priv, 0.0, (int64_t)kPrivCopies * g->ncells, c->stream));
        if (A.ali_self) {
            A.priv_self = (double *)(src.base + kNaPrivSelf);
            HIPCHK(c, launch_fill_f64(A.priv_self, 0.0, (int64_t)kPrivCopies * g->ncells, c->stream));
        }
    }
    HIPCHK(c, launch_fill_u64((unsigned long long *)A.st_call, 0ull, (int64_t)(sizeof(DevStats) / 8), c->stream));
    HIPCHK(c, launch_fill_u64(A.next_id, 0ull, 1, c->stream));
    HIPCHK(c, launch_mc(A, (int)(c->num_cus * c->blocks_per_cu), (int)c->block, c->stream));
    if (A.priv) HIPCHK(c, launch_fold_copies(d_absorbed, A.priv, g->ncells, A.brick, g->nx, g->ny, g->nroot, c->stream));
    if (A.priv_self)
        HIPCHK(c, launch_fold_copies(A.ali_self, A.priv_self, g->ncells, A.brick, g->nx, g->ny, g->nroot, c->stream));
    if (stats) {
        DevStats h;
        HIPCHK(c, hipMemcpyAsync(&h, A.st_call, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        to_public(h, stats);
    }
    return SOC_OK;
}

soc_status soc_read_stats(soc_ctx c, soc_sim_stats *out, int32_t reset)
{
    if (!c || !out) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    HIPCHK(c, hipSetDevice(c->device));
    DevStats h;
    HIPCHK(c, hipMemcpyAsync(&h, c->d_stats + 1, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    to_public(h, out);
    if (reset) HIPCHK(c, launch_fill_u64((unsigned long long *)(c->d_stats + 1), 0ull, (int64_t)(sizeof(DevStats) / 8), c->stream));
    return SOC_OK;
}

soc_status soc_scatter_map(soc_ctx c, soc_grid g, const soc_freq *f, const soc_sources *s, uint64_t seed,
                           uint32_t iteration, uint32_t freq_index, const soc_scatter_params *sp, double *d_image,
                           int32_t npx, int32_t npy, soc_scatter_stats *stats)
{
    if (!c) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    if (!sp || !d_image) return fail(c, SOC_EINVAL, "NULL argument");
    if (!s) return fail(c, SOC_EINVAL, "sources is NULL");
    if (s->d_T && s->n_dust > 0) return fail(c, SOC_EINVAL, "scattered-light runs take no dust emission");
    if (s->d_ali_self || s->d_ali_emitted) return fail(c, SOC_EINVAL, "scattered-light runs keep no ALI tallies");
    if ((sp->axis & 3) > 2 || (sp->axis & ~7) != 0) return fail(c, SOC_EINVAL, "axis must be 0..2, optionally | 4");
    if (sp->max_scatter < 0) return fail(c, SOC_EINVAL, "max_scatter must be >= 0");
    if (!f || !(f->w_nu > 0.0)) return fail(c, SOC_EINVAL, "w_nu must be > 0 for an image");
    HIPCHK(c, hipSetDevice(c->device));
    McArgs A;
    soc_status st = prepare(c, g, f, s, seed, iteration, freq_index, nullptr, A);
    if (st) return st;
    PeelArgs P;
    std::memset(&P, 0, sizeof P);
    P.axis = sp->axis & 3;
    const bool neg = (sp->axis & 4) != 0;
    P.ox = P.axis == 0 ? (neg ? -1.0f : 1.0f) : 0.0f;
    P.oy = P.axis == 1 ? (neg ? -1.0f : 1.0f) : 0.0f;
    P.oz = P.axis == 2 ? (neg ? -1.0f : 1.0f) : 0.0f;
    const int32_t N[3] = {g->nx, g->ny, g->nz};
    const int b = P.axis == 0 ? 1 : 0, cc = P.axis == 2 ? 1 : 2;
    const int64_t fine = (int64_t)1 << (g->nlevels - 1);
    if ((int64_t)npx != N[b] * fine || (int64_t)npy != N[cc] * fine)
        return fail(c, SOC_EINVAL, "image must be %lld x %lld pixels", (long long)(N[b] * fine), (long long)(N[cc] * fine));
    P.npx = npx;
    P.npy = npy;
    P.psz = 1.0 / (double)fine;
    const double pix_cm = g->root_cell_cm * P.psz;
    P.scale = 1.0 / (pix_cm * pix_cm * f->w_nu);
    P.forced = sp->forced ? 1 : 0;
    P.max_scatter = sp->max_scatter;
    P.direct = sp->direct ? 1 : 0;
    P.image = d_image;
    if ((st = grow(c, &c->d_peel, c->cap_peel, 8))) return st;
    HIPCHK(c, launch_fill_f64(c->d_peel, 0.0, 8, c->stream));
    P.totals = c->d_peel;
    HIPCHK(c, launch_fill_u64(c->d_counter, 0ull, 1, c->stream));   // id pool of the refill
    const int blocks = (int)(c->num_cus * 8);
    HIPCHK(c, launch_peel(A, P, blocks, c->stream));
    if (stats) {
        double h[6];
        HIPCHK(c, hipMemcpyAsync(h, c->d_peel, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        stats->packages = (uint64_t)h[0];
        stats->cell_steps = (uint64_t)h[1];
        stats->scatterings = (uint64_t)h[2];
        stats->ray_steps = (uint64_t)h[3];
        stats->e_emitted = h[4];
        stats->e_escaped = h[5];
    }
    return SOC_OK;
}

soc_status soc_shg_model_create(soc_ctx c, int32_t K, const double *nu, const double *w, int32_t S,
                                const double *abundance, const double *sigma, int32_t N, const double *U,
                                const double *T, soc_shg_model *out)
{
    if (!c) return SOC_EINVAL;
    if (!out) return fail(c, SOC_EINVAL, "out is NULL");
    *out = nullptr;
    if (K < 1 || K > kShgMaxK) return fail(c, SOC_EINVAL, "K must be in [1, %d]", kShgMaxK);
    if (N < 2 || N > kShgMaxN) return fail(c, SOC_EINVAL, "the enthalpy grid needs 2..%d bins", kShgMaxN);
    if (S < 1 || S > 4096) return fail(c, SOC_EINVAL, "S must be in [1, 4096]");
    if (!nu || !w || !abundance || !sigma || !U || !T) return fail(c, SOC_EINVAL, "NULL table");
    for (int k = 0; k < K; ++k) {
        if (!(nu[k] > 0.0) || !std::isfinite(nu[k]) || !finite_nonneg(w[k]))
            return fail(c, SOC_EINVAL, "nu must be > 0 and w >= 0");
        if (k > 0 && !(nu[k] > nu[k - 1])) return fail(c, SOC_EINVAL, "frequencies must increase");
    }
    for (int i = 0; i < S; ++i)
        if (!finite_nonneg(abundance[i])) return fail(c, SOC_EINVAL, "abundances must be finite and >= 0");
    for (int64_t i = 0; i < (int64_t)S * K; ++i)
        if (!finite_nonneg(sigma[i])) return fail(c, SOC_EINVAL, "cross sections must be finite and >= 0");
    for (int s2 = 0; s2 < S; ++s2)
        for (int i = 0; i < N; ++i) {
            const double u = U[(int64_t)s2 * N + i], t = T[(int64_t)s2 * N + i];
            if (!std::isfinite(u) || !(t > 0.0) || !std::isfinite(t)) return fail(c, SOC_EINVAL, "bad enthalpy grid");
            if (i > 0 && !(u > U[(int64_t)s2 * N + i - 1])) return fail(c, SOC_EINVAL, "enthalpies must increase");
        }
    HIPCHK(c, hipSetDevice(c->device));
    soc_shg_model m = new (std::nothrow) soc_shg_model_s;
    if (!m) return fail(c, SOC_ENOMEM, "out of host memory");
    m->ctx = c;
    m->device = c->device;
    m->S = S; m->K = K; m->N = N;
    const int64_t sk = (int64_t)S * K, sn = (int64_t)S * N;
    // layout: nu hnu inv_hnu w | abundance | sigma | U | T | share | emit | icool | idu | ks (bytes) | band (int32)
    int64_t ks_off = 4 * (int64_t)K + S + sk + 2 * sn + sk + sn * K + sn + sn;
    ks_off += ks_off & 1;   // 16-byte aligned
    const int64_t total = ks_off + ((int64_t)S * shg_ks_stride(N) + 4 * (int64_t)S + 7) / 8;
    if (hipMalloc((void **)&m->d_buf, sizeof(double) * (size_t)total) != hipSuccess) {
        delete m;
        return fail(c, SOC_ENOMEM, "device allocation of the grain model failed");
    }
    std::vector<double> h(4 * (size_t)K + S + sk + 2 * sn);
    const double hP = 6.62607015e-27;
    for (int k = 0; k < K; ++k) {
        h[k] = nu[k];
        h[K + k] = hP * nu[k];
        h[2 * K + k] = 1.0 / (hP * nu[k]);
        h[3 * K + k] = w[k];
    }
    std::memcpy(&h[4 * K], abundance, sizeof(double) * S);
    std::memcpy(&h[4 * K + S], sigma, sizeof(double) * sk);
    std::memcpy(&h[4 * K + S + sk], U, sizeof(double) * sn);
    std::memcpy(&h[4 * K + S + sk + sn], T, sizeof(double) * sn);
    double *d = m->d_buf;
    hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, c->stream);
    soc::ShgModelDev &v = m->dev;
    v.S = S; v.K = K; v.N = N;
    v.nu = d; v.hnu = d + K; v.inv_hnu = d + 2 * K;
    const double *dw = d + 3 * K;
    v.abundance = d + 4 * K;
    v.sigma = d + 4 * K + S;
    v.U = d + 4 * K + S + sk;
    v.T = d + 4 * K + S + sk + sn;
    v.share = d + 4 * K + S + sk + 2 * sn;
    v.emit = v.share + sk;
    v.icool = v.emit + sn * K;
    v.idu = v.icool + sn;
    v.ks = (uint8_t *)(d + ks_off);
    v.band = (int32_t *)(v.ks + (int64_t)S * shg_ks_stride(N));
    if (e == hipSuccess) e = launch_shg_prep(v, dw, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipFree(m->d_buf);
        delete m;
        return fail(c, SOC_EHIP, "grain model setup: %s", hipGetErrorString(e));
    }
    *out = m;
    return SOC_OK;
}

void soc_shg_model_destroy(soc_shg_model m)
{
    if (!m) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    (void)hipFree(m->d_buf);
    (void)hipSetDevice(cur);
    delete m;
}

soc_status soc_shg_solve(soc_ctx c, soc_grid g, soc_shg_model m, const double *d_absorbed, double *d_emission,
                         double *d_P)
{
    if (!c) return SOC_EINVAL;
    if (!g || !m || !d_absorbed || !d_emission) return fail(c, SOC_EINVAL, "NULL argument");
    if (g->ctx != c || m->ctx != c) return fail(c, SOC_EINVAL, "grid/model belong to another context");
    HIPCHK(c, hipSetDevice(c->device));
    ShgArgs a;
    std::memset(&a, 0, sizeof a);
    a.model = m->dev;
    a.words = g->d_words;
    a.ncells = g->ncells;
    for (int i = 0; i <= kMaxLevels; ++i) a.level_offset[i] = i <= g->nlevels ? g->level_offset[i] : g->ncells;
    a.nlevels = g->nlevels;
    a.root_cell_cm = g->root_cell_cm;
    a.absorbed = d_absorbed;
    a.emission = d_emission;
    a.P = d_P;
    HIPCHK(c, launch_shg(a, c->stream));
    return SOC_OK;
}

soc_status soc_reference_blend(soc_ctx c, int64_t n, double beta, const double *d_x, double *d_ref)
{
    if (!c) return SOC_EINVAL;
    if (n < 0) return fail(c, SOC_EINVAL, "n must be >= 0");
    if (n > 0 && (!d_x || !d_ref)) return fail(c, SOC_EINVAL, "array is NULL");
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(c, SOC_EINVAL, "beta must be in [0, 1]");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_blend(d_x, d_ref, n, beta, c->stream));
    return SOC_OK;
}

soc_status soc_trace_packages(soc_ctx c, soc_grid g, const soc_freq *f, const soc_sources *s, uint64_t seed,
                              uint32_t iteration, uint32_t freq_index, uint32_t cls, const uint32_t *ids, int32_t n,
                              int32_t precision, soc_segment *out, int32_t max_seg, int32_t *n_seg)
{
    if (!c) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    if (!ids || !out || !n_seg || n <= 0 || max_seg <= 0) return fail(c, SOC_EINVAL, "bad trace buffers");
    if (precision != 0 && precision != 1) return fail(c, SOC_EINVAL, "precision must be 0 or 1");
    HIPCHK(c, hipSetDevice(c->device));
    if (!s) return fail(c, SOC_EINVAL, "sources is NULL");
    soc_sources s_trace = *s;
    s_trace.ref_beta = 0.0;   // tracing leaves the reference emission and the ALI tallies as they are
    s_trace.d_ali_self = nullptr;
    s_trace.d_ali_emitted = nullptr;
    McArgs A;
    soc_status st = prepare(c, g, f, &s_trace, seed, iteration, freq_index, nullptr, A);
    if (st) return st;
    uint64_t limit;
    if (cls == kClassBg) limit = A.n_bg;
    else if (cls == kClassDust) limit = A.n_dust;
    else if (cls >= kClassPs0 && (int32_t)(cls - kClassPs0) < A.n_ps) limit = A.n_ps_pk;
    else return fail(c, SOC_EINVAL, "class %u has no packages", cls);
    for (int32_t i = 0; i < n; ++i)
        if (ids[i] >= limit) return fail(c, SOC_EINVAL, "package id %u out of range for class %u", ids[i], cls);
    static_assert(sizeof(SegmentDev) == sizeof(soc_segment), "segment layout");
    uint32_t *d_ids = nullptr;
    SegmentDev *d_out = nullptr;
    int32_t *d_n = nullptr;
    auto cleanup = [&](soc_status r) {
        (void)hipFree(d_ids); (void)hipFree(d_out); (void)hipFree(d_n);
        return r;
    };
    if (hipMalloc((void **)&d_ids, sizeof(uint32_t) * n) != hipSuccess ||
        hipMalloc((void **)&d_out, sizeof(SegmentDev) * (size_t)n * max_seg) != hipSuccess ||
        hipMalloc((void **)&d_n, sizeof(int32_t) * n) != hipSuccess)
        return cleanup(fail(c, SOC_ENOMEM, "trace buffers"));
    TraceArgs T;
    T.cls = cls;
    T.ids = d_ids;
    T.n = n;
    T.max_seg = max_seg;
    T.out = d_out;
    T.nseg = d_n;
    if (hipMemcpyAsync(d_ids, ids, sizeof(uint32_t) * n, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "copy ids"));
    hipError_t e = launch_trace(A, T, precision, c->stream);
    if (e != hipSuccess) return cleanup(fail(c, SOC_EHIP, "trace launch: %s", hipGetErrorString(e)));
    if (hipMemcpyAsync(out, d_out, sizeof(SegmentDev) * (size_t)n * max_seg, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(n_seg, d_n, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "trace readback: %s", hipGetErrorString(hipGetLastError())));
    return cleanup(SOC_OK);
}

soc_status soc_temp_table_build(soc_ctx c, int32_t K, const double *nu, const double *w_nu, const double *sigma_abs,
                                double T_floor, double T_max, int32_t nT, soc_temp_table *out)
{
    if (!c) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    if (!out || !nu || !w_nu || !sigma_abs || K < 1) return fail(c, SOC_EINVAL, "bad temperature table inputs");
    if (!(T_floor > 0.0 && T_max > T_floor && std::isfinite(T_max))) return fail(c, SOC_EINVAL, "need 0 < T_floor < T_max");
    if (nT < 16 || nT > 4096) return fail(c, SOC_EINVAL, "nT must be in [16,4096]");
    for (int k = 0; k < K; ++k)
        if (!(nu[k] > 0.0 && std::isfinite(nu[k])) || !finite_nonneg(w_nu[k]) || !finite_nonneg(sigma_abs[k]))
            return fail(c, SOC_EINVAL, "frequency %d: bad nu, w or sigma_abs", k);
    *out = nullptr;
    HIPCHK(c, hipSetDevice(c->device));
    soc_temp_table t = new (std::nothrow) soc_temp_table_s;
    if (!t) return fail(c, SOC_ENOMEM, "host allocation");
    t->ctx = c;
    t->device = c->device;
    t->nT = nT;
    t->T_floor = T_floor;
    t->T_max = T_max;
    t->lnTf = std::log(T_floor);
    t->dlnT = (std::log(T_max) - t->lnTf) / (nT - 1);
    double *d_f = nullptr;
    auto cleanup = [&](soc_status r) {
        (void)hipFree(d_f);
        if (r != SOC_OK) soc_temp_table_destroy(t);
        return r;
    };
    if (hipMalloc((void **)&t->d_lnG, sizeof(double) * nT) != hipSuccess ||
        hipMalloc((void **)&d_f, sizeof(double) * 3 * K) != hipSuccess)
        return cleanup(fail(c, SOC_ENOMEM, "temperature table"));
    if (hipMemcpyAsync(d_f, nu, sizeof(double) * K, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(d_f + K, w_nu, sizeof(double) * K, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(d_f + 2 * K, sigma_abs, sizeof(double) * K, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "table upload"));
    if (launch_temp_table(d_f, d_f + K, d_f + 2 * K, K, t->lnTf, t->dlnT, nT, t->d_lnG, c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "table launch"));
    std::vector<double> h(nT);
    if (hipMemcpyAsync(h.data(), t->d_lnG, sizeof(double) * nT, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "table readback"));
    for (int j = 0; j < nT; ++j) {
        if (!std::isfinite(h[j]) || (j > 0 && !(h[j] > h[j - 1])))
            return cleanup(fail(c, SOC_EINVAL, "Gamma(T) is not finite and increasing on [T_floor, T_max] (bin %d)", j));
    }
    *out = t;
    return cleanup(SOC_OK);
}

void soc_temp_table_destroy(soc_temp_table t)
{
    if (!t) return;
    (void)hipSetDevice(t->device);
    (void)hipFree(t->d_lnG);
    delete t;
}

// Statistics scratch of the temperature kernels (allocated on first use),
// with the fine histogram cleared by kernels (no memset nodes in graphs).
static soc_status temp_stats_buffers(soc_ctx c, TempArgs &a)
{
    if (!c->d_tpart) {
        if (c->capturing) return fail(c, SOC_ESTATE, "first temperature statistics call inside a graph capture");
        if (hipMalloc((void **)&c->d_tpart, (size_t)kTempBlocks * 8 * sizeof(double)) != hipSuccess ||
            hipMalloc((void **)&c->d_thist, (size_t)(kTempBlocks + 1) * kHistBins * sizeof(unsigned int)) != hipSuccess ||
            hipMalloc((void **)&c->d_tmeta, 8 * sizeof(double)) != hipSuccess ||
            hipMalloc((void **)&c->d_tfine_n, kHistBins * sizeof(unsigned int)) != hipSuccess ||
            hipMalloc((void **)&c->d_tfine_T, kHistBins * sizeof(double)) != hipSuccess)
            return fail(c, SOC_ENOMEM, "temperature statistics buffers");
    }
    HIPCHK(c, launch_fill_i32((int32_t *)c->d_tfine_n, 0, kHistBins, c->stream));
    HIPCHK(c, launch_fill_f64(c->d_tfine_T, 0.0, kHistBins, c->stream));
    a.part = c->d_tpart;
    a.hist_part = c->d_thist;
    a.hist_total = c->d_thist + (size_t)kTempBlocks * kHistBins;
    a.meta = c->d_tmeta;
    a.fine_n = c->d_tfine_n;
    a.fine_T = c->d_tfine_T;
    return SOC_OK;
}

static soc_status update_temperature(soc_ctx c, soc_grid g, soc_temp_table t, const double *d_absorbed,
                                     const double *d_self, const double *d_emitted, const float *d_T_old,
                                     float *d_T_new, soc_temp_stats *stats);

soc_status soc_update_temperature(soc_ctx c, soc_grid g, soc_temp_table t, const double *d_absorbed,
                                  const float *d_T_old, float *d_T_new, soc_temp_stats *stats)
{
    return update_temperature(c, g, t, d_absorbed, nullptr, nullptr, d_T_old, d_T_new, stats);
}

soc_status soc_update_temperature_ali(soc_ctx c, soc_grid g, soc_temp_table t, const double *d_absorbed,
                                      const double *d_ali_self, const double *d_ali_emitted, const float *d_T_old,
                                      float *d_T_new, soc_temp_stats *stats)
{
    if (!c) return SOC_EINVAL;
    if (!d_ali_self || !d_ali_emitted) return fail(c, SOC_EINVAL, "ALI tallies are NULL");
    return update_temperature(c, g, t, d_absorbed, d_ali_self, d_ali_emitted, d_T_old, d_T_new, stats);
}

static soc_status update_temperature(soc_ctx c, soc_grid g, soc_temp_table t, const double *d_absorbed,
                                     const double *d_self, const double *d_emitted, const float *d_T_old,
                                     float *d_T_new, soc_temp_stats *stats)
{
    if (!c) return SOC_EINVAL;
    if (!g || !t || !d_absorbed || !d_T_new) return fail(c, SOC_EINVAL, "NULL argument");
    if (g->ctx != c || t->ctx != c) return fail(c, SOC_EINVAL, "grid/table belong to another context");
    if (c->capturing && stats) return fail(c, SOC_ESTATE, "statistics not allowed during graph capture");
    HIPCHK(c, hipSetDevice(c->device));
    TempArgs a;
    std::memset(&a, 0, sizeof a);
    a.words = g->d_words;
    a.ncells = g->ncells;
    for (int i = 0; i <= kMaxLevels; ++i) a.level_offset[i] = i <= g->nlevels ? g->level_offset[i] : g->ncells;
    a.nlevels = g->nlevels;
    a.root_cell_cm = g->root_cell_cm;
    a.lnG = t->d_lnG;
    a.nT = t->nT;
    a.lnTf = t->lnTf;
    a.dlnT = t->dlnT;
    a.T_floor = t->T_floor;
    a.T_max = t->T_max;
    a.absorbed = d_absorbed;
    a.ali_self = d_self;
    a.ali_emit = d_emitted;
    a.T_old = d_T_old;
    a.T_new = d_T_new;
    int64_t blocks = (g->ncells + 255) / 256;
    a.blocks = (int32_t)(blocks < kTempBlocks ? (blocks < 1 ? 1 : blocks) : kTempBlocks);
    if (stats) {
        soc_status st = temp_stats_buffers(c, a);
        if (st != SOC_OK) return st;
    }
    HIPCHK(c, launch_temp_update(a, c->stream));
    if (stats) {
        HIPCHK(c, launch_temp_stats(a, c->d_tmp_out, c->stream));
        double h[4];
        HIPCHK(c, hipMemcpyAsync(h, c->d_tmp_out, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        stats->mean_T = h[0];
        stats->hot5_mean_T = h[1];
        stats->mean_rel_change = h[2];
        stats->clamped = (uint64_t)h[3];
    }
    return SOC_OK;
}

soc_status soc_temperature_stats(soc_ctx c, soc_grid g, soc_temp_table t, const float *d_T, soc_temp_stats *stats)
{
    if (!c) return SOC_EINVAL;
    if (!g || !t || !d_T || !stats) return fail(c, SOC_EINVAL, "NULL argument");
    if (g->ctx != c || t->ctx != c) return fail(c, SOC_EINVAL, "grid/table belong to another context");
    NOT_WHILE_CAPTURING(c);
    HIPCHK(c, hipSetDevice(c->device));
    TempArgs a;
    std::memset(&a, 0, sizeof a);
    a.words = g->d_words;
    a.ncells = g->ncells;
    for (int i = 0; i <= kMaxLevels; ++i) a.level_offset[i] = i <= g->nlevels ? g->level_offset[i] : g->ncells;
    a.nlevels = g->nlevels;
    a.root_cell_cm = g->root_cell_cm;
    a.lnG = t->d_lnG;
    a.nT = t->nT;
    a.lnTf = t->lnTf;
    a.dlnT = t->dlnT;
    a.T_floor = t->T_floor;
    a.T_max = t->T_max;
    a.T_new = const_cast<float *>(d_T);   // read only: the kernels never write in this mode
    a.given = 1;
    const int64_t blocks = (g->ncells + 255) / 256;
    a.blocks = (int32_t)(blocks < kTempBlocks ? (blocks < 1 ? 1 : blocks) : kTempBlocks);
    soc_status st = temp_stats_buffers(c, a);
    if (st != SOC_OK) return st;
    HIPCHK(c, launch_temp_update(a, c->stream));
    HIPCHK(c, launch_temp_stats(a, c->d_tmp_out, c->stream));
    double h[4];
    HIPCHK(c, hipMemcpyAsync(h, c->d_tmp_out, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    stats->mean_T = h[0];
    stats->hot5_mean_T = h[1];
    stats->mean_rel_change = 0.0;
    stats->clamped = 0;
    return SOC_OK;
}

soc_status soc_map(soc_ctx c, soc_grid g, const soc_freq *f, const float *d_T, int32_t axis, float *d_image,
                   int32_t npx, int32_t npy)
{
    if (!c) return SOC_EINVAL;
    soc_status st = check_freq(c, f);
    if (st) return st;
    if (!g || !d_T || !d_image) return fail(c, SOC_EINVAL, "NULL argument");
    if (g->ctx != c) return fail(c, SOC_EINVAL, "grid belongs to another context");
    const int a = axis & 3;
    if (a > 2 || (axis & ~7)) return fail(c, SOC_EINVAL, "axis must be 0..2, optionally | 4");
    const int64_t scale = (int64_t)1 << (g->nlevels - 1);
    const int32_t N[3] = {g->nx, g->ny, g->nz};
    const int b = a == 0 ? 1 : 0, cc = a == 2 ? 1 : 2;
    if ((int64_t)npx != N[b] * scale || (int64_t)npy != N[cc] * scale)
        return fail(c, SOC_EINVAL, "image must be %lld x %lld pixels", (long long)(N[b] * scale), (long long)(N[cc] * scale));
    HIPCHK(c, hipSetDevice(c->device));
    MapArgs m;
    m.words = g->d_words;
    m.nx = g->nx; m.ny = g->ny; m.nz = g->nz; m.nlevels = g->nlevels;
    m.root_cell_cm = g->root_cell_cm;
    m.axis = a;
    m.neg = (axis >> 2) & 1;
    m.npx = npx;
    m.npy = npy;
    m.nu = f->nu;
    m.sigma_abs = f->sigma_abs;
    m.sigma_ext = f->sigma_abs + f->sigma_sca;
    m.T = d_T;
    m.image = d_image;
    HIPCHK(c, launch_map(m, c->stream));
    return SOC_OK;
}

// ---------------------------------------------------------------- learned start
namespace {

// n and b of a regular cubic grid split into S^3 blocks, or an error.
soc_status sur_shape(soc_ctx c, soc_grid g, int32_t S, int32_t &n, int32_t &b)
{
    if (!g) return fail(c, SOC_EINVAL, "grid is NULL");
    if (g->ctx != c) return fail(c, SOC_EINVAL, "grid belongs to another context");
    if (g->nlevels != 1 || g->nx != g->ny || g->nx != g->nz)
        return fail(c, SOC_EINVAL, "the learned start takes regular cubic grids");
    if (S < 1 || g->nx % S != 0) return fail(c, SOC_EINVAL, "S must divide the grid size %d", g->nx);
    n = g->nx;
    b = n / S;
    return SOC_OK;
}

soc_status sur_table(soc_ctx c, soc_temp_table t)
{
    if (!t) return fail(c, SOC_EINVAL, "table is NULL");
    if (t->ctx != c) return fail(c, SOC_EINVAL, "table belongs to another context");
    return SOC_OK;
}

}  // namespace

soc_status soc_surrogate_features(soc_ctx c, soc_grid g, soc_temp_table t, int32_t S, int32_t K,
                                  const double *w_nu, const double *sigma_abs, const double *I_bg, double sigma_v,
                                  int32_t n_ps, const double *ps_pos, const double *ps_Lnu, const float *d_T1,
                                  float *d_features)
{
    if (!c) return SOC_EINVAL;
    int32_t n = 0, b = 0;
    soc_status st = sur_shape(c, g, S, n, b);
    if (st) return st;
    if ((st = sur_table(c, t))) return st;
    if (K < 1 || !w_nu || !sigma_abs || !I_bg || !d_T1 || !d_features) return fail(c, SOC_EINVAL, "NULL argument");
    if (n_ps < 0 || n_ps > kMaxPs || (n_ps > 0 && (!ps_pos || !ps_Lnu)))
        return fail(c, SOC_EINVAL, "n_ps must be in [0, %d] with positions and luminosities", kMaxPs);
    if (!(sigma_v > 0.0 && std::isfinite(sigma_v))) return fail(c, SOC_EINVAL, "sigma_v must be finite and > 0");
    SurFeatArgs a;
    std::memset(&a, 0, sizeof a);
    double F = 0.0, J = 0.0;
    for (int k = 0; k < K; ++k) {
        if (!finite_nonneg(w_nu[k]) || !finite_nonneg(sigma_abs[k]) || !finite_nonneg(I_bg[k]))
            return fail(c, SOC_EINVAL, "frequency %d: bad w, sigma_abs or I_bg", k);
        F += w_nu[k] * I_bg[k];
        J += w_nu[k] * sigma_abs[k] * I_bg[k];
    }
    if (!(F > 0.0)) return fail(c, SOC_EINVAL, "the external field must be > 0 at some frequency");
    a.F_ext = 4.0 * M_PI * F;
    a.Jbg = J;
    a.n_ps = n_ps;
    for (int p = 0; p < n_ps; ++p) {
        const double *q = ps_pos + 3 * p;
        if (!(q[0] >= 0.0 && q[0] < n && q[1] >= 0.0 && q[1] < n && q[2] >= 0.0 && q[2] < n))
            return fail(c, SOC_EINVAL, "point source %d lies outside the box", p);
        a.px[p] = q[0] / b;
        a.py[p] = q[1] / b;
        a.pz[p] = q[2] / b;
        double L = 0.0, Lw = 0.0;
        for (int k = 0; k < K; ++k) {
            const double v = ps_Lnu[(size_t)p * K + k];
            if (!finite_nonneg(v)) return fail(c, SOC_EINVAL, "point source %d: bad L_nu at frequency %d", p, k);
            L += w_nu[k] * v;
            Lw += w_nu[k] * sigma_abs[k] * v;
        }
        a.Lbol[p] = L;
        a.Lw[p] = Lw;
    }
    a.words = g->d_words;
    a.T1 = d_T1;
    a.n = n;
    a.S = S;
    a.b = b;
    a.cell_cm = g->root_cell_cm * b;
    a.sigma_v = sigma_v;
    a.T_floor = t->T_floor;
    a.lnG = t->d_lnG;
    a.nT = t->nT;
    a.lnTf = t->lnTf;
    a.dlnT = t->dlnT;
    a.out = d_features;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_sur_features(a, c->stream));
    return SOC_OK;
}

namespace {

soc_status sur_map_args(soc_ctx c, soc_grid g, int32_t S, int32_t stride, int32_t channel, double scale,
                        SurMapArgs &a)
{
    int32_t n = 0, b = 0;
    soc_status st = sur_shape(c, g, S, n, b);
    if (st) return st;
    if (stride < 1 || channel < 0 || channel >= stride)
        return fail(c, SOC_EINVAL, "need stride >= 1 and 0 <= channel < stride");
    if (!(std::isfinite(scale) && scale != 0.0)) return fail(c, SOC_EINVAL, "scale must be finite and non-zero");
    std::memset(&a, 0, sizeof a);
    a.words = g->d_words;
    a.n = n;
    a.S = S;
    a.b = b;
    a.stride = stride;
    a.channel = channel;
    a.scale = scale;
    return SOC_OK;
}

}  // namespace

soc_status soc_surrogate_target(soc_ctx c, soc_grid g, soc_temp_table t, int32_t S, const float *d_T,
                                const float *d_T1, double scale, float *d_target, int32_t stride, int32_t channel)
{
    if (!c) return SOC_EINVAL;
    SurMapArgs a;
    soc_status st = sur_map_args(c, g, S, stride, channel, scale, a);
    if (st) return st;
    if ((st = sur_table(c, t))) return st;
    if (!d_T || !d_T1 || !d_target) return fail(c, SOC_EINVAL, "NULL argument");
    if (!(scale > 0.0)) return fail(c, SOC_EINVAL, "scale must be > 0");
    a.T_floor = t->T_floor;
    a.T_max = t->T_max;
    a.T = d_T;
    a.T1 = d_T1;
    a.coarse = d_target;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_sur_target(a, c->stream));
    return SOC_OK;
}

soc_status soc_surrogate_target_absorbed(soc_ctx c, soc_grid g, int32_t S, const double *d_A, const double *d_A1,
                                         double scale, float *d_target, int32_t stride, int32_t channel)
{
    if (!c) return SOC_EINVAL;
    SurMapArgs a;
    soc_status st = sur_map_args(c, g, S, stride, channel, scale, a);
    if (st) return st;
    if (!d_A || !d_A1 || !d_target) return fail(c, SOC_EINVAL, "NULL argument");
    if (!(scale > 0.0)) return fail(c, SOC_EINVAL, "scale must be > 0");
    a.absorbed = 1;
    a.A = d_A;
    a.A1 = d_A1;
    a.coarse = d_target;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_sur_target(a, c->stream));
    return SOC_OK;
}

soc_status soc_surrogate_apply(soc_ctx c, soc_grid g, soc_temp_table t, int32_t S, const float *d_pred,
                               int32_t stride, int32_t channel, double scale, double offset, const float *d_T1,
                               float *d_T)
{
    if (!c) return SOC_EINVAL;
    SurMapArgs a;
    soc_status st = sur_map_args(c, g, S, stride, channel, scale, a);
    if (st) return st;
    if ((st = sur_table(c, t))) return st;
    if (!d_pred || !d_T1 || !d_T) return fail(c, SOC_EINVAL, "NULL argument");
    if (!std::isfinite(offset)) return fail(c, SOC_EINVAL, "offset must be finite");
    a.T_floor = t->T_floor;
    a.T_max = t->T_max;
    a.offset = offset;
    a.T1 = d_T1;
    a.pred = d_pred;
    a.T_out = d_T;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_sur_apply(a, c->stream));
    return SOC_OK;
}

soc_status soc_surrogate_apply_absorbed(soc_ctx c, soc_grid g, int32_t S, const float *d_pred, int32_t stride,
                                        int32_t channel, double scale, const double *d_A1, double *d_A)
{
    if (!c) return SOC_EINVAL;
    SurMapArgs a;
    soc_status st = sur_map_args(c, g, S, stride, channel, scale, a);
    if (st) return st;
    if (!d_pred || !d_A1 || !d_A) return fail(c, SOC_EINVAL, "NULL argument");
    a.absorbed = 1;
    a.A1 = d_A1;
    a.pred = d_pred;
    a.A_out = d_A;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_sur_apply(a, c->stream));
    return SOC_OK;
}

soc_status soc_batch_create(soc_ctx c, int32_t n_grids, const soc_grid *grids, int32_t n_pairs,
                            const soc_batch_pair *pairs, uint64_t seed, uint64_t tile_packages, soc_batch *out)
{
    if (!c) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    if (!out || !grids || !pairs || n_grids <= 0 || n_pairs <= 0) return fail(c, SOC_EINVAL, "bad batch arguments");
    if (tile_packages < 64 || tile_packages > 0x7FFFFFFFull) return fail(c, SOC_EINVAL, "tile_packages must be in [64, 2^31)");
    *out = nullptr;
    for (int32_t i = 0; i < n_grids; ++i) {
        if (!grids[i] || grids[i]->ctx != c) return fail(c, SOC_EINVAL, "grid %d is NULL or belongs to another context", i);
        if (grids[i]->nlevels != 1) return fail(c, SOC_EINVAL, "grid %d: batches take regular grids", i);
    }
    std::vector<PairDev> hp(n_pairs);
    std::vector<PsArg> hps;
    std::vector<int64_t> ps_off(n_pairs, 0);
    struct TileCost { double cost; TileDev t; };
    std::vector<TileCost> tiles;
    struct LdsPair { double cost; int32_t pair; };
    std::vector<LdsPair> lds;
    uint64_t total = 0;
    for (int32_t i = 0; i < n_pairs; ++i) {
        const soc_batch_pair &q = pairs[i];
        if (q.grid < 0 || q.grid >= n_grids) return fail(c, SOC_EINVAL, "pair %d: grid index out of range", i);
        const soc_grid g = grids[q.grid];
        soc_status st = check_freq(c, &q.freq);
        if (st) return st;
        if (!q.d_absorbed) return fail(c, SOC_EINVAL, "pair %d: d_absorbed is NULL", i);
        if (!finite_nonneg(q.I_bg_nu)) return fail(c, SOC_EINVAL, "pair %d: bad I_bg_nu", i);
        if (q.n_ps < 0 || q.n_ps > kMaxPs || (q.n_ps > 0 && !q.ps)) return fail(c, SOC_EINVAL, "pair %d: bad point sources", i);
        if (q.n_bg > 0xFFFFFFFFull || q.n_ps_pk > 0xFFFFFFFFull) return fail(c, SOC_EINVAL, "pair %d: package count too large", i);
        PairDev &P = hp[i];
        std::memset(&P, 0, sizeof P);
        P.words = g->d_words;
        P.absorbed = q.d_absorbed;
        P.nx = g->nx; P.ny = g->ny; P.nz = g->nz;
        P.ncells = g->ncells;
        const double s_cm = g->root_cell_cm;
        P.ks_f = (float)(q.freq.sigma_sca * s_cm);
        P.ka_f = (float)(q.freq.sigma_abs * s_cm);
        P.g_f = (float)q.freq.g;
        const double N0 = g->nx, N1 = g->ny, N2 = g->nz;
        const double area[6] = {N1 * N2, N1 * N2, N0 * N2, N0 * N2, N0 * N1, N0 * N1};
        double tot = 0.0, cum = 0.0;
        for (int k = 0; k < 6; ++k) tot += area[k];
        for (int k = 0; k < 6; ++k) { cum += area[k]; P.face_cum[k] = cum; }
        P.face_tot = tot;
        const double E_bg = M_PI * q.I_bg_nu * q.freq.w_nu * tot * (s_cm * s_cm);
        P.n_bg = q.n_bg;
        P.W_bg = q.n_bg ? E_bg / (double)q.n_bg : 0.0;
        P.n_ps = q.n_ps;
        P.n_ps_pk = q.n_ps > 0 ? q.n_ps_pk : 0;
        ps_off[i] = (int64_t)hps.size();
        for (int k = 0; k < q.n_ps; ++k) {
            const soc_point_source &ps = q.ps[k];
            if (!(ps.x >= 0.0 && ps.x < N0 && ps.y >= 0.0 && ps.y < N1 && ps.z >= 0.0 && ps.z < N2) || !finite_nonneg(ps.L_nu))
                return fail(c, SOC_EINVAL, "pair %d: point source %d outside the box or bad L_nu", i, k);
            PsArg a;
            a.x = ps.x; a.y = ps.y; a.z = ps.z;
            a.W = P.n_ps_pk ? ps.L_nu * q.freq.w_nu / (double)P.n_ps_pk : 0.0;
            hps.push_back(a);
        }
        P.n_total = P.n_bg + (uint64_t)P.n_ps * P.n_ps_pk;
        if (P.n_total > 0xFFFFFFFFull) return fail(c, SOC_EINVAL, "pair %d: more than 2^32 packages", i);
        P.key0 = (uint32_t)seed;
        P.key1 = (uint32_t)(seed >> 32) ^ (uint32_t)q.grid;
        P.freq_index = q.freq_index;
        // tiles, costed by packages x (optical size + grid extent); a pair
        // of a small grid is one workgroup's whole (LDS tally)
        const double extent = (double)(g->nx + g->ny + g->nz);
        if (g->ncells <= c->batch_lds_cells) {
            if (P.n_total > 0) lds.push_back({(double)P.n_total * extent, i});
            total += P.n_total;
            continue;
        }
        for (uint64_t b = 0; b < P.n_total; b += tile_packages) {
            TileCost tc;
            tc.t.pair = i;
            tc.t.begin = (uint32_t)b;
            tc.t.end = (uint32_t)std::min<uint64_t>(P.n_total, b + tile_packages);
            tc.t.pad = 0;
            tc.cost = (double)(tc.t.end - tc.t.begin) * extent;
            tiles.push_back(tc);
        }
        total += P.n_total;
    }
    // brick-ordered tallies (private copies on): one per array that only
    // tiled pairs of one grid with even dimensions add into
    struct Target { int32_t grid; bool ok; int64_t off; };
    std::map<double *, Target> targets;
    for (int32_t i = 0; i < n_pairs; ++i) {
        const soc_grid g = grids[pairs[i].grid];
        const bool tiled = g->ncells > c->batch_lds_cells;
        const bool even = g->nx % 2 == 0 && g->ny % 2 == 0 && g->nz % 2 == 0;
        auto it = targets.find(pairs[i].d_absorbed);
        if (it == targets.end())
            targets[pairs[i].d_absorbed] = Target{pairs[i].grid, tiled && even && c->xcd_copies != 0, 0};
        else if (it->second.grid != pairs[i].grid || !tiled)
            it->second.ok = false;
    }
    std::vector<BrickFold> folds;
    int64_t brick_cells = 0, max_fold_cells = 0;
    for (auto &kv : targets) {
        if (!kv.second.ok) continue;
        const soc_grid g = grids[kv.second.grid];
        kv.second.off = brick_cells;
        BrickFold f;
        f.tally = nullptr;   // set once the scratch exists
        f.absorbed = kv.first;
        f.nx = g->nx;
        f.ny = g->ny;
        f.ncells = g->ncells;
        folds.push_back(f);
        brick_cells += g->ncells;
        max_fold_cells = std::max<int64_t>(max_fold_cells, g->ncells);
    }
    std::stable_sort(tiles.begin(), tiles.end(), [](const TileCost &a, const TileCost &b) { return a.cost > b.cost; });
    std::stable_sort(lds.begin(), lds.end(), [](const LdsPair &a, const LdsPair &b) { return a.cost > b.cost; });
    std::vector<int32_t> hl(lds.size());
    int64_t lds_cells = 0;
    for (size_t i = 0; i < lds.size(); ++i) {
        hl[i] = lds[i].pair;
        lds_cells = std::max<int64_t>(lds_cells, hp[lds[i].pair].ncells);
    }
    HIPCHK(c, hipSetDevice(c->device));
    soc_batch b = new (std::nothrow) soc_batch_s;
    if (!b) return fail(c, SOC_ENOMEM, "host allocation");
    b->ctx = c;
    b->device = c->device;
    b->n_tiles = (int32_t)tiles.size();
    b->n_packages = total;
    b->n_lds_pairs = (int32_t)hl.size();
    b->lds_cells = lds_cells;
    b->n_folds = (int32_t)folds.size();
    b->max_fold_cells = max_fold_cells;
    auto cleanup = [&](soc_status r) {
        if (r != SOC_OK) soc_batch_destroy(b);
        return r;
    };
    if (hipMalloc((void **)&b->d_pairs, sizeof(PairDev) * n_pairs) != hipSuccess ||
        hipMalloc((void **)&b->d_tiles, sizeof(TileDev) * std::max<size_t>(1, tiles.size())) != hipSuccess ||
        hipMalloc((void **)&b->d_ps, sizeof(PsArg) * std::max<size_t>(1, hps.size())) != hipSuccess ||
        hipMalloc((void **)&b->d_counter, 2 * sizeof(unsigned int)) != hipSuccess ||
        hipMalloc((void **)&b->d_iteration, sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&b->d_lds_pairs, sizeof(int32_t) * std::max<size_t>(1, hl.size())) != hipSuccess ||
        hipMalloc((void **)&b->d_folds, sizeof(BrickFold) * std::max<size_t>(1, folds.size())) != hipSuccess ||
        (brick_cells > 0 && hipMalloc((void **)&b->d_brick, sizeof(double) * (size_t)brick_cells) != hipSuccess))
        return cleanup(fail(c, SOC_ENOMEM, "batch tables"));
    if (brick_cells > 0 && launch_fill_f64(b->d_brick, 0.0, brick_cells, c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "batch init"));
    for (auto &f : folds) f.tally = b->d_brick + targets[f.absorbed].off;
    for (int32_t i = 0; i < n_pairs; ++i) {
        hp[i].ps = hp[i].n_ps ? b->d_ps + ps_off[i] : nullptr;
        const Target &t = targets[hp[i].absorbed];
        hp[i].tally = t.ok ? b->d_brick + t.off : hp[i].absorbed;
        hp[i].brick = t.ok ? 1 : 0;
    }
    std::vector<TileDev> ht(tiles.size());
    for (size_t i = 0; i < tiles.size(); ++i) ht[i] = tiles[i].t;
    if (hipMemcpy(b->d_pairs, hp.data(), sizeof(PairDev) * n_pairs, hipMemcpyHostToDevice) != hipSuccess ||
        (ht.size() && hipMemcpy(b->d_tiles, ht.data(), sizeof(TileDev) * ht.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (hps.size() && hipMemcpy(b->d_ps, hps.data(), sizeof(PsArg) * hps.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (hl.size() && hipMemcpy(b->d_lds_pairs, hl.data(), sizeof(int32_t) * hl.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (folds.size() && hipMemcpy(b->d_folds, folds.data(), sizeof(BrickFold) * folds.size(), hipMemcpyHostToDevice) != hipSuccess))
        return cleanup(fail(c, SOC_EHIP, "batch upload"));
    if (launch_advance_iteration(b->d_iteration, 0, 0u, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return cleanup(fail(c, SOC_EHIP, "batch init"));
    *out = b;
    return SOC_OK;
}

void soc_batch_destroy(soc_batch b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipFree(b->d_pairs);
    (void)hipFree(b->d_tiles);
    (void)hipFree(b->d_ps);
    (void)hipFree(b->d_counter);
    (void)hipFree(b->d_iteration);
    (void)hipFree(b->d_lds_pairs);
    (void)hipFree(b->d_folds);
    (void)hipFree(b->d_brick);
    delete b;
}

soc_status soc_batch_info(soc_batch b, int32_t *n_tiles, uint64_t *n_packages)
{
    if (!b) return SOC_EINVAL;
    if (n_tiles) *n_tiles = b->n_tiles + b->n_lds_pairs;
    if (n_packages) *n_packages = b->n_packages;
    return SOC_OK;
}

soc_status soc_batch_run(soc_batch b, uint32_t iteration, soc_sim_stats *stats)
{
    if (!b) return SOC_EINVAL;
    soc_ctx c = b->ctx;
    if (c->capturing && (stats || c->timing)) return fail(c, SOC_ESTATE, "statistics/timing not allowed during graph capture");
    if (iteration != SOC_ITER_ADVANCE && iteration > 0xFFFFFFu) return fail(c, SOC_EINVAL, "iteration must be < 2^24");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_fill_u64((unsigned long long *)c->d_stats, 0ull, (int64_t)(sizeof(DevStats) / 8), c->stream));
    HIPCHK(c, launch_fill_i32((int32_t *)b->d_counter, 0, 2, c->stream));
    HIPCHK(c, launch_advance_iteration(b->d_iteration, iteration == SOC_ITER_ADVANCE ? 1 : 0,
                                       iteration == SOC_ITER_ADVANCE ? 0u : iteration, c->stream));
    BatchArgs a;
    a.pairs = b->d_pairs;
    a.tiles = b->d_tiles;
    a.n_tiles = b->n_tiles;
    a.next_tile = b->d_counter;
    a.lds_pairs = b->d_lds_pairs;
    a.n_lds_pairs = b->n_lds_pairs;
    a.next_lds = b->d_counter + 1;
    a.iteration = b->d_iteration;
    a.step_cap = c->step_cap;
    a.st_call = c->d_stats;
    a.st_total = c->d_stats + 1;
    a.refill_min = (int32_t)c->refill_min;
    a.inner_steps = (int32_t)c->inner_steps;
    a.scatter_min = (int32_t)c->scatter_min;
    a.chunk = (int32_t)c->chunk;
    int blocks = (int)(c->num_cus * c->blocks_per_cu), threads = (int)c->block;
    if (b->n_lds_pairs > 0) {
        // a workgroup holds a small grid's tally: 512-lane workgroups, as many
        // per compute unit as their LDS allows (at most two)
        threads = kMcMaxBlock;
        const int64_t ring = (int64_t)kRingStride * threads * (int64_t)(sizeof(double) + sizeof(int32_t));
        const int64_t need = std::max<int64_t>(ring, b->lds_cells * (int64_t)sizeof(double)) + 256;
        const int64_t per_cu = std::min<int64_t>(2, std::max<int64_t>(1, c->lds_per_cu / need));
        blocks = (int)(c->num_cus * per_cu);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    HIPCHK(c, launch_mc_batch(a, blocks, threads, b->lds_cells, c->stream));
    HIPCHK(c, launch_batch_fold(b->d_folds, b->n_folds, b->max_fold_cells, c->stream));
    if (c->timing) {
        HIPCHK(c, hipEventRecord(e1, c->stream));
        c->ev_start.push_back(e0);
        c->ev_stop.push_back(e1);
    }
    if (stats) {
        DevStats h;
        HIPCHK(c, hipMemcpyAsync(&h, c->d_stats, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        to_public(h, stats);
    }
    return SOC_OK;
}

soc_status soc_ubench(soc_ctx c, int32_t which, void *d_buf, void *d_buf2, uint64_t n, int32_t per_thread,
                      int32_t mode, int32_t blocks, int32_t threads, double *ms)
{
    if (!c) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    if (!d_buf || !ms || n == 0 || n > 0xFFFFFFFFull || per_thread < 1 || blocks < 1 || threads < 64 ||
        threads > 1024 || which < 0 || which > 2 || (which != 0 && !d_buf2) ||
        (which == 0 && (mode < 0 || mode > 6 || (mode == 2 && n < 64) || (mode == 3 && n < 4096))))
        return fail(c, SOC_EINVAL, "bad micro-benchmark arguments");
    HIPCHK(c, hipSetDevice(c->device));
    struct Events {   // destroyed on every return path
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events()
        {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    HIPCHK(c, hipEventCreate(&ev.e[0]));
    HIPCHK(c, hipEventCreate(&ev.e[1]));
    HIPCHK(c, hipEventRecord(ev.e[0], c->stream));
    HIPCHK(c, launch_ubench(which, d_buf, d_buf2, n, per_thread, mode, blocks, threads, c->stream));
    HIPCHK(c, hipEventRecord(ev.e[1], c->stream));
    HIPCHK(c, hipEventSynchronize(ev.e[1]));
    float t = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&t, ev.e[0], ev.e[1]));
    *ms = t;
    return SOC_OK;
}

soc_status soc_graph_begin(soc_ctx c)
{
    if (!c) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    if (!c->stream) return fail(c, SOC_ESTATE, "graph capture needs a stream other than the null stream");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    c->capturing = true;
    return SOC_OK;
}

soc_status soc_graph_end(soc_ctx c, soc_graph *out)
{
    if (!c || !out) return SOC_EINVAL;
    if (!c->capturing) return fail(c, SOC_ESTATE, "no capture in progress");
    c->capturing = false;
    hipGraph_t graph = nullptr;
    HIPCHK(c, hipStreamEndCapture(c->stream, &graph));
    soc_graph g = new (std::nothrow) soc_graph_s;
    if (!g) {
        (void)hipGraphDestroy(graph);
        return fail(c, SOC_ENOMEM, "host allocation");
    }
    g->device = c->device;
    g->stream = c->stream;
    g->graph = graph;
    hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        soc_graph_destroy(g);
        return fail(c, SOC_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *out = g;
    return SOC_OK;
}

soc_status soc_graph_launch(soc_graph g)
{
    if (!g) return SOC_EINVAL;
    if (hipSetDevice(g->device) != hipSuccess) return SOC_EHIP;
    return hipGraphLaunch(g->exec, g->stream) == hipSuccess ? SOC_OK : SOC_EHIP;
}

void soc_graph_destroy(soc_graph g)
{
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"

// ---------------------------------------------------------------- surrogate
struct soc_unet_s {
    soc_ctx ctx = nullptr;   // identity check only
    int device = 0;
    soc::unet::Net net;
};

#define UNET_ARGS(c, u)                                                            \
    do {                                                                           \
        if (!(c) || !(u)) return SOC_EINVAL;                                       \
        if ((u)->device != (c)->device)                                            \
            return fail((c), SOC_EINVAL, "network and context on different devices"); \
        HIPCHK((c), hipSetDevice((c)->device));                                    \
    } while (0)

soc_status soc_unet_create(soc_ctx c, const soc_unet_desc *d, uint64_t seed, soc_unet *out)
{
    if (!c || !d || !out) return SOC_EINVAL;
    NOT_WHILE_CAPTURING(c);
    *out = nullptr;
    HIPCHK(c, hipSetDevice(c->device));
    soc_unet u = new (std::nothrow) soc_unet_s;
    if (!u) return fail(c, SOC_ENOMEM, "host allocation failed");
    u->ctx = c;
    u->device = c->device;
    const auto st =
        u->net.create(c->device, d->cin, d->cout, d->base, d->levels, d->nmax, d->nz, d->ny, d->nx, seed, c->stream);
    if (st.code != soc::unet::Net::OK) {
        delete u;
        const soc_status code = st.code == soc::unet::Net::BAD_SHAPE   ? SOC_EINVAL
                                : st.code == soc::unet::Net::NO_MEMORY ? SOC_ENOMEM
                                                                       : SOC_EHIP;
        return fail(c, code, "soc_unet_create: %s", st.msg.c_str());
    }
    *out = u;
    return SOC_OK;
}

void soc_unet_destroy(soc_unet u)
{
    if (!u) return;
    (void)hipSetDevice(u->device);
    delete u;
}

soc_status soc_unet_param_count(soc_unet u, int64_t *count)
{
    if (!u || !count) return SOC_EINVAL;
    *count = u->net.param_count();
    return SOC_OK;
}

soc_status soc_unet_set_params(soc_ctx c, soc_unet u, const float *h_params)
{
    UNET_ARGS(c, u);
    NOT_WHILE_CAPTURING(c);
    if (!h_params) return fail(c, SOC_EINVAL, "NULL parameters");
    HIPCHK(c, u->net.set_params(h_params, c->stream));
    return SOC_OK;
}

soc_status soc_unet_get_params(soc_ctx c, soc_unet u, float *h_params)
{
    UNET_ARGS(c, u);
    NOT_WHILE_CAPTURING(c);
    if (!h_params) return fail(c, SOC_EINVAL, "NULL parameters");
    HIPCHK(c, u->net.get_params(h_params, c->stream));
    return SOC_OK;
}

soc_status soc_unet_get_grads(soc_ctx c, soc_unet u, float *h_grads)
{
    UNET_ARGS(c, u);
    NOT_WHILE_CAPTURING(c);
    if (!h_grads) return fail(c, SOC_EINVAL, "NULL gradients");
    HIPCHK(c, u->net.get_grads(h_grads, c->stream));
    return SOC_OK;
}

soc_status soc_unet_forward(soc_ctx c, soc_unet u, int32_t n, const float *d_x, float *d_y)
{
    UNET_ARGS(c, u);
    if (n < 1 || n > u->net.nmax_ || !d_x || !d_y)
        return fail(c, SOC_EINVAL, "soc_unet_forward: batch %d outside [1, %d] or NULL buffer", n, u->net.nmax_);
    HIPCHK(c, u->net.forward(n, d_x, d_y, c->stream));
    return SOC_OK;
}

soc_status soc_unet_backward(soc_ctx c, soc_unet u, const float *d_dy)
{
    UNET_ARGS(c, u);
    if (!d_dy) return fail(c, SOC_EINVAL, "NULL output gradient");
    if (u->net.n_last_ < 1) return fail(c, SOC_ESTATE, "soc_unet_backward before any forward");
    HIPCHK(c, u->net.backward(d_dy, c->stream));
    return SOC_OK;
}

soc_status soc_unet_backward_to(soc_ctx c, soc_unet u, const float *d_dy, int32_t stop_layer)
{
    UNET_ARGS(c, u);
    if (!d_dy) return fail(c, SOC_EINVAL, "NULL output gradient");
    if (stop_layer < 0 || stop_layer >= u->net.layer_count())
        return fail(c, SOC_EINVAL, "soc_unet_backward_to: layer %d outside [0, %d)", stop_layer, u->net.layer_count());
    if (u->net.n_last_ < 1) return fail(c, SOC_ESTATE, "soc_unet_backward_to before any forward");
    HIPCHK(c, u->net.backward(d_dy, c->stream, stop_layer));
    return SOC_OK;
}

soc_status soc_unet_read(soc_ctx c, soc_unet u, int32_t layer, int32_t which, float *h_out, int64_t count)
{
    UNET_ARGS(c, u);
    NOT_WHILE_CAPTURING(c);
    const auto st = u->net.read(layer, which, h_out, count, c->stream);
    if (st.code == soc::unet::Net::HIP_ERROR) return fail(c, SOC_EHIP, "soc_unet_read: %s", st.msg.c_str());
    if (st.code != soc::unet::Net::OK) return fail(c, SOC_EINVAL, "soc_unet_read: %s", st.msg.c_str());
    return SOC_OK;
}

soc_status soc_unet_mse(soc_ctx c, soc_unet u, int32_t n, const float *d_y, const float *d_t, float *d_dy,
                        double *loss)
{
    UNET_ARGS(c, u);
    if (loss) NOT_WHILE_CAPTURING(c);
    if (n < 1 || n > u->net.nmax_ || !d_y || !d_t) return fail(c, SOC_EINVAL, "soc_unet_mse: bad arguments");
    HIPCHK(c, u->net.mse(n, d_y, d_t, d_dy, loss, c->stream));
    return SOC_OK;
}

soc_status soc_unet_adam(soc_ctx c, soc_unet u, float lr, float beta1, float beta2, float eps, int32_t step)
{
    UNET_ARGS(c, u);
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
        step < 1)
        return fail(c, SOC_EINVAL, "soc_unet_adam: bad hyper-parameters");
    HIPCHK(c, u->net.adam(lr, beta1, beta2, eps, step, c->stream));
    return SOC_OK;
}

soc_status soc_unet_flops(soc_unet u, int32_t n, int64_t *flops)
{
    if (!u || !flops || n < 1) return SOC_EINVAL;
    *flops = u->net.flops_forward(n);
    return SOC_OK;
}
