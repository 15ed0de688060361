// setup.hip -- per-frequency setup and grid preparation kernels.
//
//  * dust luminosity per cell, 4 pi sigma_abs n V B_nu(T) w (Sect. 3.2 dust
//    re-emission), or its difference to a reference emission (Sect. 2.1.2),
//    its inclusive prefix sum, the capped expected package counts and the
//    systematic selection of the cell of every weighted dust package;
//  * the running-mean blend of the reference field;
//  * device-side validation of the hierarchical grid and construction of
//    the reverse (parent) links and the leaf list (Sect. 2.1.1);
//  * small fills used instead of hipMemsetAsync so that captured graphs
//    contain only kernels.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "soc_kernels.h"

namespace soc {

// ------------------------------------------------------------------ fills
template <typename T>
__global__ void fill_kernel(T *p, T v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
static hipError_t fill(T *p, T v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }

__global__ void copy_f64_kernel(const double *src, double *dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

// Private copies of the absorbed array: add the kPrivCopies copies into the
// caller's array in copy order and leave them zero for the next launch.
// Brick order of the root cells (hx = nx / 2 > 0, hy = ny / 2, entries
// i < nroot): copy entry i is root cell (2 bx + i mod 2, 2 by + (i / 2) mod 2,
// 2 bz + (i / 4) mod 2) of brick i / 8 = bx + hx (by + hy bz); the other
// entries are in cell order.
__global__ void fold_copies_kernel(double *absorbed, double *priv, int64_t n, int32_t hx, int32_t hy, int64_t nroot)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (uint32_t x = 0; x < kPrivCopies; ++x) {
            s += priv[x * n + i];
            priv[x * n + i] = 0.0;
        }
        int64_t c = i;
        if (hx > 0 && i < nroot) {
            const int64_t b = i >> 3, bx = b % hx, t = b / hx, by = t % hy, bz = t / hy;
            c = ((2 * bz + ((i >> 2) & 1)) * (2 * hy) + 2 * by + ((i >> 1) & 1)) * (2 * hx) + 2 * bx + (i & 1);
        }
        if (s != 0.0) absorbed[c] += s;
    }
}

hipError_t launch_fold_copies(double *absorbed, double *priv, int64_t n, int32_t brick, int32_t nx, int32_t ny,
                              int64_t nroot, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(fold_copies_kernel, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s, absorbed, priv, n,
                       brick ? nx / 2 : 0, brick ? ny / 2 : 0, nroot);
    return hipGetLastError();
}

// ------------------------------------------------------------------ levels
__device__ inline int level_of(int64_t c, const int64_t *lo, int32_t nlevels)
{
    int L = 0;
    while (L + 1 < nlevels && c >= lo[L + 1]) ++L;
    return L;
}

struct Levels {
    int64_t off[kMaxLevels + 1];
};

// ------------------------------------------------------------------ Planck
// B_nu(T) = 2 h nu^3 / c^2 / (exp(h nu / k T) - 1), CODATA 2018 cgs.
__device__ inline double planck_nu(double nu, double T)
{
    const double h = 6.62607015e-27, k = 1.380649e-16, c = 2.99792458e10;
    if (!(T > 0.0)) return 0.0;
    const double x = h * nu / (k * T);
    const double pre = 2.0 * h * nu * nu * nu / (c * c);
    if (x > 700.0) return pre * exp(-x);
    return pre / expm1(x);
}

// Dust luminosity of cell c in one frequency band: 4 pi sigma_abs n V B_nu(T) w_nu
// (Sect. 3.2); zero for a refined cell.
__device__ inline double cell_luminosity(const uint32_t *words, int64_t c, const Levels &lv, int32_t nlevels,
                                         double root_cell_cm, double nu, double sigma_abs, double w_nu,
                                         const float *T)
{
    const double four_pi = 12.566370614359172;
    const uint32_t w = words[c];
    if ((int32_t)w < 0) return 0.0;
    const double n = (double)__uint_as_float(w);
    const int Lv = level_of(c, lv.off, nlevels);
    const double s = ldexp(root_cell_cm, -Lv);
    return four_pi * sigma_abs * n * (s * s * s) * planck_nu(nu, (double)T[c]) * w_nu;
}

__global__ void dust_luminosity_kernel(const uint32_t *words, int64_t ncells, Levels lv, int32_t nlevels,
                                       double root_cell_cm, double nu, double sigma_abs, double w_nu,
                                       const float *T, double *L)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += (int64_t)gridDim.x * blockDim.x)
        L[c] = cell_luminosity(words, c, lv, nlevels, root_cell_cm, nu, sigma_abs, w_nu, T);
}

hipError_t launch_dust_luminosity(const uint32_t *words, int64_t ncells, const int64_t *level_offset,
                                  int32_t nlevels, double root_cell_cm, double nu, double sigma_abs,
                                  double w_nu, const float *T, double *L, hipStream_t s)
{
    Levels lv;
    for (int i = 0; i <= kMaxLevels; ++i) lv.off[i] = i <= nlevels ? level_offset[i] : ncells;
    int64_t blocks = (ncells + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(dust_luminosity_kernel, dim3((unsigned)blocks), dim3(256), 0, s, words, ncells, lv,
                       nlevels, root_cell_cm, nu, sigma_abs, w_nu, T, L);
    return hipGetLastError();
}

// Reference-field emission (Sect. 2.1.2): the difference between the
// dust emission at T and the reference emission, its magnitude (the
// selection weight), and the reference blended towards the current
// emission with weight beta.
__global__ void dust_correction_kernel(const uint32_t *words, int64_t ncells, Levels lv, int32_t nlevels,
                                       double root_cell_cm, double nu, double sigma_abs, double w_nu,
                                       const float *T, double *L_ref, double beta, double *dL, double *a)
{
    const double four_pi = 12.566370614359172;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t w = words[c];
        double L = 0.0;
        if ((int32_t)w >= 0) {
            const double n = (double)__uint_as_float(w);
            const int Lv = level_of(c, lv.off, nlevels);
            const double s = ldexp(root_cell_cm, -Lv);
            L = four_pi * sigma_abs * n * (s * s * s) * planck_nu(nu, (double)T[c]) * w_nu;
        }
        const double r = L_ref[c];
        const double d = L - r;
        dL[c] = d;
        a[c] = fabs(d);
        if (beta != 0.0) L_ref[c] = r + beta * d;
    }
}

hipError_t launch_dust_correction(const uint32_t *words, int64_t ncells, const int64_t *level_offset,
                                  int32_t nlevels, double root_cell_cm, double nu, double sigma_abs,
                                  double w_nu, const float *T, double *L_ref, double beta, double *dL, double *a,
                                  hipStream_t s)
{
    Levels lv;
    for (int i = 0; i <= kMaxLevels; ++i) lv.off[i] = i <= nlevels ? level_offset[i] : ncells;
    int64_t blocks = (ncells + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(dust_correction_kernel, dim3((unsigned)blocks), dim3(256), 0, s, words, ncells, lv,
                       nlevels, root_cell_cm, nu, sigma_abs, w_nu, T, L_ref, beta, dL, a);
    return hipGetLastError();
}

__global__ void abs_f64_kernel(const double *L, double *a, int64_t n)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        a[c] = fabs(L[c]);
}

hipError_t launch_abs_f64(const double *L, double *a, int64_t n, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(abs_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, L, a, n);
    return hipGetLastError();
}

// Emission-weighting cap (Sect. 3.2): the expected package count of a
// cell, N a_c / S, limited to `cap`; the excess is not re-assigned.
__global__ void dust_cap_kernel(double *a, int64_t n, const double *S_in, double *S_out, uint64_t n_dust, double cap)
{
    const double S = *S_in;
    if (threadIdx.x == 0 && blockIdx.x == 0) *S_out = S;
    const double scale = S > 0.0 ? (double)n_dust / S : 0.0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        a[c] = fmin(a[c] * scale, cap);
}

hipError_t launch_dust_cap(double *a, int64_t n, const double *S_in, double *S_out, uint64_t n_dust, double cap,
                           hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(dust_cap_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, n, S_in, S_out, n_dust, cap);
    return hipGetLastError();
}

// Diagonal ALI, emitted dust energy per cell.  The packages of a cell form
// one run of the non-decreasing cell list; the thread at the end of a run
// finds its start by binary search and adds count x weight, so every cell
// has one writer and no atomics are needed.
__global__ void dust_emitted_weighted_kernel(const int32_t *cell, uint64_t n_dust, const double *dL, const double *S,
                                             int32_t mode, double cap, double *E)
{
    const double WN = *S / (double)n_dust;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_dust; j += (uint64_t)gridDim.x * blockDim.x) {
        const int32_t c = cell[j];
        if (c < 0) continue;
        if (j + 1 < n_dust && cell[j + 1] == c) continue;
        uint64_t lo = 0, hi = j;   // first index whose cell is c (cells are non-decreasing before any -1)
        while (lo < hi) {
            const uint64_t mid = lo + ((hi - lo) >> 1);
            if (cell[mid] < c) lo = mid + 1; else hi = mid;
        }
        const double W0 = (mode == 1 && !(cap > 0.0)) ? WN : weighted_package_weight(WN, cap, dL[c]);
        E[c] += (double)(j - lo + 1) * W0;
    }
}

hipError_t launch_dust_emitted_weighted(const int32_t *cell, uint64_t n_dust, const double *dL, const double *S,
                                        int32_t mode, double cap, double *E, hipStream_t s)
{
    if (n_dust == 0) return hipSuccess;
    uint64_t blocks = (n_dust + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(dust_emitted_weighted_kernel, dim3((unsigned)blocks), dim3(256), 0, s, cell, n_dust, dL, S,
                       mode, cap, E);
    return hipGetLastError();
}

__global__ void dust_emitted_uniform_kernel(const int64_t *leaves, int64_t nleaves, const double *L, uint64_t per_leaf,
                                            double *E)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nleaves; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = leaves ? leaves[i] : i;
        E[c] += (double)per_leaf * (L[c] / (double)per_leaf);
    }
}

hipError_t launch_dust_emitted_uniform(const int64_t *leaves, int64_t nleaves, const double *L, uint64_t per_leaf,
                                       double *E, hipStream_t s)
{
    if (nleaves == 0) return hipSuccess;
    int64_t blocks = (nleaves + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(dust_emitted_uniform_kernel, dim3((unsigned)blocks), dim3(256), 0, s, leaves, nleaves, L,
                       per_leaf, E);
    return hipGetLastError();
}

__global__ void blend_kernel(const double *x, double *ref, int64_t n, double beta)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const double r = ref[c];
        ref[c] = r + beta * (x[c] - r);
    }
}

hipError_t launch_blend(const double *x, double *ref, int64_t n, double beta, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(blend_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, ref, n, beta);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scans
// Three-pass inclusive scan: tile sums, a single-workgroup scan of the tile
// sums (looping over chunks with a carry), then the per-tile scan with its
// offset.  Tiles of 256 threads x 8 items.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ inline T block_inclusive_scan(T v, T *sh)
{
    // Hillis-Steele over the workgroup through LDS
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        T add = t >= o ? sh[t - o] : (T)0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    T r = sh[t];
    __syncthreads();
    return r;
}

// The three passes of the scan as block bodies (tile = the block's tile),
// shared by the single-array kernels and the batched ones below.
template <typename T>
__device__ inline void tile_sums_body(const T *in, int64_t n, T *sums, int64_t tile, T *sh)
{
    const int64_t base = tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        if (i < n) acc += in[i];
    }
    T tot = block_inclusive_scan<T>(acc, sh);
    if (threadIdx.x == kScanThreads - 1) sums[tile] = tot;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_tile_sums(const T *in, int64_t n, T *sums)
{
    __shared__ T sh[kScanThreads];
    tile_sums_body<T>(in, n, sums, blockIdx.x, sh);
}

template <typename T>
__device__ inline void sums_exclusive_body(T *sums, int64_t m)
{
    __shared__ T sh[kScanThreads];
    __shared__ T tail;
    T carry = 0;
    for (int64_t base = 0; base < m; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        const T v = i < m ? sums[i] : (T)0;
        const T inc = block_inclusive_scan<T>(v, sh);
        if (i < m) sums[i] = carry + inc - v;
        if (threadIdx.x == kScanThreads - 1) tail = inc;
        __syncthreads();
        carry += tail;
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_sums_exclusive(T *sums, int64_t m)
{
    sums_exclusive_body<T>(sums, m);
}

// Every thread reads its items before it writes, and the threads' ranges
// are disjoint, so `out` may be `in`.
template <typename T>
__device__ inline void tiles_apply_body(const T *in, int64_t n, const T *offsets, T *out, int inclusive, int64_t tile,
                                        T *sh)
{
    const int64_t base = tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        v[k] = i < n ? in[i] : (T)0;
        acc += v[k];
    }
    const T inc = block_inclusive_scan<T>(acc, sh);
    T run = offsets[tile] + inc - acc;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        const T before = run;
        run += v[k];
        if (i < n) out[i] = inclusive ? run : before;
    }
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_tiles_apply(const T *in, int64_t n, const T *offsets, T *out,
                                                                 int inclusive)
{
    __shared__ T sh[kScanThreads];
    tiles_apply_body<T>(in, n, offsets, out, inclusive, blockIdx.x, sh);
}

template <typename T>
static hipError_t scan_generic(const T *in, T *out, int64_t n, T *scratch, int inclusive, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tile_sums<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, n, scratch);
    hipLaunchKernelGGL(scan_sums_exclusive<T>, dim3(1), dim3(kScanThreads), 0, s, scratch, tiles);
    hipLaunchKernelGGL(scan_tiles_apply<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, n,
                       (const T *)scratch, out, inclusive);
    return hipGetLastError();
}

size_t scan_f64_scratch_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }
size_t scan_i64_scratch_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

hipError_t launch_scan_f64(const double *in, double *out, int64_t n, double *scratch, hipStream_t s)
{
    return scan_generic<double>(in, out, n, scratch, 1, s);
}

// Weighted dust emission: package j takes the first cell whose inclusive
// cumulative weight exceeds x_j = (j + u) S / N (systematic sampling:
// every cell receives floor or ceil of N a_c / S packages).  In package
// units (capped expected counts) x_j = j + u, and positions at or past the
// total emit nothing.
__device__ inline void dust_select_body(const double *incl, int64_t ncells, uint64_t n_dust, double u_sys,
                                        int32_t package_units, int32_t *cell)
{
    const double S = incl[ncells - 1];
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_dust; j += (uint64_t)gridDim.x * blockDim.x) {
        const double x = package_units ? (double)j + u_sys : (((double)j + u_sys) * S) / (double)n_dust;
        if (package_units ? !(x < S) : !(S > 0.0)) {   // past the capped total, or nothing to emit
            cell[j] = -1;
            continue;
        }
        int64_t lo = 0, hi = ncells;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (incl[mid] > x) hi = mid; else lo = mid + 1;
        }
        if (lo >= ncells) {
            // rounding pushed x to S: take the last cell with L > 0
            lo = ncells - 1;
            while (lo > 0 && incl[lo - 1] == incl[ncells - 1]) --lo;
        }
        cell[j] = (int32_t)lo;
    }
}

__global__ void dust_select_kernel(const double *incl, int64_t ncells, uint64_t n_dust, double u_sys,
                                   int32_t package_units, int32_t *cell)
{
    dust_select_body(incl, ncells, n_dust, u_sys, package_units, cell);
}

hipError_t launch_dust_select(const double *incl, int64_t ncells, uint64_t n_dust, double u_sys, int32_t package_units,
                              int32_t *cell_out, hipStream_t s)
{
    if (n_dust == 0) return hipSuccess;
    uint64_t blocks = (n_dust + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(dust_select_kernel, dim3((unsigned)blocks), dim3(256), 0, s, incl, ncells, n_dust, u_sys,
                       package_units, cell_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ batched dust setup
// The same luminosity, inclusive cumulative sum and package cells for
// every frequency of a multi-frequency launch at once: blockIdx.y is the
// frequency's job, blockIdx.x the same block index as in the one-array
// kernels, so each row's values are those of the per-frequency path bit
// for bit.  The luminosity is written into the row and scanned in place.
__global__ void dust_luminosity_rows_kernel(const uint32_t *words, int64_t ncells, Levels lv, int32_t nlevels,
                                            double root_cell_cm, const DustJob *jobs)
{
    const DustJob &J = jobs[blockIdx.y];
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += (int64_t)gridDim.x * blockDim.x)
        J.incl[c] = cell_luminosity(words, c, lv, nlevels, root_cell_cm, J.nu, J.sigma_abs, J.w_nu, J.T);
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums_rows_kernel(const DustJob *jobs, int64_t n)
{
    __shared__ double sh[kScanThreads];
    const DustJob &J = jobs[blockIdx.y];
    tile_sums_body<double>(J.incl, n, J.sums, blockIdx.x, sh);
}

__global__ __launch_bounds__(kScanThreads) void scan_sums_exclusive_rows_kernel(const DustJob *jobs, int64_t m)
{
    sums_exclusive_body<double>(jobs[blockIdx.y].sums, m);
}

__global__ __launch_bounds__(kScanThreads) void scan_tiles_apply_rows_kernel(const DustJob *jobs, int64_t n)
{
    __shared__ double sh[kScanThreads];
    const DustJob &J = jobs[blockIdx.y];
    tiles_apply_body<double>(J.incl, n, J.sums, J.incl, 1, blockIdx.x, sh);
}

__global__ void dust_select_rows_kernel(const DustJob *jobs, int64_t ncells)
{
    const DustJob &J = jobs[blockIdx.y];
    dust_select_body(J.incl, ncells, J.n_dust, J.u_sys, 0, J.cell);
}

hipError_t launch_dust_setup_rows(const uint32_t *words, int64_t ncells, const int64_t *level_offset, int32_t nlevels,
                                  double root_cell_cm, const DustJob *d_jobs, int32_t njobs, uint64_t max_dust,
                                  hipStream_t s)
{
    if (njobs <= 0 || ncells <= 0) return hipSuccess;
    if (njobs > 65535) return hipErrorInvalidValue;
    Levels lv;
    for (int i = 0; i <= kMaxLevels; ++i) lv.off[i] = i <= nlevels ? level_offset[i] : ncells;
    // about 16 K workgroups in all, at least 64 per row
    const int64_t per_row = std::max<int64_t>(64, 16384 / njobs);
    const int64_t bl = std::min<int64_t>((ncells + 255) / 256, per_row);
    hipLaunchKernelGGL(dust_luminosity_rows_kernel, dim3((unsigned)bl, (unsigned)njobs), dim3(256), 0, s, words,
                       ncells, lv, nlevels, root_cell_cm, d_jobs);
    const int64_t tiles = (ncells + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tile_sums_rows_kernel, dim3((unsigned)tiles, (unsigned)njobs), dim3(kScanThreads), 0, s,
                       d_jobs, ncells);
    hipLaunchKernelGGL(scan_sums_exclusive_rows_kernel, dim3(1, (unsigned)njobs), dim3(kScanThreads), 0, s, d_jobs,
                       tiles);
    hipLaunchKernelGGL(scan_tiles_apply_rows_kernel, dim3((unsigned)tiles, (unsigned)njobs), dim3(kScanThreads), 0, s,
                       d_jobs, ncells);
    if (max_dust > 0) {
        const int64_t bs = std::min<int64_t>((int64_t)((max_dust + 255) / 256), per_row);
        hipLaunchKernelGGL(dust_select_rows_kernel, dim3((unsigned)bs, (unsigned)njobs), dim3(256), 0, s, d_jobs,
                           ncells);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ grid checks
// flags[0] |= 1: bad link (range, alignment, level); 2: bad density;
// 4: octet linked more or less than once.
__global__ void validate_grid_kernel(const uint32_t *words, int64_t ncells, Levels lv, int32_t nlevels,
                                     int64_t nroot, int32_t *parent, int32_t *octet_count, int32_t *flags)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += (int64_t)gridDim.x * blockDim.x) {
        const int32_t w = (int32_t)words[c];
        if (w < 0) {
            const int L = level_of(c, lv.off, nlevels);
            const int64_t first = -(int64_t)w;
            bool ok = L + 1 < nlevels;
            if (ok) {
                const int64_t a = lv.off[L + 1], b = lv.off[L + 2];
                ok = first >= a && first + 8 <= b && ((first - a) & 7) == 0;
            }
            if (!ok) {
                atomicOr(flags, 1);
            } else {
                const int64_t oct = (first - nroot) >> 3;
                atomicAdd(&octet_count[oct], 1);
                parent[oct] = (int32_t)c;
            }
        } else {
            const float v = __uint_as_float((uint32_t)w);
            if (!(v >= 0.0f) || !(v <= 3.4e38f)) atomicOr(flags, 2);
        }
    }
}

hipError_t launch_validate_grid(const uint32_t *words, int64_t ncells, const int64_t *level_offset,
                                int32_t nlevels, int64_t nroot, int32_t *parent, int32_t *octet_count,
                                int32_t *flags, hipStream_t s)
{
    Levels lv;
    for (int i = 0; i <= kMaxLevels; ++i) lv.off[i] = i <= nlevels ? level_offset[i] : ncells;
    int64_t blocks = (ncells + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(validate_grid_kernel, dim3((unsigned)blocks), dim3(256), 0, s, words, ncells, lv, nlevels,
                       nroot, parent, octet_count, flags);
    return hipGetLastError();
}

__global__ void check_octets_kernel(const int32_t *cnt, int64_t noct, int32_t *flags)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < noct; i += (int64_t)gridDim.x * blockDim.x)
        if (cnt[i] != 1) atomicOr(flags, 4);
}

hipError_t launch_check_octets(const int32_t *octet_count, int64_t noct, int32_t *flags, hipStream_t s)
{
    if (noct <= 0) return hipSuccess;
    int64_t blocks = (noct + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(check_octets_kernel, dim3((unsigned)blocks), dim3(256), 0, s, octet_count, noct, flags);
    return hipGetLastError();
}

// Leaf list: exclusive scan of the leaf flags, then scatter.
__global__ void leaf_flags_kernel(const uint32_t *words, int64_t n, int64_t *flag)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        flag[c] = (int32_t)words[c] >= 0 ? 1 : 0;
}

__global__ void leaf_scatter_kernel(const uint32_t *words, int64_t n, const int64_t *pos, int64_t *leaves)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        if ((int32_t)words[c] >= 0) leaves[pos[c]] = c;
}

hipError_t launch_leaf_list(const uint32_t *words, int64_t ncells, int64_t *scan_tmp, int64_t *scratch,
                            int64_t *leaves, hipStream_t s)
{
    int64_t blocks = (ncells + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(leaf_flags_kernel, dim3((unsigned)blocks), dim3(256), 0, s, words, ncells, leaves);
    hipError_t e = scan_generic<int64_t>(leaves, scan_tmp, ncells, scratch, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(leaf_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, s, words, ncells,
                       (const int64_t *)scan_tmp, leaves);
    return hipGetLastError();
}

}  // namespace soc
