// temp_map.hip -- equilibrium dust temperature and emission maps
// (Juvela 2019, Sect. 2.1.1: separate kernels solve the dust temperature
// from the frequency-integrated absorbed energy and make surface-brightness
// maps from that solution).
//
// Temperature: Gamma(T) = 4 pi sum_k w_k sigma_abs,k B_nu_k(T) is tabulated
// once on a log-T grid; each cell inverts ln Gamma -> ln T by binary search
// in the table (staged in LDS) and linear interpolation in the log-log
// plane.  The pass is a streaming pass over the cells (A: 8 B, word: 4 B,
// T_old: 4 B, T_new: 4 B), bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include "soc_kernels.h"

namespace soc {

__device__ inline double planck_b(double nu, double T)
{
    const double h = 6.62607015e-27, k = 1.380649e-16, c = 2.99792458e10;
    if (!(T > 0.0)) return 0.0;
    const double x = h * nu / (k * T);
    const double pre = 2.0 * h * nu * nu * nu / (c * c);
    if (x > 700.0) return pre * exp(-x);
    return pre / expm1(x);
}

__global__ void temp_table_kernel(const double *nu, const double *w, const double *sabs, int32_t K, double lnTf,
                                  double dlnT, int32_t nT, double *lnG)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nT) return;
    const double T = exp(lnTf + dlnT * j);
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += w[k] * sabs[k] * planck_b(nu[k], T);
    lnG[j] = log(12.566370614359172 * s);
}

hipError_t launch_temp_table(const double *nu, const double *w, const double *sabs, int32_t K, double lnTf,
                             double dlnT, int32_t nT, double *lnG, hipStream_t s)
{
    hipLaunchKernelGGL(temp_table_kernel, dim3((nT + 255) / 256), dim3(256), 0, s, nu, w, sabs, K, lnTf, dlnT, nT, lnG);
    return hipGetLastError();
}

__device__ inline int level_index(int64_t c, const int64_t *lo, int32_t nlevels)
{
    int L = 0;
    while (L + 1 < nlevels && c >= lo[L + 1]) ++L;
    return L;
}

constexpr int kTempThreads = 256;

__device__ inline int coarse_bin(double lnT, double lnTf, double scale)
{
    int b = (int)((lnT - lnTf) * scale);
    return b < 0 ? 0 : (b >= kHistBins ? kHistBins - 1 : b);
}

// Temperature of every leaf (given: T_new already holds the temperatures
// and only the statistics are taken).  With statistics requested, each workgroup
// also writes its partial sums (count, sum T, sum |dT|/T_old, count with
// T_old > 0, clamped) and its histogram of ln T over kHistBins coarse bins
// (privatised in LDS) to its own row -- no global atomics, so the result
// is deterministic.
__global__ __launch_bounds__(kTempThreads) void temp_update_kernel(TempArgs a)
{
    extern __shared__ double lds_lnG[];
    __shared__ unsigned int sh_hist[kHistBins];
    __shared__ double sh_red[kTempThreads / 64][5];
    const bool want = a.part != nullptr;
    for (int j = threadIdx.x; j < a.nT; j += blockDim.x) lds_lnG[j] = a.lnG[j];
    if (want)
        for (int j = threadIdx.x; j < kHistBins; j += blockDim.x) sh_hist[j] = 0u;
    __syncthreads();
    const double G0 = lds_lnG[0], Gn = lds_lnG[a.nT - 1];
    double cnt = 0.0, sumT = 0.0, sumrel = 0.0, nrel = 0.0, ncl = 0.0;
    const double hist_scale = (double)kHistBins / ((a.nT - 1) * a.dlnT);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncells; c += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t w = a.words[c];
        const float nf = __uint_as_float(w);
        float Tout = 0.0f;
        if ((int32_t)w >= 0 && nf > 0.0f) {
            double T;
            bool clamped = false;
            if (a.given) {
                T = (double)a.T_new[c];
            } else {
                const int L = level_index(c, a.level_offset, a.nlevels);
                const double s = ldexp(a.root_cell_cm, -L);
                double y = a.absorbed[c] / ((double)nf * (s * s * s));
                if (a.ali_self) {
                    // diagonal ALI: the cell re-absorbs the fraction self/emitted of its own
                    // emission, so its emission is the absorption from elsewhere over the
                    // escape probability (kept >= 1e-6)
                    const double e = a.ali_emit[c];
                    const double esc = e > 0.0 ? fmax(1.0 - a.ali_self[c] / e, 1e-6) : 1.0;
                    y /= esc;
                }
                if (!(y > 0.0)) {
                    T = a.T_floor;
                    clamped = true;
                } else {
                    const double ly = log(y);
                    if (!(ly > G0)) {
                        T = a.T_floor;
                        clamped = true;
                    } else if (ly >= Gn) {
                        T = a.T_max;
                        clamped = true;
                    } else {
                        int lo = 0, hi = a.nT - 1;   // lnG[lo] < ly < lnG[hi]
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (lds_lnG[mid] <= ly) lo = mid; else hi = mid;
                        }
                        const double t = (ly - lds_lnG[lo]) / (lds_lnG[hi] - lds_lnG[lo]);
                        T = exp(a.lnTf + a.dlnT * ((double)lo + t));
                    }
                }
            }
            Tout = (float)T;
            if (want) {
                const double Tf = (double)Tout;
                cnt += 1.0;
                sumT += Tf;
                ncl += clamped ? 1.0 : 0.0;
                if (a.T_old) {
                    const float To = a.T_old[c];
                    if (To > 0.0f) {
                        sumrel += fabs(Tf - (double)To) / (double)To;
                        nrel += 1.0;
                    }
                }
                atomicAdd(&sh_hist[coarse_bin(log(fmax(Tf, 1e-30)), a.lnTf, hist_scale)], 1u);
            }
        }
        if (!a.given) a.T_new[c] = Tout;
    }
    if (!want) return;
    for (int o = 32; o >= 1; o >>= 1) {
        cnt += __shfl_xor(cnt, o, 64);
        sumT += __shfl_xor(sumT, o, 64);
        sumrel += __shfl_xor(sumrel, o, 64);
        nrel += __shfl_xor(nrel, o, 64);
        ncl += __shfl_xor(ncl, o, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh_red[wv][0] = cnt;
        sh_red[wv][1] = sumT;
        sh_red[wv][2] = sumrel;
        sh_red[wv][3] = nrel;
        sh_red[wv][4] = ncl;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double v = 0.0;
        for (int k = 0; k < kTempThreads / 64; ++k) v += sh_red[k][threadIdx.x];
        a.part[(int64_t)blockIdx.x * 8 + threadIdx.x] = v;
    }
    for (int j = threadIdx.x; j < kHistBins; j += blockDim.x) a.hist_part[(int64_t)blockIdx.x * kHistBins + j] = sh_hist[j];
}

hipError_t launch_temp_update(const TempArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(temp_update_kernel, dim3((unsigned)a.blocks), dim3(kTempThreads), sizeof(double) * a.nT, s, a);
    return hipGetLastError();
}

// Reduce the per-workgroup partial sums and histograms, then locate the
// coarse bin holding the k-th hottest leaf (k = ceil(0.05 n)).
// meta: [0] count [1] sum T [2] sum rel [3] n rel [4] clamped
//       [5] threshold bin [6] cells still needed from that bin [7] k
constexpr int kFinThreads = 1024;
constexpr int kFinPer = kHistBins / kFinThreads;

__global__ __launch_bounds__(kFinThreads) void temp_stats_reduce_kernel(TempArgs a)
{
    __shared__ double sh_n[kFinThreads];
    __shared__ double sh_p[8];
    const int t = threadIdx.x;
    if (t < 5) {
        double v = 0.0;
        for (int b = 0; b < a.blocks; ++b) v += a.part[(int64_t)b * 8 + t];
        sh_p[t] = v;
    }
    // chunk t covers bins [hi - per, hi), counted from the top
    const int hi = kHistBins - t * kFinPer;
    double loc[kFinPer];
    double n = 0.0;
    for (int q = 0; q < kFinPer; ++q) {
        loc[q] = (double)a.hist_total[hi - 1 - q];
        n += loc[q];
    }
    sh_n[t] = n;
    __syncthreads();
    for (int o = 1; o < kFinThreads; o <<= 1) {
        const double add = t >= o ? sh_n[t - o] : 0.0;
        __syncthreads();
        sh_n[t] += add;
        __syncthreads();
    }
    const double count = sh_p[0];
    const double k = ceil(0.05 * count);
    const double before = t > 0 ? sh_n[t - 1] : 0.0;
    if (count > 0.0 && before < k && sh_n[t] >= k) {
        double cn = before;
        for (int q = 0; q < kFinPer; ++q) {
            if (cn + loc[q] >= k) {
                a.meta[5] = (double)(hi - 1 - q);
                a.meta[6] = k - cn;
                break;
            }
            cn += loc[q];
        }
    }
    if (t < 5) a.meta[t] = sh_p[t];
    if (t == 0) {
        a.meta[7] = k;
        if (!(count > 0.0)) {
            a.meta[5] = (double)kHistBins;
            a.meta[6] = 0.0;
        }
    }
}

// Second pass over the temperatures: exact sum of T above the threshold
// bin (per-workgroup partials) and a fine histogram (counts and sums) of
// the cells inside it, which are few.
__global__ __launch_bounds__(kTempThreads) void temp_stats_refine_kernel(TempArgs a)
{
    __shared__ double sh[kTempThreads / 64];
    const int tb = (int)a.meta[5];
    const double hist_scale = (double)kHistBins / ((a.nT - 1) * a.dlnT);
    const double lo_b = a.lnTf + (double)tb / hist_scale;
    const double fine_scale = hist_scale * (double)kHistBins;
    double above = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncells; c += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t w = a.words[c];
        if ((int32_t)w < 0 || !(__uint_as_float(w) > 0.0f)) continue;
        const double Tf = (double)a.T_new[c];
        const double lt = log(fmax(Tf, 1e-30));   // a given field may hold zeros
        const int b = coarse_bin(lt, a.lnTf, hist_scale);
        if (b > tb) {
            above += Tf;
        } else if (b == tb) {
            int f = (int)((lt - lo_b) * fine_scale);
            f = f < 0 ? 0 : (f >= kHistBins ? kHistBins - 1 : f);
            atomicAdd(&a.fine_n[f], 1u);
            unsafeAtomicAdd(&a.fine_T[f], Tf);
        }
    }
    for (int o = 32; o >= 1; o >>= 1) above += __shfl_xor(above, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = above;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int k = 0; k < kTempThreads / 64; ++k) v += sh[k];
        a.part[(int64_t)blockIdx.x * 8 + 5] = v;
    }
}

// Final statistics: mean T, hottest-5% mean (cells above the threshold bin
// plus the hottest cells inside it, resolved on the fine histogram whose
// bins are 2^-24 of the ln T range wide), mean relative change, clamps.
__global__ __launch_bounds__(kFinThreads) void temp_stats_finish_kernel(TempArgs a, double *out)
{
    __shared__ double sh_n[kFinThreads];
    __shared__ double sh_T[kFinThreads];
    __shared__ double sh_above;
    const int t = threadIdx.x;
    if (t == 0) {
        double v = 0.0;
        for (int b = 0; b < a.blocks; ++b) v += a.part[(int64_t)b * 8 + 5];
        sh_above = v;
    }
    const int hi = kHistBins - t * kFinPer;
    double n = 0.0, sT = 0.0;
    for (int b = hi - 1; b >= hi - kFinPer; --b) {
        n += (double)a.fine_n[b];
        sT += a.fine_T[b];
    }
    sh_n[t] = n;
    sh_T[t] = sT;
    __syncthreads();
    for (int o = 1; o < kFinThreads; o <<= 1) {
        const double an = t >= o ? sh_n[t - o] : 0.0;
        const double aT = t >= o ? sh_T[t - o] : 0.0;
        __syncthreads();
        sh_n[t] += an;
        sh_T[t] += aT;
        __syncthreads();
    }
    const double count = a.meta[0];
    const double need = a.meta[6];
    const double k = a.meta[7];
    const double before_n = t > 0 ? sh_n[t - 1] : 0.0;
    const double before_T = t > 0 ? sh_T[t - 1] : 0.0;
    if (count > 0.0 && need > 0.0 && before_n < need && sh_n[t] >= need) {
        double cn = before_n, cT = before_T;
        for (int b = hi - 1; b >= hi - kFinPer; --b) {
            const double bn = (double)a.fine_n[b];
            if (cn + bn >= need) {
                cT += (need - cn) * (a.fine_T[b] / bn);
                break;
            }
            cn += bn;
            cT += a.fine_T[b];
        }
        out[1] = (sh_above + cT) / k;
    }
    if (t == 0) {
        out[0] = count > 0.0 ? a.meta[1] / count : 0.0;
        out[2] = a.meta[3] > 0.0 ? a.meta[2] / a.meta[3] : __builtin_nan("");
        out[3] = a.meta[4];
        if (!(count > 0.0)) out[1] = 0.0;
        else if (!(need > 0.0)) out[1] = sh_above / k;
    }
}

// Sum of the per-workgroup histograms, one bin per thread (coalesced).
__global__ __launch_bounds__(256) void temp_hist_reduce_kernel(TempArgs a)
{
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    if (bin >= kHistBins) return;
    unsigned int sum = 0;
    for (int b = 0; b < a.blocks; ++b) sum += a.hist_part[(int64_t)b * kHistBins + bin];
    a.hist_total[bin] = sum;
}

hipError_t launch_temp_stats(const TempArgs &a, double *out4, hipStream_t s)
{
    hipLaunchKernelGGL(temp_hist_reduce_kernel, dim3(kHistBins / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(temp_stats_reduce_kernel, dim3(1), dim3(kFinThreads), 0, s, a);
    hipLaunchKernelGGL(temp_stats_refine_kernel, dim3((unsigned)a.blocks), dim3(kTempThreads), 0, s, a);
    hipLaunchKernelGGL(temp_stats_finish_kernel, dim3(1), dim3(kFinThreads), 0, s, a, out4);
    return hipGetLastError();
}

// ------------------------------------------------------------------ map
// One thread per pixel (pixel = finest cell).  The ray runs along the axis
// from the observer side; each leaf on it adds S (1 - e^{-dtau}) e^{-tau},
// S = (sigma_abs / sigma_ext) B_nu(T), accumulated in FP64.
__device__ inline int64_t leaf_lookup(const uint32_t *words, int32_t nx, int32_t ny, double px, double py, double pz,
                                      double &lox, double &loy, double &loz, double &size)
{
    const int64_t ix = (int64_t)floor(px), iy = (int64_t)floor(py), iz = (int64_t)floor(pz);
    int64_t c = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
    lox = (double)ix; loy = (double)iy; loz = (double)iz; size = 1.0;
    int32_t w = (int32_t)words[c];
    while (w < 0) {
        const int64_t first = -(int64_t)w;
        size *= 0.5;
        const int ox = px >= lox + size, oy = py >= loy + size, oz = pz >= loz + size;
        lox += ox * size; loy += oy * size; loz += oz * size;
        c = first + ox + 2 * oy + 4 * oz;
        w = (int32_t)words[c];
    }
    return c;
}

__global__ void map_kernel(MapArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= a.npx || j >= a.npy) return;
    const int ax = a.axis;
    const int bx = ax == 0 ? 1 : 0, cx = ax == 2 ? 1 : 2;
    const int32_t N[3] = {a.nx, a.ny, a.nz};
    const double psz = ldexp(1.0, -(a.nlevels - 1));
    double p[3];
    p[bx] = (i + 0.5) * psz;
    p[cx] = (j + 0.5) * psz;
    const double Na = (double)N[ax];
    double x = a.neg ? 0.0 : Na;
    double I = 0.0, tau = 0.0;
    const double half = 0.5 * ldexp(1.0, -(a.nlevels + 1));   // quarter of the finest cell
    if (a.sigma_ext > 0.0) {
        while (a.neg ? (x < Na) : (x > 0.0)) {
            p[ax] = a.neg ? x + half : x - half;
            double lo[3], size;
            const int64_t c = leaf_lookup(a.words, a.nx, a.ny, p[0], p[1], p[2], lo[0], lo[1], lo[2], size);
            const double xn = a.neg ? lo[ax] + size : lo[ax];
            const double ds = fabs(xn - x);
            const float nf = __uint_as_float(a.words[c]);
            if (nf > 0.0f) {
                const double dt = a.sigma_ext * (double)nf * ds * a.root_cell_cm;
                const double S = (a.sigma_abs / a.sigma_ext) * planck_b(a.nu, (double)a.T[c]);
                I += S * (-expm1(-dt)) * exp(-tau);
                tau += dt;
            }
            x = xn;
        }
    }
    a.image[(int64_t)j * a.npx + i] = (float)I;
}

hipError_t launch_map(const MapArgs &a, hipStream_t s)
{
    dim3 block(64), grid((a.npx + 63) / 64, a.npy);
    hipLaunchKernelGGL(map_kernel, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace soc
