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

__global__ __launch_bounds__(kTempThreads) void temp_update_kernel(TempArgs a)
{
    extern __shared__ double lds_lnG[];
    for (int j = threadIdx.x; j < a.nT; j += blockDim.x) lds_lnG[j] = a.lnG[j];
    __syncthreads();
    const double G0 = lds_lnG[0], Gn = lds_lnG[a.nT - 1];
    const bool want = a.acc != nullptr;
    double cnt = 0.0, sumT = 0.0, sumrel = 0.0, nrel = 0.0, ncl = 0.0;
    const double hist_scale = (double)kHistBins / ((a.nT - 1) * a.dlnT);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncells; c += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t w = a.words[c];
        const float nf = __uint_as_float(w);
        float Tout = 0.0f;
        if ((int32_t)w >= 0 && nf > 0.0f) {
            const int L = level_index(c, a.level_offset, a.nlevels);
            const double s = ldexp(a.root_cell_cm, -L);
            const double y = a.absorbed[c] / ((double)nf * (s * s * s));
            double T;
            bool clamped = false;
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
                int b = (int)((log(Tf) - a.lnTf) * hist_scale);
                b = b < 0 ? 0 : (b >= kHistBins ? kHistBins - 1 : b);
                atomicAdd(&a.hist_n[b], 1u);
                unsafeAtomicAdd(&a.hist_T[b], Tf);
            }
        }
        a.T_new[c] = Tout;
    }
    if (want) {
        // wave reduction, then one atomic per wave
        for (int o = 32; o >= 1; o >>= 1) {
            cnt += __shfl_xor(cnt, o, 64);
            sumT += __shfl_xor(sumT, o, 64);
            sumrel += __shfl_xor(sumrel, o, 64);
            nrel += __shfl_xor(nrel, o, 64);
            ncl += __shfl_xor(ncl, o, 64);
        }
        if ((threadIdx.x & 63) == 0 && cnt > 0.0) {
            unsafeAtomicAdd(&a.acc[0], cnt);
            unsafeAtomicAdd(&a.acc[1], sumT);
            unsafeAtomicAdd(&a.acc[2], sumrel);
            unsafeAtomicAdd(&a.acc[3], nrel);
            unsafeAtomicAdd(&a.acc[4], ncl);
        }
    }
}

hipError_t launch_temp_update(const TempArgs &a, hipStream_t s)
{
    int64_t blocks = (a.ncells + kTempThreads - 1) / kTempThreads;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(temp_update_kernel, dim3((unsigned)blocks), dim3(kTempThreads), sizeof(double) * a.nT, s, a);
    return hipGetLastError();
}

// Hottest-5% mean from the histogram: chunks of bins from the top, a
// workgroup scan of chunk counts, then the chunk holding the k-th hottest
// cell resolves it bin by bin (the partial bin contributes its mean T).
constexpr int kFinThreads = 1024;
constexpr int kFinPer = kHistBins / kFinThreads;

__global__ __launch_bounds__(kFinThreads) void temp_finish_kernel(TempArgs a, double *out)
{
    __shared__ double sh_n[kFinThreads];
    __shared__ double sh_T[kFinThreads];
    const int t = threadIdx.x;
    // chunk t covers bins [top - (t+1)*per, top - t*per)
    const int hi = kHistBins - t * kFinPer;
    double n = 0.0, sT = 0.0;
    for (int b = hi - 1; b >= hi - kFinPer; --b) {
        n += (double)a.hist_n[b];
        sT += a.hist_T[b];
    }
    sh_n[t] = n;
    sh_T[t] = sT;
    __syncthreads();
    // inclusive scans from the top (Hillis-Steele)
    for (int o = 1; o < kFinThreads; o <<= 1) {
        const double an = t >= o ? sh_n[t - o] : 0.0;
        const double aT = t >= o ? sh_T[t - o] : 0.0;
        __syncthreads();
        sh_n[t] += an;
        sh_T[t] += aT;
        __syncthreads();
    }
    const double count = a.acc[0];
    const double k = ceil(0.05 * count);
    const double before_n = t > 0 ? sh_n[t - 1] : 0.0;
    const double before_T = t > 0 ? sh_T[t - 1] : 0.0;
    if (count > 0.0 && before_n < k && sh_n[t] >= k) {
        double cn = before_n, cT = before_T;
        for (int b = hi - 1; b >= hi - kFinPer; --b) {
            const double bn = (double)a.hist_n[b];
            if (cn + bn >= k) {
                cT += (k - cn) * (a.hist_T[b] / bn);
                break;
            }
            cn += bn;
            cT += a.hist_T[b];
        }
        out[1] = cT / k;
    }
    if (t == 0) {
        out[0] = count > 0.0 ? a.acc[1] / count : 0.0;
        out[2] = a.acc[3] > 0.0 ? a.acc[2] / a.acc[3] : __builtin_nan("");
        out[3] = a.acc[4];
        if (!(count > 0.0)) out[1] = 0.0;
    }
}

hipError_t launch_temp_finish(const TempArgs &a, double *out4, hipStream_t s)
{
    hipLaunchKernelGGL(temp_finish_kernel, dim3(1), dim3(kFinThreads), 0, s, a, out4);
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
