// surrogate.hip -- device side of the learned starting temperatures.
//
// The paper shortens the iteration with a reference field (Sect. 2.1.2):
// the closer the field the dust iterations start from, the fewer of them
// are needed before the temperatures settle (Sect. 3.3).  Here a 3-D U-Net
// (unet.hip) predicts, on an S^3 grid of block averages, the part of
// log10 T that the dust re-emission adds to the temperatures T1 of the
// constant sources (the first iteration of the plain method, always run).
// Three streaming kernels surround the network:
//
//   features  n^3 cloud + T1 -> [S^3][4] network input
//   target    n^3 T, T1      -> [S^3] training target (block mean of
//                               log10 T/T1, divided by a fixed scale)
//   apply     [S^3] output, T1 -> n^3 start temperatures: the output is
//                               trilinearly interpolated to the fine cells
//                               (cell-centre convention) and applied to T1
//
// Features of a coarse cell (x, y, z), centre (x + 1/2, ...) in coarse
// units, cell edge s cm:
//   f0 = log10(sigma_V <n> s + 1e-4) / 2           optical depth of the cell
//   f1 = log10(1 + sum_p L_p / (4 pi d_p^2) / F_ext) / 4
//        bolometric flux of the unattenuated point sources against the
//        external field's 4 pi J
//   f2 = (log10 T_thin - 1.5) / 0.5, T_thin the equilibrium temperature of
//        dust in the unattenuated field: Gamma(T_thin) = 4 pi (J_bg,w +
//        sum_p Lw_p / (16 pi^2 d_p^2)), inverted in the temperature table
//   f3 = (<log10 max(T1, T_floor)> - 1.5) / 0.5
// with d_p^2 = (|r - r_p|^2 + 1/4) s^2 (softened at the source's cell),
// L_p = sum_k w_k L_p,k, Lw_p = sum_k w_k sigma_k L_p,k, J_bg,w = sum_k
// w_k sigma_k I_k, F_ext = 4 pi sum_k w_k I_k.  Empty cells count at
// T_floor in f3 and in the target.
#include <hip/hip_runtime.h>

#include "soc_kernels.h"

namespace soc {

namespace {

__device__ inline double sur_log10_T(uint32_t word, float T, double T_floor)
{
    const float n = __uint_as_float(word);
    const double t = n > 0.0f ? fmax((double)T, T_floor) : T_floor;
    return log10(t);
}

// ln T of the table entry where ln Gamma = ly (clamped to the table's ends).
__device__ inline double table_lnT(const double *lnG, int32_t nT, double lnTf, double dlnT, double ly)
{
    if (!(ly > lnG[0])) return lnTf;
    if (ly >= lnG[nT - 1]) return lnTf + dlnT * (nT - 1);
    int lo = 0, hi = nT - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (lnG[mid] <= ly) lo = mid; else hi = mid;
    }
    const double t = (ly - lnG[lo]) / (lnG[hi] - lnG[lo]);
    return lnTf + dlnT * ((double)lo + t);
}

__global__ __launch_bounds__(256) void sur_features_kernel(SurFeatArgs a)
{
    const int64_t S3 = (int64_t)a.S * a.S * a.S;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S3) return;
    const int x = (int)(i % a.S), y = (int)((i / a.S) % a.S), z = (int)(i / ((int64_t)a.S * a.S));
    const int b = a.b;
    const int64_t n = a.n;
    double rho = 0.0, lt = 0.0;
    for (int dz = 0; dz < b; ++dz)
        for (int dy = 0; dy < b; ++dy) {
            const int64_t row = ((int64_t)(z * b + dz) * n + (y * b + dy)) * n + (int64_t)x * b;
            for (int dx = 0; dx < b; ++dx) {
                const uint32_t w = a.words[row + dx];
                rho += (double)__uint_as_float(w);
                lt += sur_log10_T(w, a.T1[row + dx], a.T_floor);
            }
        }
    const double inv = 1.0 / ((double)b * b * b);
    rho *= inv;
    lt *= inv;
    const double cx = x + 0.5, cy = y + 0.5, cz = z + 0.5;
    double ratio = 0.0, Jw = a.Jbg;
    for (int p = 0; p < a.n_ps; ++p) {
        const double ex = cx - a.px[p], ey = cy - a.py[p], ez = cz - a.pz[p];
        const double d2 = (ex * ex + ey * ey + ez * ez + 0.25) * a.cell_cm * a.cell_cm;
        ratio += a.Lbol[p] / (12.566370614359172 * d2);
        Jw += a.Lw[p] / (157.91367041742973 * d2);   // 16 pi^2
    }
    ratio /= a.F_ext;
    const double lnT = table_lnT(a.lnG, a.nT, a.lnTf, a.dlnT, log(12.566370614359172 * Jw));
    float *o = a.out + 4 * i;
    o[0] = (float)(log10(a.sigma_v * rho * a.cell_cm + 1e-4) * 0.5);
    o[1] = (float)(log10(1.0 + ratio) * 0.25);
    o[2] = (float)((lnT * 0.43429448190325176 - 1.5) * 2.0);
    o[3] = (float)((lt - 1.5) * 2.0);
}

// log10 of the ratio a fine cell contributes to the target: temperatures
// with the floor convention, absorbed energies where the reference is > 0.
__device__ inline double sur_log_ratio(const SurMapArgs &a, int64_t c)
{
    const uint32_t w = a.words[c];
    if (a.absorbed) {
        const double A1 = a.A1[c], A = a.A[c];
        return (__uint_as_float(w) > 0.0f && A1 > 0.0 && A > 0.0) ? log10(A / A1) : 0.0;
    }
    return sur_log10_T(w, a.T[c], a.T_floor) - sur_log10_T(w, a.T1[c], a.T_floor);
}

__global__ __launch_bounds__(256) void sur_target_kernel(SurMapArgs a)
{
    const int64_t S3 = (int64_t)a.S * a.S * a.S;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S3) return;
    const int x = (int)(i % a.S), y = (int)((i / a.S) % a.S), z = (int)(i / ((int64_t)a.S * a.S));
    const int b = a.b;
    const int64_t n = a.n;
    double s = 0.0;
    for (int dz = 0; dz < b; ++dz)
        for (int dy = 0; dy < b; ++dy) {
            const int64_t row = ((int64_t)(z * b + dz) * n + (y * b + dy)) * n + (int64_t)x * b;
            for (int dx = 0; dx < b; ++dx) s += sur_log_ratio(a, row + dx);
        }
    a.coarse[i * a.stride + a.channel] = (float)(s / ((double)b * b * b) / a.scale);
}

// Interpolation weights along one axis, cell-centre convention: fine cell
// j of n maps to coarse coordinate (j + 1/2) S / n - 1/2, clamped to
// [0, S - 1].
__device__ inline void sur_axis(int j, int n, int S, int &i0, int &i1, float &t)
{
    float u = ((float)j + 0.5f) * (float)S / (float)n - 0.5f;
    u = fmaxf(u, 0.0f);
    i0 = min((int)u, S - 1);
    i1 = min(i0 + 1, S - 1);
    t = u - (float)i0;
}

__global__ __launch_bounds__(256) void sur_apply_kernel(SurMapArgs a)
{
    const int64_t n = a.n;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n * n * n) return;
    const uint32_t w = a.words[c];
    if (!(__uint_as_float(w) > 0.0f)) {
        if (a.absorbed) a.A_out[c] = 0.0;
        else a.T_out[c] = 0.0f;
        return;
    }
    const int x = (int)(c % n), y = (int)((c / n) % n), z = (int)(c / (n * n));
    int x0, x1, y0, y1, z0, z1;
    float tx, ty, tz;
    sur_axis(x, (int)n, a.S, x0, x1, tx);
    sur_axis(y, (int)n, a.S, y0, y1, ty);
    sur_axis(z, (int)n, a.S, z0, z1, tz);
    const int64_t S = a.S;
    auto at = [&](int zz, int yy, int xx) { return a.pred[(((int64_t)zz * S + yy) * S + xx) * a.stride + a.channel]; };
    const float c00 = at(z0, y0, x0) + tx * (at(z0, y0, x1) - at(z0, y0, x0));
    const float c01 = at(z0, y1, x0) + tx * (at(z0, y1, x1) - at(z0, y1, x0));
    const float c10 = at(z1, y0, x0) + tx * (at(z1, y0, x1) - at(z1, y0, x0));
    const float c11 = at(z1, y1, x0) + tx * (at(z1, y1, x1) - at(z1, y1, x0));
    const float c0 = c00 + ty * (c01 - c00), c1 = c10 + ty * (c11 - c10);
    const double lr = (double)(c0 + tz * (c1 - c0)) * a.scale + a.offset;
    if (a.absorbed) {
        a.A_out[c] = a.A1[c] * exp10(lr);
        return;
    }
    const double T1 = fmax((double)a.T1[c], a.T_floor);
    a.T_out[c] = (float)fmin(fmax(T1 * exp10(lr), a.T_floor), a.T_max);
}

}  // namespace

hipError_t launch_sur_features(const SurFeatArgs &a, hipStream_t s)
{
    const int64_t S3 = (int64_t)a.S * a.S * a.S;
    hipLaunchKernelGGL(sur_features_kernel, dim3((unsigned)((S3 + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sur_target(const SurMapArgs &a, hipStream_t s)
{
    const int64_t S3 = (int64_t)a.S * a.S * a.S;
    hipLaunchKernelGGL(sur_target_kernel, dim3((unsigned)((S3 + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sur_apply(const SurMapArgs &a, hipStream_t s)
{
    const int64_t n3 = (int64_t)a.n * a.n * a.n;
    hipLaunchKernelGGL(sur_apply_kernel, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace soc
