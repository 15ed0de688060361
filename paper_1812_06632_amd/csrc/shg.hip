// shg.hip -- temperature distributions and emission of stochastically heated
// grains (Sect. 2.1.1, Appendix B: the "thermal continuous" approximation,
// cooling only into the next lower enthalpy bin, solved by forward
// substitution in double precision).
//
// One wave per cell, all grain sizes in turn.  For size s the photon rates
// per grain r_k come from the cell's absorbed energy in each band; the
// upward rate from bin i to the bins >= j is the sum of r_k over photons
// whose target U_i + h nu_k lies at or above bin j, plus the share (linear
// in U) of those landing between bins j-1 and j.  With the photon energies
// increasing along k, each lane keeps a pointer per owned bin that only moves
// forward as j grows, over suffix sums of r_k.  The stationary populations
// follow from P_j L_j / (U_j - U_{j-1}) = sum_{i<j} P_i (upward rate from i
// to >= j), a wave-wide sum per bin.  Emission per Hz: 4 pi sigma_k
// sum_i P_i B_nu_k(T_i) per grain, times the grains of the cell.
#include <hip/hip_runtime.h>

#include "soc_kernels.h"

namespace soc {

__device__ inline double shg_planck(double nu, double T)
{
    const double h = 6.62607015e-27, k = 1.380649e-16, c = 2.99792458e10;
    const double x = h * nu / (k * T);
    const double pre = 2.0 * h * nu * nu * nu / (c * c);
    if (x > 700.0) return pre * exp(-x);
    return pre / expm1(x);
}

// Model tables: share[s][k], emit[s][i][k] = 4 pi sigma_sk B(nu_k, T_si),
// cool[s][i] = (4 pi sum_k sigma_sk B(nu_k, T_si) w_k) / (U_si - U_s,i-1).
__global__ void shg_prep_kernel(ShgModelDev m, const double *w)
{
    const double four_pi = 12.566370614359172;
    const int S = m.S, K = m.K, N = m.N;
    const int64_t n_emit = (int64_t)S * N * K;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_emit; t += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(t % K);
        const int i = (int)((t / K) % N);
        const int s = (int)(t / ((int64_t)K * N));
        m.emit[t] = four_pi * m.sigma[s * K + k] * shg_planck(m.nu[k], m.T[s * N + i]);
    }
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)S * N; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % N), s = (int)(t / N);
        double L = 0.0;
        for (int k = 0; k < K; ++k) L += four_pi * m.sigma[s * K + k] * shg_planck(m.nu[k], m.T[s * N + i]) * w[k];
        m.cool[t] = i > 0 ? L / (m.U[s * N + i] - m.U[s * N + i - 1]) : 0.0;
    }
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)K; t += (int64_t)gridDim.x * blockDim.x) {
        double tot = 0.0;
        for (int s = 0; s < S; ++s) tot += m.abundance[s] * m.sigma[s * K + t];
        for (int s = 0; s < S; ++s) m.share[s * K + t] = tot > 0.0 ? m.abundance[s] * m.sigma[s * K + t] / tot : 0.0;
    }
}

hipError_t launch_shg_prep(const ShgModelDev &m, const double *w, hipStream_t s)
{
    const int64_t work = (int64_t)m.S * m.N * m.K;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(shg_prep_kernel, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s, m, w);
    return hipGetLastError();
}

// LDS written by some lanes of a wave and read by others: order the
// accesses within the wave.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Bin of target t in grid U[0..N): m with U[m] <= t < U[m+1] and the share
// f of the upper bin; a target at or above the top goes wholly to the top.
__device__ inline int target_bin(const double *U, int N, double t, double &f)
{
    if (t >= U[N - 1]) {
        f = 1.0;
        return N - 2;
    }
    int lo = 0, hi = N - 1;   // U[lo] <= t < U[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (U[mid] <= t) lo = mid; else hi = mid;
    }
    f = (t - U[lo]) / (U[lo + 1] - U[lo]);
    return lo;
}

constexpr int kShgWaves = 4;   // waves (cells) per workgroup

__global__ __launch_bounds__(64 * kShgWaves) void shg_kernel(ShgArgs a)
{
    __shared__ double sh_r[kShgWaves][kShgMaxK];
    __shared__ double sh_sr[kShgWaves][kShgMaxK + 1];
    __shared__ double sh_U[kShgWaves][kShgMaxN];
    __shared__ double sh_P[kShgWaves][kShgMaxN];
    const ShgModelDev &m = a.model;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int K = m.K, N = m.N, S = m.S;
    double *r = sh_r[wv], *sr = sh_sr[wv], *U = sh_U[wv], *P = sh_P[wv];
    const int64_t nwaves = (int64_t)gridDim.x * kShgWaves;
    for (int64_t c = (int64_t)blockIdx.x * kShgWaves + wv; c < a.ncells; c += nwaves) {
        const uint32_t word = a.words[c];
        const float nf = __uint_as_float(word);
        double em[kShgMaxK / 64];
        for (int q = 0; q < kShgMaxK / 64; ++q) em[q] = 0.0;
        if ((int32_t)word >= 0 && nf > 0.0f) {
            int L = 0;
            while (L + 1 < a.nlevels && c >= a.level_offset[L + 1]) ++L;
            const double side = ldexp(a.root_cell_cm, -L);
            const double nHV = (double)nf * side * side * side;
            double Ak[kShgMaxK / 64];
            for (int q = 0; q < kShgMaxK / 64; ++q) {
                const int k = lane + 64 * q;
                Ak[q] = k < K ? a.absorbed[(int64_t)k * a.ncells + c] : 0.0;
            }
            for (int s = 0; s < S; ++s) {
                const double Ns = m.abundance[s] * nHV;
                for (int q = 0; q < kShgMaxK / 64; ++q) {
                    const int k = lane + 64 * q;
                    if (k < K) r[k] = Ns > 0.0 ? Ak[q] * m.share[s * K + k] * m.inv_hnu[k] / Ns : 0.0;
                }
                for (int i = lane; i < N; i += 64) U[i] = m.U[s * N + i];
                wave_sync();
                // suffix sums sr[k] = sum_{k' >= k} r[k'] (one lane; K is small)
                if (lane == 0) {
                    double acc = 0.0;
                    sr[K] = 0.0;
                    for (int k = K - 1; k >= 0; --k) {
                        acc += r[k];
                        sr[k] = acc;
                    }
                }
                wave_sync();
                // per owned bin i = lane + 64 q: pointer b (first photon whose
                // target bin is >= the current j)
                int b[kShgMaxN / 64];
                for (int q = 0; q < kShgMaxN / 64; ++q) b[q] = 0;
                double Pown[kShgMaxN / 64];
                for (int q = 0; q < kShgMaxN / 64; ++q) Pown[q] = lane + 64 * q == 0 ? 1.0 : 0.0;
                for (int j = 1; j < N; ++j) {
                    double contrib = 0.0;
                    for (int q = 0; q < kShgMaxN / 64; ++q) {
                        const int i = lane + 64 * q;
                        if (i >= j) continue;
                        double part = 0.0;
                        int bb = b[q];
                        while (bb < K) {
                            double f;
                            const int tm = target_bin(U, N, U[i] + m.hnu[bb], f);
                            if (tm >= j) break;
                            if (tm == j - 1) part += r[bb] * f;
                            ++bb;
                        }
                        b[q] = bb;
                        contrib += Pown[q] * (sr[bb] + part);
                    }
                    const double v = wave_sum(contrib);
                    double Pj = v / m.cool[s * N + j];
                    if (Pj > 1e200) {   // keep the unnormalised populations in range
                        for (int q = 0; q < kShgMaxN / 64; ++q) Pown[q] *= 1e-200;
                        Pj *= 1e-200;
                    }
                    if ((j & 63) == lane) Pown[j >> 6] = Pj;
                }
                double tot = 0.0;
                for (int q = 0; q < kShgMaxN / 64; ++q)
                    if (lane + 64 * q < N) tot += Pown[q];
                tot = wave_sum(tot);
                for (int q = 0; q < kShgMaxN / 64; ++q) {
                    const int i = lane + 64 * q;
                    if (i < N) {
                        const double pv = Pown[q] / tot;
                        P[i] = pv;
                        if (a.P) a.P[((int64_t)c * S + s) * N + i] = pv;
                    }
                }
                wave_sync();
                for (int q = 0; q < kShgMaxK / 64; ++q) {
                    const int k = lane + 64 * q;
                    if (k >= K) continue;
                    double acc = 0.0;
                    const double *e = m.emit + (int64_t)s * N * K + k;
                    for (int i = 0; i < N; ++i) acc += P[i] * e[(int64_t)i * K];
                    em[q] += Ns * acc;
                }
                wave_sync();
            }
        } else if (a.P) {
            for (int64_t t = lane; t < (int64_t)S * N; t += 64) a.P[(int64_t)c * S * N + t] = 0.0;
        }
        for (int q = 0; q < kShgMaxK / 64; ++q) {
            const int k = lane + 64 * q;
            if (k < K) a.emission[(int64_t)k * a.ncells + c] = em[q];
        }
    }
}

hipError_t launch_shg(const ShgArgs &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(shg_kernel, dim3((unsigned)blocks), dim3(64 * kShgWaves), 0, s, a);
    return hipGetLastError();
}

}  // namespace soc
