// shg.hip -- temperature distributions and emission of stochastically heated
// grains (Sect. 2.1.1, Appendix A: the "thermal continuous" approximation,
// cooling only into the next lower enthalpy bin, solved by forward
// substitution in double precision).
//
// For size s the photon rates per grain r_k come from a cell's absorbed
// energy in each band.  A photon k absorbed in bin i lands between the two
// bins around U_i + h nu_k, split linearly in U, so the upward rate from bin
// i to the bins >= j is
//     up[j][i] = sum_{k: target >= j} r_k + sum_{k: target in [j-1, j)} r_k f_ik.
// With the photon energies increasing along k, the first sum is a suffix sum
// sr[ks(i, j)] of r over the photons k >= ks(i, j), and the second runs over
// the photons between ks(i, j-1) and ks(i, j), f_ik = (U_i + h nu_k -
// U_{j-1}) / (U_j - U_{j-1}); ks depends only on the model and is tabulated.
// Most photons of a bin land in the bin itself or the next one (j = i + 1):
// up[i+1][i] = sum_k r_k min(U_i + h nu_k - U_i, U_{i+1} - U_i) / (U_{i+1} -
// U_i) is formed for all bins before the serial part; the later ranges hold
// a few photons at most.  No photon reaches beyond a band of bins above its
// own (the largest photon energy), so bins further below j are skipped.  The
// stationary populations follow from
//     P_j L(T_j) / (U_j - U_{j-1}) = sum_{i<j} P_i up[j][i],
// one bin after the other.  Emission per Hz: 4 pi sigma_k sum_i P_i B_nu_k(T_i)
// per grain, times the grains of the cell.
//
// Layout on the GPU: one wave solves G cells at once, L = 64 / G lanes per
// cell, lane l of a cell owning the bins i = l + L m.  The serial step j is
// a sum over the owned bins and a reduction over the cell's L lanes (DPP,
// no LDS); the step's new population stays in the register of its owner.
// Everything a step reads sits in LDS: the size's ks table, enthalpies,
// inverse bin widths and cooling rates (shared by the workgroup, whose waves
// go through the sizes together), and per cell the rates r and their suffix
// sums.  Afterwards the cell's LDS holds the G cells' grain populations
// N_s P_i, which the wave multiplies with the size's emission table (lanes
// along frequency), so the table is read once per G cells.
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
// icool[s][i] = (U_si - U_s,i-1) / (4 pi sum_k sigma_sk B(nu_k, T_si) w_k),
// idu[s][i] = 1 / (U_si - U_s,i-1), ks[s][j][i].
__global__ void shg_prep_kernel(ShgModelDev m, const double *w)
{
    const double four_pi = 12.566370614359172;
    const int S = m.S, K = m.K, N = m.N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_emit = (int64_t)S * N * K;
    for (int64_t t = t0; t < n_emit; t += stride) {
        const int k = (int)(t % K);
        const int i = (int)((t / K) % N);
        const int s = (int)(t / ((int64_t)K * N));
        m.emit[t] = four_pi * m.sigma[s * K + k] * shg_planck(m.nu[k], m.T[s * N + i]);
    }
    for (int64_t t = t0; t < (int64_t)S * N; t += stride) {
        const int i = (int)(t % N), s = (int)(t / N);
        double L = 0.0;
        for (int k = 0; k < K; ++k) L += four_pi * m.sigma[s * K + k] * shg_planck(m.nu[k], m.T[s * N + i]) * w[k];
        m.icool[t] = i > 0 ? (m.U[s * N + i] - m.U[s * N + i - 1]) / L : 0.0;
    }
    for (int64_t t = t0; t < (int64_t)K; t += stride) {
        double tot = 0.0;
        for (int s = 0; s < S; ++s) tot += m.abundance[s] * m.sigma[s * K + t];
        for (int s = 0; s < S; ++s) m.share[s * K + t] = tot > 0.0 ? m.abundance[s] * m.sigma[s * K + t] / tot : 0.0;
    }
    for (int64_t t = t0; t < (int64_t)S * N; t += stride) {
        const int i = (int)(t % N);
        m.idu[t] = i > 0 ? 1.0 / (m.U[t] - m.U[t - 1]) : 0.0;
    }
    // ks[s][j][i]: the photons of bin i whose lower target bin lies below j.
    // The lower target bin of U_i + h nu_k is the last lo <= N-2 with U_lo <=
    // U_i + h nu_k (at or above the top bin, all of it goes to the top bin),
    // so lo >= j  <=>  U_j <= U_i + h nu_k for j <= N-2, and lo never reaches N-1
    const int ksz = shg_ks_stride(N);
    for (int64_t t = t0; t < (int64_t)S * ksz; t += stride) {
        const int s = (int)(t / ksz);
        const int ij = (int)(t % ksz);
        const int i = ij % N, j = ij / N;
        int n = 0;
        if (j >= N) {   // padding
        } else if (j == N - 1) {
            n = K;
        } else {
            const double *U = m.U + (int64_t)s * N;
            while (n < K && U[i] + m.hnu[n] < U[j]) ++n;
        }
        m.ks[t] = (uint8_t)n;
    }
}

// band[s]: 2 + the largest number of bins a photon can lift a grain of size
// s (to the lower of its two target bins), so that the upward rate from bin i
// to the bins >= j is exactly 0 once j - i >= band
__global__ void shg_band_kernel(ShgModelDev m)
{
    const int N = m.N;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < m.S; s += gridDim.x * blockDim.x) {
        const double *U = m.U + (int64_t)s * N;
        int jump = 0;
        for (int i = 0; i < N - 1; ++i) {
            const double x = U[i] + m.hnu[m.K - 1];
            int lo = i;
            while (lo + 1 < N - 1 && U[lo + 1] <= x) ++lo;
            if (lo - i > jump) jump = lo - i;
        }
        m.band[s] = jump + 2;
    }
}

hipError_t launch_shg_prep(const ShgModelDev &m, const double *w, hipStream_t s)
{
    const int64_t work = (int64_t)m.S * m.N * (m.K > m.N ? m.K : m.N);
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(shg_prep_kernel, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s, m, w);
    hipLaunchKernelGGL(shg_band_kernel, dim3((unsigned)((m.S + 63) / 64)), dim3(64), 0, s, m);
    return hipGetLastError();
}

// LDS written by some lanes of a wave and read by others: order the
// accesses within the wave.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Lane permutation of a double through DPP (all 64 lanes active).
template <int Ctrl>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), Ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), Ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over each aligned group of L lanes, the result in every lane of it.
template <int L>
__device__ inline double group_sum(double v)
{
    static_assert(L == 8 || L == 16 || L == 32, "groups of 8, 16 or 32 lanes");
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_f64<0x141>(v);   // row_half_mirror: the other quad of the 8
    if (L >= 16) v += dpp_f64<0x140>(v);   // row_mirror: the other 8 of the 16
    if (L == 32) v += __shfl_xor(v, 16, 64);
    return v;
}

// H atoms in a cell (n_H V); 0 outside the grid, for refined parents and
// empty cells.
__device__ inline double cell_nhv(const ShgArgs &a, int64_t cell)
{
    if (cell >= a.ncells) return 0.0;
    const uint32_t word = a.words[cell];
    const float nf = __uint_as_float(word);
    if ((int32_t)word < 0 || !(nf > 0.0f)) return 0.0;
    int lv = 0;
    while (lv + 1 < a.nlevels && cell >= a.level_offset[lv + 1]) ++lv;
    const double side = ldexp(a.root_cell_cm, -lv);
    return (double)nf * side * side * side;
}

constexpr int kShgWaves = 4;   // waves per workgroup, each on its own tiles

__host__ __device__ inline int shg_cell_stride(int K, int N)
{
    const int n = 2 * K + 1 > N ? 2 * K + 1 : N;
    return n | 1;   // odd, so that the cells of a wave start in different LDS banks
}

// Photons k in [k0, k1) of bin i (enthalpy Ui), all with lower target bin
// j - 1: sum of r_k (U_i + h nu_k - U_{j-1}), the numerator of their shares f
// of bin j, each at most the bin width dU (photons at or above the top bin go
// wholly to it).  Two photons per pass so that their reads overlap.
__device__ inline double range_sum(const double *r, const double *E, double Ui, double Ulo, double dU, int k0, int k1)
{
    double part = 0.0;
    for (int k = k0; k < k1; k += 2) {
        const int kn = k + 1 < k1 ? k + 1 : k;
        const double d0 = fmin(Ui + E[k] - Ulo, dU), d1 = fmin(Ui + E[kn] - Ulo, dU);
        const double r0 = r[k], r1 = k + 1 < k1 ? r[kn] : 0.0;
        part += r0 * d0;
        part += r1 * d1;
    }
    return part;
}

template <int G>
__global__ __launch_bounds__(64 * kShgWaves, 3) void shg_kernel(ShgArgs a)
{
    constexpr int L = 64 / G;              // lanes per cell
    constexpr int M = kShgMaxN / L;        // bins per lane at most
    extern __shared__ double lds[];
    const ShgModelDev &m = a.model;
    const int K = m.K, N = m.N, S = m.S;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cg = lane / L, l = lane % L;   // this lane's cell in the tile, its place among the cell's lanes
    const int cr = lane % G;                 // cell whose rates this lane forms
    const int cs = shg_cell_stride(K, N);
    const int ksz = shg_ks_stride(N);
    double *const W = lds + (size_t)wv * G * (cs + K);
    double *const rc = W + cg * cs;          // r[0..K-1], sr[K..2K] of this lane's cell; later N_s P_i
    double *const EM = W + G * cs;           // emission of the tile summed over sizes, [k][G]
    // tables of the current size, shared by the workgroup
    double *const Us = lds + (size_t)kShgWaves * G * (cs + K);   // U_i
    double *const Idu = Us + N;                                   // 1 / (U_i - U_{i-1})
    double *const Ic = Idu + N;                                   // (U_i - U_{i-1}) / L(T_i)
    double *const Eh = Ic + N;                                    // h nu_k
    uint8_t *const KS = (uint8_t *)(Eh + K);                       // ks[j][i]
    const int64_t ntiles = (a.ncells + G - 1) / G;
    const int64_t ngroups = (ntiles + kShgWaves - 1) / kShgWaves;
    // the workgroup's waves take consecutive tiles and go through the sizes
    // together; a tile past the end holds no cells
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int64_t c0 = (grp * kShgWaves + wv) * G;
        const int64_t cell = c0 + cg;
        const double nhv = cell_nhv(a, cell);
        const double nhv_r = cell_nhv(a, c0 + cr);
        for (int t = lane; t < G * K; t += 64) EM[t] = 0.0;
        for (int s = 0; s < S; ++s) {
            const int band = m.band[s];
            __syncthreads();   // every wave is done with the previous size's tables
            {
                const uint4 *src = (const uint4 *)(m.ks + (int64_t)s * ksz);
                uint4 *dst = (uint4 *)KS;
                for (int t = threadIdx.x; t < ksz / 16; t += 64 * kShgWaves) dst[t] = src[t];
                for (int t = threadIdx.x; t < N; t += 64 * kShgWaves) {
                    Us[t] = m.U[(int64_t)s * N + t];
                    Idu[t] = m.idu[(int64_t)s * N + t];
                    Ic[t] = m.icool[(int64_t)s * N + t];
                }
                for (int t = threadIdx.x; t < K; t += 64 * kShgWaves) Eh[t] = m.hnu[t];
            }
            // photon rates per grain, lanes over (cell, k) with cells fastest
            {
                const double ns_r = m.abundance[s] * nhv_r;
                double *rr = W + cr * cs;
                for (int t = lane; t < G * K; t += 64) {
                    const int k = t / G;
                    rr[k] = ns_r > 0.0 ? a.absorbed[(int64_t)k * a.ncells + c0 + cr] * m.share[s * K + k] * m.inv_hnu[k] / ns_r
                                       : 0.0;
                }
            }
            __syncthreads();
            if (lane < G) {   // suffix sums sr[k] = sum_{k' >= k} r[k'], one lane per cell
                double *x = W + lane * cs;
                double acc = 0.0;
                x[2 * K] = 0.0;
                for (int k = K - 1; k >= 0; --k) {
                    acc += x[k];
                    x[K + k] = acc;
                }
            }
            // owned bins: populations, up[i+1][i], and where the next photon range starts
            double P[M], up1[M];
            int b[M];
            {
                double Ui[M], dU[M];
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    const int i = l + L * q;
                    P[q] = i == 0 ? 1.0 : 0.0;
                    const int ic = i < N - 1 ? i : N - 2;
                    Ui[q] = Us[ic];
                    dU[q] = Us[ic + 1] - Us[ic];
                    up1[q] = 0.0;
                }
                for (int k = 0; k < K; ++k) {
                    const double rk = rc[k], ek = Eh[k];
#pragma unroll
                    for (int q = 0; q < M; ++q) up1[q] += rk * fmin(Ui[q] + ek - Ui[q], dU[q]);
                }
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const int i = l + L * q;
                b[q] = i < N - 1 ? KS[(i + 1) * N + i] : 0;
                up1[q] *= i < N - 1 ? Idu[i + 1] : 0.0;
            }
            // forward substitution over the bins, block mb of L steps sets bin l + L mb of every lane
#pragma unroll
            for (int mb = 0; mb < M; ++mb) {
                if (L * mb >= N) break;
#pragma unroll 1
                for (int jl = 0; jl < L; ++jl) {
                    const int j = L * mb + jl;
                    if (j >= N) break;
                    if (j == 0) continue;
                    const uint8_t *ksj = KS + j * N;
                    const double ic = Ic[j], idu = Idu[j], ulo = Us[j - 1], du = Us[j] - Us[j - 1];
                    const int jb = j - band;   // no photon of a bin <= jb reaches j
                    double contrib = 0.0;
#pragma unroll
                    for (int q = 0; q <= mb; ++q) {
                        if (L * q + L - 1 <= jb) continue;
                        const int i = l + L * q;
                        // bins below j - 1 take the next photon range; only the
                        // last two blocks hold bins >= j - 1
                        const int kb = q + 1 < mb || i < j - 1 ? ksj[i] : b[q];
                        double up = rc[K + kb];
                        if (kb > b[q]) up += range_sum(rc, Eh, Us[i], ulo, du, b[q], kb) * idu;
                        b[q] = kb;
                        if (q + 1 >= mb && i == j - 1) up = up1[q];
                        contrib += P[q] * up;   // P is 0 for the bins >= j
                    }
                    double Pj = group_sum<L>(contrib) * ic;
                    if (Pj > 1e200) {   // keep the unnormalised populations in range
#pragma unroll
                        for (int q = 0; q < M; ++q) P[q] *= 1e-200;
                        Pj *= 1e-200;
                    }
                    if (l == jl) P[mb] = Pj;
                }
            }
            double tot = 0.0;
#pragma unroll
            for (int q = 0; q < M; ++q)
                if (l + L * q < N) tot += P[q];
            tot = group_sum<L>(tot);
            const double scale = m.abundance[s] * nhv / tot;   // the tile holds grains per bin: N_s P_i
            wave_sync();
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const int i = l + L * q;
                if (i < N) {
                    rc[i] = P[q] * scale;
                    if (a.P && cell < a.ncells) a.P[((int64_t)cell * S + s) * N + i] = nhv > 0.0 ? P[q] / tot : 0.0;
                }
            }
            wave_sync();
            // emission of the tile at this size: EM[k][c] += sum_i (N_s P_i)[c] emit[s][i][k]
            const double *e = m.emit + (int64_t)s * N * K;
            for (int k = lane; k < K; k += 64) {
                double em[G];
#pragma unroll
                for (int c = 0; c < G; ++c) em[c] = 0.0;
                for (int i = 0; i < N; ++i) {
                    const double ev = e[i * K + k];
#pragma unroll
                    for (int c = 0; c < G; ++c) em[c] += W[c * cs + i] * ev;
                }
#pragma unroll
                for (int c = 0; c < G; ++c) EM[k * G + c] += em[c];
            }
            wave_sync();
        }
        // stores run along cells
        for (int t = lane; t < G * K; t += 64) {
            const int c = t % G, k = t / G;
            if (c0 + c < a.ncells) a.emission[(int64_t)k * a.ncells + c0 + c] = EM[t];
        }
        wave_sync();
    }
}

#ifndef SOC_SHG_CELLS_PER_WAVE
#define SOC_SHG_CELLS_PER_WAVE 4
#endif
constexpr int kShgG = SOC_SHG_CELLS_PER_WAVE;

size_t shg_lds_bytes(int K, int N)
{
    return sizeof(double) * ((size_t)kShgWaves * kShgG * (shg_cell_stride(K, N) + K) + 3 * (size_t)N + K) +
           (size_t)shg_ks_stride(N);
}

int64_t shg_blocks(int64_t ncells)
{
    const int64_t tiles = (ncells + kShgG - 1) / kShgG;
    int64_t blocks = (tiles + kShgWaves - 1) / kShgWaves;   // one group of tiles per workgroup
    if (blocks > 16384) blocks = 16384;   // grid-stride beyond
    return blocks < 1 ? 1 : blocks;
}

hipError_t launch_shg(const ShgArgs &a, hipStream_t s)
{
    const size_t lds_bytes = shg_lds_bytes(a.model.K, a.model.N);
    if (lds_bytes > 65536) {   // above the default dynamic LDS limit (160 KB per CU)
        const hipError_t e = hipFuncSetAttribute((const void *)shg_kernel<kShgG>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(shg_kernel<kShgG>, dim3((unsigned)shg_blocks(a.ncells)), dim3(64 * kShgWaves), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace soc
