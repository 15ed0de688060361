// peel.hip -- images of scattered light (Sect. 2.1.1: separate runs with
// forced first scattering and peel-off).
//
// Packages of the external field and the point sources are traced with the
// production emission and step code.  At every scattering the package of
// weight W at position r, moving along u, sends W Phi(u.o) exp(-tau_ext) to
// the distant observer in direction o: Phi the normalised Henyey-Greenstein
// function, tau_ext the extinction optical depth from r to the boundary
// along o (a ray march with the same step code), added to the pixel under r.
// With forced first scattering a package first measures the scattering
// optical depth tau_esc ahead of it, keeps the fraction 1 - exp(-tau_esc) of
// its weight that scatters inside the box, and draws its first free path
// from the exponential truncated at tau_esc (the same uniform that would
// otherwise give -ln u).  One package per lane, grid-stride over the ids.
#include <hip/hip_runtime.h>

#include "soc_device.h"
#include "soc_kernels.h"

namespace soc {

// Optical depth from the package's position along direction (ox, oy, oz)
// to the box boundary: scattering only, or extinction (absorption +
// scattering).  A probe copy of the package steps through the grid with an
// infinite free path.
template <bool Oct>
__device__ inline float ray_tau(const Pkg<float> &p0, const McArgs &A, float ox, float oy, float oz, bool ext,
                                unsigned long long &steps)
{
    Pkg<float> q = p0;
    q.ux = ox;
    q.uy = oy;
    q.uz = oz;
    set_inverse(q);
    q.tau = __builtin_huge_valf();
    q.W = 1.0;
    q.Wfloor = 0.0;
    q.steps = 0;
    const float k = ext ? A.ks_f + A.ka_f : A.ks_f;
    float tau = 0.0f;
    for (;;) {
        const float n = q.n;
        float d;
        const StepOut o = step<float, Oct>(q, A, A.ks_f, A.ka_f, d);
        tau += n * k * d;
        ++steps;
        if (o.event == kEvEscape || o.event == kEvRunaway) break;
    }
    return tau;
}

// Absolute position in root units.  Octree: up from the leaf through the
// reverse links, halving the position and adding the octant at each level.
template <bool Oct>
__device__ inline void abs_pos(const Pkg<float> &p, const McArgs &A, double &x, double &y, double &z)
{
    double fx = p.fx, fy = p.fy, fz = p.fz;
    if (Oct) {
        int32_t c = p.c;
        for (int L = p.L; L > 0; --L) {
            const int o = (c - (int32_t)A.nroot) & 7;
            fx = 0.5 * (fx + (o & 1));
            fy = 0.5 * (fy + ((o >> 1) & 1));
            fz = 0.5 * (fz + ((o >> 2) & 1));
            c = A.parent[(c - A.nroot) >> 3];
        }
    }
    x = p.cx + fx;
    y = p.cy + fy;
    z = p.cz + fz;
}

__device__ inline int64_t pixel_of(const PeelArgs &P, double x, double y, double z)
{
    const double pos[3] = {x, y, z};
    const int b = P.axis == 0 ? 1 : 0, c = P.axis == 2 ? 1 : 2;
    int64_t i = (int64_t)floor(pos[b] / P.psz), j = (int64_t)floor(pos[c] / P.psz);
    i = i < 0 ? 0 : (i >= P.npx ? P.npx - 1 : i);
    j = j < 0 ? 0 : (j >= P.npy ? P.npy - 1 : j);
    return j * P.npx + i;
}

__device__ inline float hg_phase(float g, float mu)
{
    const float inv4pi = 0.0795774715459476679f;
    if (fabsf(g) < 1e-4f) return inv4pi;
    const float d = 1.0f + g * g - 2.0f * g * mu;
    return inv4pi * (1.0f - g * g) / (d * sqrtf(d));
}

template <bool Oct>
__global__ __launch_bounds__(256) void peel_kernel(McArgs A, PeelArgs P)
{
    const HG<float> hg(A.g_f);
    unsigned long long n_pk = 0, n_st = 0, n_sc = 0, n_ray = 0;
    double e_em = 0.0, e_es = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < A.n_total; id += stride) {
        Pkg<float> p;
        Rng rng;
        uint32_t cls, pid;
        double W0;
        n_pk += 1;
        if (!emit_base<float, Oct>(A, id, p, rng, cls, pid, W0)) continue;
        e_em += W0;
        if (P.direct && cls >= kClassPs0) {
            const PsArg &s = A.ps[cls - kClassPs0];
            const float t = ray_tau<Oct>(p, A, P.ox, P.oy, P.oz, true, n_ray);
            unsafeAtomicAdd(&P.image[pixel_of(P, s.x, s.y, s.z)], W0 * (0.0795774715459476679 * exp(-(double)t)) * P.scale);
        }
        const float xi = next_u<float>(rng, A);
        if (P.forced) {
            const float tesc = ray_tau<Oct>(p, A, p.ux, p.uy, p.uz, false, n_ray);
            const float q = -expm1f(-tesc);
            if (!(q > 0.0f)) continue;
            p.W *= (double)q;
            p.tau = -log1pf(-xi * q);
        } else {
            p.tau = -m_log(xi);
        }
        int nscat = 0;
        for (;;) {
            float d;
            const StepOut o = step<float, Oct>(p, A, A.ks_f, A.ka_f, d);
            n_st += 1;
            if (o.event == kEvEscape) {
                e_es += p.W;
                break;
            }
            if (o.event != kEvScatter && o.event != kEvCross) break;   // weight floor or step cap
            if (o.event == kEvCross) continue;
            // peel off towards the observer, then scatter
            n_sc += 1;
            const float mu = p.ux * P.ox + p.uy * P.oy + p.uz * P.oz;
            const float t = ray_tau<Oct>(p, A, P.ox, P.oy, P.oz, true, n_ray);
            double x, y, z;
            abs_pos<Oct>(p, A, x, y, z);
            unsafeAtomicAdd(&P.image[pixel_of(P, x, y, z)], p.W * (double)hg_phase(A.g_f, mu) * exp(-(double)t) * P.scale);
            if (P.max_scatter > 0 && ++nscat >= P.max_scatter) break;
            scatter_new_direction<float>(p, rng, A, hg);
        }
    }
    // totals: summed over the wave, one set of atomics per wave
    double v[6] = {(double)n_pk, (double)n_st, (double)n_sc, (double)n_ray, e_em, e_es};
    for (int k = 0; k < 6; ++k)
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 6; ++k) unsafeAtomicAdd(&P.totals[k], v[k]);
}

hipError_t launch_peel(const McArgs &a, const PeelArgs &p, int blocks, hipStream_t s)
{
    if (a.nlevels > 1) hipLaunchKernelGGL(peel_kernel<true>, dim3(blocks), dim3(256), 0, s, a, p);
    else hipLaunchKernelGGL(peel_kernel<false>, dim3(blocks), dim3(256), 0, s, a, p);
    return hipGetLastError();
}

}  // namespace soc
