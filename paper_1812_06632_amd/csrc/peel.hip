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
// otherwise give -ln u).
//
// Each lane is a small state machine: idle, transporting its package, or
// marching a ray to the boundary (the direct light of a point source, the
// escape depth of forced scattering, or a peel-off).  Every pass of the loop
// takes one step of whichever it is doing, so long rays and long packages do
// not hold the rest of the wave; idle lanes are refilled together from a
// wave-private id pool topped up with one atomic per `chunk` ids, as in the
// Monte Carlo kernel.
#include <hip/hip_runtime.h>

#include "soc_device.h"
#include "soc_kernels.h"

namespace soc {

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

// Start a ray from the package's position along (ox, oy, oz): a probe copy
// with an infinite free path and no weight floor.
__device__ inline void ray_start(Pkg<float> &q, const Pkg<float> &p, float ox, float oy, float oz)
{
    q = p;
    q.ux = ox;
    q.uy = oy;
    q.uz = oz;
    set_inverse(q);
    q.tau = __builtin_huge_valf();
    q.W = 1.0;
    q.Wfloor = 0.0;
    q.steps = 0;
}

enum : int { kIdle = 0, kTransport = 1, kRay = 2, kAfterDirect = 3 };
enum : int { kRayDirect = 0, kRayEscape = 1, kRayPeel = 2 };

template <bool Oct>
__global__ __launch_bounds__(256, 3) void peel_kernel(McArgs A, PeelArgs P)
{
    const HG<float> hg(A.g_f);
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long n_pk = 0, n_st = 0, n_sc = 0, n_ray = 0;
    double e_em = 0.0, e_es = 0.0;
    // q is what the lane steps: its package, or the probe of one of the
    // package's rays while p keeps the package
    Pkg<float> p, q;
    Rng rng;
    int mode = kIdle, ray = kRayDirect, nscat = 0;
    float xi = 0.0f, rtau = 0.0f, rk = 0.0f;
    double W0 = 0.0;
    int64_t src_pix = 0;
    unsigned long long pool_next = 0, pool_end = 0;   // wave-uniform
    bool exhausted = false;                           // wave-uniform
    for (;;) {
        // refill idle lanes from the wave's id pool
        const unsigned long long idle = __ballot(mode == kIdle);
        const int nidle = __popcll(idle);
        if (!exhausted && nidle > 0) {
            const unsigned long long avail = pool_end - pool_next;
            unsigned long long grant = 0;
            if (avail < (unsigned long long)nidle) {
                const int leader = __ffsll((long long)idle) - 1;
                unsigned long long b = 0;
                if (lane == leader) b = atomicAdd(A.next_id, (unsigned long long)A.chunk);
                grant = (unsigned long long)__shfl((long long)b, leader, 64);
            }
            if (mode == kIdle) {
                const unsigned long long r = (unsigned long long)__popcll(idle & below);
                const unsigned long long id = r < avail ? pool_next + r : grant + (r - avail);
                if (id < A.n_total) {
                    uint32_t cls, pid;
                    n_pk += 1;
                    if (emit_base<float, Oct>(A, id, q, rng, cls, pid, W0)) {
                        e_em += W0;
                        nscat = 0;
                        xi = next_u<float>(rng, A);
                        if (P.direct && cls >= kClassPs0) {
                            const PsArg &s = A.ps[cls - kClassPs0];
                            src_pix = pixel_of(P, s.x, s.y, s.z);
                            p = q;
                            ray_start(q, p, P.ox, P.oy, P.oz);
                            ray = kRayDirect;
                            rk = A.ks_f + A.ka_f;
                            rtau = 0.0f;
                            mode = kRay;
                        } else {
                            mode = kAfterDirect;
                        }
                    }
                }
            }
            if (avail < (unsigned long long)nidle) {
                pool_next = grant + ((unsigned long long)nidle - avail);
                pool_end = grant + (unsigned long long)A.chunk;
            } else {
                pool_next += (unsigned long long)nidle;
            }
            if (pool_next >= A.n_total) exhausted = true;
        }
        // after the direct light (or at once): the escape depth, or the first free path
        if (mode == kAfterDirect) {
            if (P.forced) {
                p = q;
                ray_start(q, p, p.ux, p.uy, p.uz);
                ray = kRayEscape;
                rk = A.ks_f;
                rtau = 0.0f;
                mode = kRay;
            } else {
                q.tau = -m_log(xi);
                mode = kTransport;
            }
        }
        if (!__any(mode != kIdle)) {
            if (exhausted) break;
            continue;
        }
        if (mode == kIdle) continue;
        const float n = q.n;
        float d;
        const StepOut o = step<float, Oct>(q, A, A.ks_f, A.ka_f, d);
        if (mode == kRay) {
            rtau += n * rk * d;
            ++n_ray;
            if (o.event == kEvEscape || o.event == kEvRunaway) {
                q = p;   // back to the package
                if (ray == kRayDirect) {
                    unsafeAtomicAdd(&P.image[src_pix], W0 * (0.0795774715459476679 * exp(-(double)rtau)) * P.scale);
                    mode = kAfterDirect;
                } else if (ray == kRayEscape) {
                    const float qf = -expm1f(-rtau);
                    if (!(qf > 0.0f)) {
                        mode = kIdle;
                    } else {
                        q.W *= (double)qf;
                        q.tau = -log1pf(-xi * qf);
                        mode = kTransport;
                    }
                } else {   // peel-off of the scattering at q
                    const float mu = q.ux * P.ox + q.uy * P.oy + q.uz * P.oz;
                    double x, y, z;
                    abs_pos<Oct>(q, A, x, y, z);
                    unsafeAtomicAdd(&P.image[pixel_of(P, x, y, z)],
                                    q.W * (double)hg_phase(A.g_f, mu) * exp(-(double)rtau) * P.scale);
                    if (P.max_scatter > 0 && ++nscat >= P.max_scatter) {
                        mode = kIdle;
                    } else {
                        scatter_new_direction<float>(q, rng, A, hg);
                        mode = kTransport;
                    }
                }
            }
        } else {
            n_st += 1;
            if (o.event == kEvEscape) {
                e_es += q.W;
                mode = kIdle;
            } else if (o.event == kEvScatter) {   // peel off towards the observer, then scatter
                n_sc += 1;
                p = q;
                ray_start(q, p, P.ox, P.oy, P.oz);
                ray = kRayPeel;
                rk = A.ks_f + A.ka_f;
                rtau = 0.0f;
                mode = kRay;
            } else if (o.event != kEvCross) {   // weight floor or step cap
                mode = kIdle;
            }
        }
    }
    // totals: summed over the wave, one set of atomics per wave
    double v[6] = {(double)n_pk, (double)n_st, (double)n_sc, (double)n_ray, e_em, e_es};
    for (int k = 0; k < 6; ++k)
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if (lane == 0)
        for (int k = 0; k < 6; ++k) unsafeAtomicAdd(&P.totals[k], v[k]);
}

hipError_t launch_peel(const McArgs &a, const PeelArgs &p, int blocks, hipStream_t s)
{
    if (a.nlevels > 1) hipLaunchKernelGGL(peel_kernel<true>, dim3(blocks), dim3(256), 0, s, a, p);
    else hipLaunchKernelGGL(peel_kernel<false>, dim3(blocks), dim3(256), 0, s, a, p);
    return hipGetLastError();
}

}  // namespace soc
