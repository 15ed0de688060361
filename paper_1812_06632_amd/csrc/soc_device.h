// soc_device.h -- device-side building blocks of the SOC Monte Carlo path
// (Juvela 2019, arXiv:1812.06632, Sect. 2.1.1): counter-based random
// numbers, source emission, Henyey-Greenstein scattering and the per-cell
// transport step on regular and octree grids.  Everything is templated on
// the tracing precision R so that the FP32 production kernel and the FP64
// deterministic trace mode execute the same code; the FP32 instantiation
// uses the hardware reciprocal / reciprocal square root (1 ulp), the FP64
// one exact division.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "soc_kernels.h"

namespace soc {

// Index (0..7) of the XCD the calling wave runs on (hardware register
// XCC_ID, bits [3:0]); wave-uniform.
__device__ inline uint32_t xcd_index()
{
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 7u;
}

// Private copy (0..kPrivCopies-1) a wave adds into: its XCD and the
// workgroup's index modulo the copies per XCD; wave-uniform.
__device__ inline uint32_t priv_index()
{
    return xcd_index() + 8u * (blockIdx.x % kPrivPerXcd);
}

// Index of cell (x, y, z) of a regular grid with even dimensions stored in
// 2 x 2 x 2 bricks (hx = nx / 2, hy = ny / 2): the eight cells of a brick
// are 64 consecutive bytes of an FP64 array, bricks in x-fastest order.
__device__ inline int32_t brick_cell(int32_t x, int32_t y, int32_t z, int32_t hx, int32_t hy)
{
    return ((((z >> 1) * hy + (y >> 1)) * hx + (x >> 1)) << 3) | ((z & 1) << 2) | ((y & 1) << 1) | (x & 1);
}

// Per-lane deposit rings in LDS: lane t's kDepSlots entries start at
// t * kRingStride (the pad entry puts neighbouring lanes' rings on
// different banks).  flush_rings adds every ring of the wave through
// add(key, value), transposed: with R = 64 / kDepSlots rings per
// instruction, instruction j takes the rings of lanes R j .. R j + R - 1,
// and lane L the slot L mod kDepSlots of ring R j + L / kDepSlots.  One
// instruction then carries consecutive deposits of a few packages instead
// of one deposit of each of 64: neighbouring cells, often in one 64-byte
// line, and the memory side performs the adds of one instruction that fall
// in one line as one transaction.  Call with the whole wave.
template <typename F>
__device__ inline void flush_rings(const double *lds_dep, const int32_t *lds_cell, int nbuf, F add)
{
    static_assert(64 % kDepSlots == 0, "rings must tile a wave");
    constexpr int R = 64 / kDepSlots;
    const int lane = (int)threadIdx.x & 63;
    const int base = (int)threadIdx.x - lane;
    const int slot = lane % kDepSlots;
#pragma unroll
    for (int j = 0; j < kDepSlots; ++j) {
        const int ring = R * j + lane / kDepSlots;
        const int nb = __shfl(nbuf, ring, 64);
        if (slot < nb) {
            const int e = (base + ring) * kRingStride + slot;
            add(lds_cell[e], lds_dep[e]);
        }
    }
}


// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products with the published multipliers; the key is
// bumped by the published Weyl constants between rounds.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__host__ __device__ inline void philox4x32_10(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * x0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * x2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = y0;
        x2 = y2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

// Uniform in (0,1) on the odd multiples of 2^-24: exact in FP32 and FP64,
// so both precisions consume bit-identical numbers.
template <typename R>
__host__ __device__ inline R u01(uint32_t x)
{
    return ((R)(x >> 9) + (R)0.5) * (R)(1.0 / 8388608.0);
}

// Per-package stream: counter (block, package id, frequency index,
// iteration << 8 | class); the key (seed) is kernel-uniform and passed in.
struct Rng {
    uint32_t blk, pid, tag;
    uint32_t b0, b1, b2, b3;
    int avail;

    __device__ void init(uint32_t package_id, uint32_t iteration, uint32_t cls)
    {
        blk = 0;
        pid = package_id;
        tag = (iteration << 8) | (cls & 0xffu);
        avail = 0;
    }
    __device__ uint32_t word(uint32_t k0, uint32_t k1, uint32_t freq_index)
    {
        if (avail == 0) {
            uint32_t x0 = blk, x1 = pid, x2 = freq_index, x3 = tag;
            philox4x32_10(x0, x1, x2, x3, k0, k1);
            b0 = x0; b1 = x1; b2 = x2; b3 = x3;
            avail = 4;
            ++blk;
        }
        const uint32_t r = b0;
        b0 = b1; b1 = b2; b2 = b3;
        --avail;
        return r;
    }
};

// ------------------------------------------------------------------ math
__device__ inline float m_sqrt(float x) { return sqrtf(x); }
__device__ inline double m_sqrt(double x) { return sqrt(x); }
__device__ inline float m_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double m_rcp(double x) { return 1.0 / x; }
__device__ inline float m_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double m_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ inline float m_log(float x) { return logf(x); }
__device__ inline double m_log(double x) { return log(x); }
__device__ inline void m_sincos2pi(float t, float *s, float *c) { sincospif(2.0f * t, s, c); }
__device__ inline void m_sincos2pi(double t, double *s, double *c) { sincospi(2.0 * t, s, c); }
__device__ inline float m_abs(float x) { return fabsf(x); }
__device__ inline double m_abs(double x) { return fabs(x); }
__device__ inline float m_min(float a, float b) { return fminf(a, b); }
__device__ inline double m_min(double a, double b) { return fmin(a, b); }
__device__ inline float m_max(float a, float b) { return fmaxf(a, b); }
__device__ inline double m_max(double a, double b) { return fmax(a, b); }
__device__ inline float m_clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ inline double m_clamp01(double x) { return fmin(1.0, fmax(0.0, x)); }
template <typename R> __device__ inline R m_inf();
template <> __device__ inline float m_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ inline double m_inf<double>() { return __builtin_huge_val(); }

// 1 - exp(-x) for x >= 0 without cancellation: a degree-6 Taylor polynomial
// below 1/16 (truncation < 2e-9 relative), the exponential above; both are
// evaluated and selected so that lanes do not diverge.
__device__ inline float one_minus_exp_neg(float x)
{
    const float poly =
        x * (1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f - x * (1.0f / 120.0f - x * (1.0f / 720.0f))))));
    const float big = 1.0f - __expf(-x);
    return x < 0.0625f ? poly : big;
}
__device__ inline double one_minus_exp_neg(double x) { return -expm1(-x); }

// ------------------------------------------------------------------ state
// One photon package.  Regular grid: (cx, cy, cz) the cell, c its linear
// index, position inside the cell in [0,1]^3 (kept cell-relative so that
// FP32 rounding does not grow with the distance travelled).  Octree:
// (cx, cy, cz) the root ancestor of the current leaf c at level L, the
// position relative to the leaf in units of its edge.  t* is the exit
// coordinate towards which each component of the direction points (1, 0,
// or 2 with an infinite reciprocal when the component is zero), so the
// distance to the exit face on each axis is (t - f) / u without branches.
// n is the density of the current cell, loaded as soon as the cell is
// known (before the deposit of the previous segment is issued).
template <typename R>
struct Pkg {
    int32_t cx, cy, cz;
    int32_t c, L;
    int32_t par;   // octree: the parent of cell c when known (L > 0), else -1
    int32_t gpar;  // octree: the parent of par when known (L > 1), else -1
    R fx, fy, fz;
    R ux, uy, uz;
    R ix, iy, iz;
    R tx, ty, tz;
    R tau, n;
    double W, Wfloor;
    uint32_t steps;
};

template <typename R>
__device__ inline void set_inverse(Pkg<R> &p)
{
    p.ix = p.ux != (R)0 ? m_rcp(p.ux) : m_inf<R>();
    p.iy = p.uy != (R)0 ? m_rcp(p.uy) : m_inf<R>();
    p.iz = p.uz != (R)0 ? m_rcp(p.uz) : m_inf<R>();
    p.tx = p.ux > (R)0 ? (R)1 : (p.ux < (R)0 ? (R)0 : (R)2);
    p.ty = p.uy > (R)0 ? (R)1 : (p.uy < (R)0 ? (R)0 : (R)2);
    p.tz = p.uz > (R)0 ? (R)1 : (p.uz < (R)0 ? (R)0 : (R)2);
}

// Henyey-Greenstein constants of one frequency.
template <typename R>
struct HG {
    R g, one_m_g, one_p_g, one_m_g2, one_p_g2, inv_2g;
    __device__ explicit HG(R gg)
        : g(gg), one_m_g((R)1 - gg), one_p_g((R)1 + gg), one_m_g2((R)1 - gg * gg), one_p_g2((R)1 + gg * gg),
          inv_2g(m_abs(gg) < (R)1e-4 ? (R)0 : (R)1 / ((R)2 * gg))
    {
    }
};

// Henyey-Greenstein draw (analytic inversion of the cumulative
// distribution; isotropic for |g| < 1e-4) and rotation of the direction
// by polar cosine mu and azimuth 2 pi xi_phi about the old direction.
// sin(theta) is formed from the factors 1 - mu and 1 + mu written without
// cancellation, and the transverse length of the old direction from its
// x and y components, so that FP32 keeps full relative accuracy near
// forward/backward scattering and near the poles.
template <typename R>
__device__ inline void hg_scatter(const HG<R> &h, R xi_mu, R xi_phi, R &ux, R &uy, R &uz)
{
    R mu, one_m, one_p;
    if (m_abs(h.g) < (R)1e-4) {
        mu = (R)2 * xi_mu - (R)1;
        one_m = (R)2 * ((R)1 - xi_mu);
        one_p = (R)2 * xi_mu;
    } else {
        const R rden = m_rcp(h.one_m_g + (R)2 * h.g * xi_mu);
        const R s = h.one_m_g2 * rden;
        mu = (h.one_p_g2 - s * s) * h.inv_2g;
        // 1 - mu = (1-g)(1-xi)(s+1-g)/den,  1 + mu = (1+g) xi (1+g+s)/den
        one_m = h.one_m_g * ((R)1 - xi_mu) * (s + h.one_m_g) * rden;
        one_p = h.one_p_g * xi_mu * (h.one_p_g + s) * rden;
    }
    mu = m_min((R)1, m_max((R)-1, mu));
    const R st = m_sqrt(m_max((R)0, one_m * one_p));
    R sp, cp;
    m_sincos2pi(xi_phi, &sp, &cp);
    R n0, n1, n2;
    const R t2 = ux * ux + uy * uy;
    if (t2 < (R)1e-30) {
        n0 = st * cp;
        n1 = st * sp;
        n2 = (uz >= (R)0 ? mu : -mu);
    } else {
        const R rt = m_rsqrt(t2);
        const R t = t2 * rt;
        n0 = st * (ux * uz * cp - uy * sp) * rt + ux * mu;
        n1 = st * (uy * uz * cp + ux * sp) * rt + uy * mu;
        n2 = -st * cp * t + uz * mu;
    }
    const R rn = m_rsqrt(n0 * n0 + n1 * n1 + n2 * n2);
    ux = n0 * rn;
    uy = n1 * rn;
    uz = n2 * rn;
}

template <typename R>
__device__ inline void iso_dir(R xi_mu, R xi_phi, R &ux, R &uy, R &uz)
{
    const R mu = (R)2 * xi_mu - (R)1;
    const R st = (R)2 * m_sqrt(xi_mu * ((R)1 - xi_mu));   // sqrt(1 - mu^2) without cancellation
    R sp, cp;
    m_sincos2pi(xi_phi, &sp, &cp);
    ux = st * cp;
    uy = st * sp;
    uz = mu;
}

template <typename R, typename AT>
__device__ inline R next_u(Rng &rng, const AT &A)
{
    return u01<R>(rng.word(A.key0, A.key1, A.freq_index));
}

// Split a coordinate (root units, FP64) into a cell index and an offset
// inside the cell.
template <typename R>
__device__ inline void split_coord(double p, int32_t n, int32_t &c, R &f)
{
    double fl = floor(p);
    if (fl > (double)(n - 1)) fl = (double)(n - 1);
    if (fl < 0.0) fl = 0.0;
    c = (int32_t)fl;
    f = (R)(p - fl);
}

// A position on the face between cells c - 1 and c (f = 0) or c and c + 1
// (f = 1) belongs to the cell the direction u points into, the cell a
// position moved an infinitesimal step along u lies in; on the box
// boundary it stays in the box.
template <typename R>
__device__ inline void face_tie(int32_t &c, R &f, R u, int32_t n)
{
    if (f == (R)0 && u < (R)0 && c > 0) {
        c -= 1;
        f = (R)1;
    } else if (f == (R)1 && u > (R)0 && c < n - 1) {
        c += 1;
        f = (R)0;
    }
}

// ------------------------------------------------------------------ octree walk
// Descend from cell p.c (position p.f in its units) to the leaf containing
// the position: child octant o = [f > 1/2, or f = 1/2 and u >= 0] per axis
// (a position on the plane between two octants goes where the direction
// points), f -> 2 f - o.  The leaf's word is its density.
template <typename R, typename AT>
__device__ inline void descend(Pkg<R> &p, const AT &A)
{
    int32_t w = (int32_t)A.words[p.c];
    while (w < 0) {
        const int32_t ox = p.fx > (R)0.5 || (p.fx == (R)0.5 && p.ux >= (R)0);
        const int32_t oy = p.fy > (R)0.5 || (p.fy == (R)0.5 && p.uy >= (R)0);
        const int32_t oz = p.fz > (R)0.5 || (p.fz == (R)0.5 && p.uz >= (R)0);
        p.fx = (R)2 * p.fx - (R)ox;
        p.fy = (R)2 * p.fy - (R)oy;
        p.fz = (R)2 * p.fz - (R)oz;
        p.gpar = p.par;
        p.par = p.c;
        p.c = -w + ox + 2 * oy + 4 * oz;
        p.L += 1;
        w = (int32_t)A.words[p.c];
    }
    p.n = (R)__int_as_float(w);
}

// Move across the face of axis `a` of the current leaf (fw: towards +):
// the partial traversal of Sect. 2.1.1 -- up through the reverse links
// while the face is also a face of the parent, across to the sibling (or
// the neighbouring root cell), then down by position.  The exit coordinate
// must already be on the face (1 when fw, 0 otherwise).  Returns false
// when the package leaves the box.  The first two steps up take the
// parent and grandparent the package passed on its way down (p.par,
// p.gpar) instead of reading the links.
// Octets are 8-aligned relative to every level offset, all of which are
// congruent to nroot mod 8, so the octant of a non-root cell is
// (c - nroot) & 7.
template <typename R, typename AT>
__device__ inline bool cross_octree(Pkg<R> &p, const AT &A, int a, bool fw)
{
    for (;;) {
        if (p.L == 0) {
            if (a == 0) {
                p.cx += fw ? 1 : -1;
                if (p.cx < 0 || p.cx >= A.nx) return false;
                p.fx = fw ? (R)0 : (R)1;
            } else if (a == 1) {
                p.cy += fw ? 1 : -1;
                if (p.cy < 0 || p.cy >= A.ny) return false;
                p.fy = fw ? (R)0 : (R)1;
            } else {
                p.cz += fw ? 1 : -1;
                if (p.cz < 0 || p.cz >= A.nz) return false;
                p.fz = fw ? (R)0 : (R)1;
            }
            p.c = p.cx + A.nx * (p.cy + A.ny * p.cz);
            p.par = -1;
            p.gpar = -1;
            break;
        }
        const int32_t o = (int32_t)((p.c - A.nroot) & 7);
        const int32_t bit = (o >> a) & 1;
        if (fw ? bit == 0 : bit == 1) {
            p.c += fw ? (1 << a) : -(1 << a);
            if (a == 0) p.fx = fw ? (R)0 : (R)1;
            else if (a == 1) p.fy = fw ? (R)0 : (R)1;
            else p.fz = fw ? (R)0 : (R)1;
            break;
        }
        p.fx = (p.fx + (R)(o & 1)) * (R)0.5;
        p.fy = (p.fy + (R)((o >> 1) & 1)) * (R)0.5;
        p.fz = (p.fz + (R)((o >> 2) & 1)) * (R)0.5;
        // the parent is known when the package came down into this octet
        // (and the next one up when it came down two levels); the link is
        // read only above that
        int32_t up = p.par;
        if (up < 0) up = A.parent[(p.c - A.nroot) >> 3];
        p.c = up;
        p.par = p.gpar;
        p.gpar = -1;
        p.L -= 1;
    }
    descend(p, A);
    return true;
}

// ------------------------------------------------------------------ emission

// Emit package `gid` (global order: background | point sources | dust) and
// draw its first free path.  Returns false for a package that carries no
// energy (it is counted but not traced).  `cls`/`pid` receive the class
// and the id within the class; W0 the package energy.
template <typename R, bool Oct, typename AT>
__device__ inline bool emit_base(const AT &A, uint64_t gid, Pkg<R> &p, Rng &rng, uint32_t &cls,
                                 uint32_t &pid, double &W0);

template <typename R, bool Oct, typename AT>
__device__ inline bool emit(const AT &A, uint64_t gid, Pkg<R> &p, Rng &rng, uint32_t &cls,
                            uint32_t &pid, double &W0)
{
    if (!emit_base<R, Oct>(A, gid, p, rng, cls, pid, W0)) return false;
    p.tau = -m_log(next_u<R>(rng, A));
    return true;
}

// Emission without the free path: position, direction, weight; the next
// uniform of the package's stream is its first free path.
template <typename R, bool Oct, typename AT>
__device__ inline bool emit_base(const AT &A, uint64_t gid, Pkg<R> &p, Rng &rng, uint32_t &cls,
                                 uint32_t &pid, double &W0)
{
    p.L = 0;
    p.par = -1;
    p.gpar = -1;
    const uint64_t nps_tot = (uint64_t)A.n_ps * A.n_ps_pk;
    if (gid < A.n_bg) {
        cls = kClassBg;
        pid = (uint32_t)gid;
        rng.init(pid, A.iteration, cls);
        W0 = A.W_bg;
        if (!(W0 > 0.0)) return false;
        const double x0 = next_u<double>(rng, A);
        const R x1 = next_u<R>(rng, A), x2 = next_u<R>(rng, A), x3 = next_u<R>(rng, A), x4 = next_u<R>(rng, A);
        const double tt = x0 * A.face_tot;
        int face = 5;
        for (int k = 0; k < 6; ++k) {
            if (tt < A.face_cum[k]) { face = k; break; }
        }
        const int a = face >> 1;
        const bool neg = (face & 1) == 0;
        const R mu = m_sqrt(x3);
        const R st = m_sqrt((R)1 - x3);   // exact 1 - x3 on the uniform grid
        R sp, cp;
        m_sincos2pi(x4, &sp, &cp);
        const R ua = neg ? mu : -mu, ub = st * cp, uc = st * sp;
        // tangential axes b < c of face axis a
        int32_t cb, cc;
        R fb, fc;
        const int32_t Nb = a == 0 ? A.ny : A.nx;
        const int32_t Nc = a == 2 ? A.ny : A.nz;
        split_coord<R>((double)x1 * Nb, Nb, cb, fb);
        split_coord<R>((double)x2 * Nc, Nc, cc, fc);
        face_tie<R>(cb, fb, ub, Nb);
        face_tie<R>(cc, fc, uc, Nc);
        const int32_t Na = a == 0 ? A.nx : (a == 1 ? A.ny : A.nz);
        const int32_t ca = neg ? 0 : Na - 1;
        const R fa = neg ? (R)0 : (R)1;
        if (a == 0) {
            p.cx = ca; p.fx = fa; p.ux = ua;
            p.cy = cb; p.fy = fb; p.uy = ub;
            p.cz = cc; p.fz = fc; p.uz = uc;
        } else if (a == 1) {
            p.cx = cb; p.fx = fb; p.ux = ub;
            p.cy = ca; p.fy = fa; p.uy = ua;
            p.cz = cc; p.fz = fc; p.uz = uc;
        } else {
            p.cx = cb; p.fx = fb; p.ux = ub;
            p.cy = cc; p.fy = fc; p.uy = uc;
            p.cz = ca; p.fz = fa; p.uz = ua;
        }
        p.c = p.cx + A.nx * (p.cy + A.ny * p.cz);
    } else if (gid < A.n_bg + nps_tot) {
        const uint64_t k = gid - A.n_bg;
        const int32_t s = (int32_t)(k / A.n_ps_pk);
        cls = kClassPs0 + (uint32_t)s;
        pid = (uint32_t)(k - (uint64_t)s * A.n_ps_pk);
        rng.init(pid, A.iteration, cls);
        W0 = A.ps[s].W;
        if (!(W0 > 0.0)) return false;
        split_coord<R>(A.ps[s].x, A.nx, p.cx, p.fx);
        split_coord<R>(A.ps[s].y, A.ny, p.cy, p.fy);
        split_coord<R>(A.ps[s].z, A.nz, p.cz, p.fz);
        const R x0 = next_u<R>(rng, A), x1 = next_u<R>(rng, A);
        iso_dir<R>(x0, x1, p.ux, p.uy, p.uz);
        face_tie<R>(p.cx, p.fx, p.ux, A.nx);   // a source on a cell face
        face_tie<R>(p.cy, p.fy, p.uy, A.ny);
        face_tie<R>(p.cz, p.fz, p.uz, A.nz);
        p.c = p.cx + A.nx * (p.cy + A.ny * p.cz);
    } else {
        const uint64_t j = gid - A.n_bg - nps_tot;
        cls = kClassDust;
        pid = (uint32_t)j;
        rng.init(pid, A.iteration, cls);
        int64_t c;
        if (A.dust_mode == 0) {
            c = A.leaves ? A.leaves[j / A.per_leaf] : (int64_t)(j / A.per_leaf);
            W0 = A.dust_L[c] / (double)A.per_leaf;
        } else {
            // a package of cell c carries L_c over the cell's expected
            // count min(N |L_c| / S, cap): S / N, or |L_c| / cap for a
            // capped cell, with the sign of L_c (mode 2 emits the signed
            // difference to the reference emission)
            c = A.dust_cell[j];
            if (c < 0) return false;
            const double WN = *A.dust_S / (double)A.n_dust;
            W0 = (A.dust_mode == 1 && !(A.dust_cap > 0.0)) ? WN : weighted_package_weight(WN, A.dust_cap, A.dust_L[c]);
        }
        if (!(fabs(W0) > 0.0)) return false;
        int64_t root = c;
        if (Oct) {
            // level of the leaf, then up through the reverse links to its root ancestor
            int L = 0;
            while (L + 1 < A.nlevels && c >= A.level_offset[L + 1]) ++L;
            p.L = L;
            for (int l = L; l > 0; --l) {
                root = A.parent[(root - A.nroot) >> 3];
                if (l == L) p.par = (int32_t)root;
                if (l == L - 1) p.gpar = (int32_t)root;
            }
        }
        p.c = (int32_t)c;
        p.cx = (int32_t)(root % A.nx);
        p.cy = (int32_t)((root / A.nx) % A.ny);
        p.cz = (int32_t)(root / ((int64_t)A.nx * A.ny));
        p.fx = next_u<R>(rng, A);
        p.fy = next_u<R>(rng, A);
        p.fz = next_u<R>(rng, A);
        const R x3 = next_u<R>(rng, A), x4 = next_u<R>(rng, A);
        iso_dir<R>(x3, x4, p.ux, p.uy, p.uz);
    }
    if (Oct && cls != kClassDust) descend(p, A);
    else p.n = (R)__uint_as_float(A.words[p.c]);
    set_inverse(p);
    p.W = W0;
    p.Wfloor = 1e-12 * fabs(W0);
    p.steps = 0;
    return true;
}

// ------------------------------------------------------------------ transport
struct StepOut {
    int32_t cell;
    int32_t event;
    double dep;     // energy deposited in `cell` by this segment (incl. floor/runaway remainder)
};

// One segment of the per-cell loop (Sect. 2.1.1): distance to the exit
// face (ties broken x < y < z) against the distance to the next
// scattering, continuous absorption W (1 - e^{-k_abs d}) deposited in the
// cell, then the crossing -- a DDA step on a regular grid, the partial
// up/down traversal on an octree -- or the scattering position; escape,
// weight floor and step cap end the package with the remainder deposited.
// On an octree distances and optical depths are in units of the current
// leaf (edge 2^-L root cells).  d_out is in root units.  The density of
// the next cell is loaded here, before the caller issues the deposit, so
// that waiting for it never waits for the atomic.  The caller adds `dep`
// to the absorbed array and draws the new direction after a scattering.
template <typename R, bool Oct, typename AT>
__device__ inline StepOut step(Pkg<R> &p, const AT &A, R ks_scale, R ka_scale, R &d_out)
{
    StepOut o;
    o.cell = p.c;
    R edge = (R)1;
    if (Oct) edge = m_rcp((R)(1 << p.L));
    const R ks = p.n * ks_scale * edge, ka = p.n * ka_scale * edge;
    const R dx = (p.tx - p.fx) * p.ix;
    const R dy = (p.ty - p.fy) * p.iy;
    const R dz = (p.tz - p.fz) * p.iz;
    const int ax = (dx <= dy && dx <= dz) ? 0 : (dy <= dz ? 1 : 2);
    const R dexit = m_max((R)0, ax == 0 ? dx : (ax == 1 ? dy : dz));
    R d;
    int ev;
    const R tcell = ks * dexit;
    if (ks > (R)0 && tcell >= p.tau) {
        d = m_min(p.tau * m_rcp(ks), dexit);
        ev = kEvScatter;
    } else {
        d = dexit;
        p.tau -= tcell;
        ev = kEvCross;
    }
    if (ev == kEvCross) {
        bool fw;
        if (ax == 0) {
            p.fy = m_clamp01(p.fy + d * p.uy);
            p.fz = m_clamp01(p.fz + d * p.uz);
            fw = p.ux > (R)0;
        } else if (ax == 1) {
            p.fx = m_clamp01(p.fx + d * p.ux);
            p.fz = m_clamp01(p.fz + d * p.uz);
            fw = p.uy > (R)0;
        } else {
            p.fx = m_clamp01(p.fx + d * p.ux);
            p.fy = m_clamp01(p.fy + d * p.uy);
            fw = p.uz > (R)0;
        }
        if (Oct) {
            if (ax == 0) p.fx = fw ? (R)1 : (R)0;
            else if (ax == 1) p.fy = fw ? (R)1 : (R)0;
            else p.fz = fw ? (R)1 : (R)0;
            if (!cross_octree(p, A, ax, fw)) ev = kEvEscape;
        } else {
            const int32_t step_i = fw ? 1 : -1;
            if (ax == 0) {
                p.fx = fw ? (R)0 : (R)1;
                p.cx += step_i;
                p.c += step_i;
                if ((uint32_t)p.cx >= (uint32_t)A.nx) ev = kEvEscape;
            } else if (ax == 1) {
                p.fy = fw ? (R)0 : (R)1;
                p.cy += step_i;
                p.c += step_i * A.nx;
                if ((uint32_t)p.cy >= (uint32_t)A.ny) ev = kEvEscape;
            } else {
                p.fz = fw ? (R)0 : (R)1;
                p.cz += step_i;
                p.c += step_i * A.nx * A.ny;
                if ((uint32_t)p.cz >= (uint32_t)A.nz) ev = kEvEscape;
            }
            if (ev != kEvEscape) p.n = (R)__uint_as_float(A.words[p.c]);
        }
    } else {
        p.fx = m_clamp01(p.fx + d * p.ux);
        p.fy = m_clamp01(p.fy + d * p.uy);
        p.fz = m_clamp01(p.fz + d * p.uz);
    }
    const R fr = one_minus_exp_neg(ka * d);
    double dep = p.W * (double)fr;
    p.W -= dep;
    p.steps += 1;
    d_out = d * edge;
    if (ev != kEvEscape) {
        if (fabs(p.W) < p.Wfloor) {
            dep += p.W;
            p.W = 0.0;
            ev = kEvFloor;
        } else if ((int64_t)p.steps >= A.step_cap) {
            dep += p.W;
            p.W = 0.0;
            ev = kEvRunaway;
        }
    }
    o.dep = dep;
    o.event = ev;
    return o;
}

template <typename R, typename AT>
__device__ inline void scatter_new_direction(Pkg<R> &p, Rng &rng, const AT &A, const HG<R> &h)
{
    const R xm = next_u<R>(rng, A), xp = next_u<R>(rng, A);
    hg_scatter<R>(h, xm, xp, p.ux, p.uy, p.uz);
    set_inverse(p);
    p.tau = -m_log(next_u<R>(rng, A));
}

}  // namespace soc
