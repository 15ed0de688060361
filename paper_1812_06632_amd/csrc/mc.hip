// mc.hip -- Monte Carlo photon-package kernels for regular and octree grids
// (Juvela 2019, Sect. 2.1.1: one package per thread, one frequency per
// launch, absorbed energy counted per cell).
//
// Production kernel: persistent waves.  Every lane owns one package; when
// lanes finish (escape, weight floor, step cap) the wave refills them
// together: a ballot of the idle lanes, their rank from the lane mask,
// ids taken from a wave-private pool that is topped up with one atomic per
// `chunk` ids.  Creation and tracking of packages are thereby interleaved
// (the scheme the paper suggests in Sect. 4.2), so lanes do not idle until
// the slowest package of the wave ends.  Deposits go straight to the FP64
// absorbed array with hardware FP64 atomics (global_atomic_add_f64), but
// not one by one: on CDNA the vector-memory counter retires loads and
// atomics in issue order, so a wait for the next cell's density would also
// wait for the previous step's atomic round trip.  Each lane therefore
// stages its deposits in an LDS ring of kDepSlots entries and the wave
// flushes the rings as one burst of atomics every kDepSlots iterations:
// one atomic latency per kDepSlots steps instead of per step.  The burst
// is transposed (flush_rings): each atomic instruction carries consecutive
// deposits of a few packages, and on a regular grid the private copies are
// kept in 2 x 2 x 2 bricks (brick_cell; on an octree its root cells, the
// eight children of a cell being contiguous already), so that these
// neighbouring cells often share a 64-byte line and one memory-side
// transaction.
#include "soc_device.h"

namespace soc {

__device__ inline unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += (unsigned long long)__shfl_xor((long long)v, o, 64);
    return v;
}
__device__ inline double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline void add_stats(DevStats *t, unsigned long long pk, unsigned long long st, unsigned long long sc,
                                 unsigned long long ru, double em, double ab, double es)
{
    atomicAdd(&t->packages, pk);
    atomicAdd(&t->steps, st);
    atomicAdd(&t->scatterings, sc);
    atomicAdd(&t->runaways, ru);
    unsafeAtomicAdd(&t->emitted, em);
    unsafeAtomicAdd(&t->absorbed, ab);
    unsafeAtomicAdd(&t->escaped, es);
}

__device__ inline void flush_stats(const McArgs &A, unsigned long long pk, unsigned long long st,
                                   unsigned long long sc, unsigned long long ru, double em, double ab, double es)
{
    pk = wave_sum_u64(pk);
    st = wave_sum_u64(st);
    sc = wave_sum_u64(sc);
    ru = wave_sum_u64(ru);
    em = wave_sum_f64(em);
    ab = wave_sum_f64(ab);
    es = wave_sum_f64(es);
    if ((threadIdx.x & 63) == 0) {
        add_stats(A.st_call, pk, st, sc, ru, em, ab, es);
        add_stats(A.st_total, pk, st, sc, ru, em, ab, es);
    }
}

// Flush of the wave's deposit rings: with diagonal ALI a dust package's
// deposits in its own emitting cell go to the self-absorption tally, marked
// by storing the complement of the cell index.
template <bool Ali>
__device__ inline void flush_deposits(double *dst, double *sdst, const double *lds_dep, const int32_t *lds_cell,
                                      int nbuf)
{
    flush_rings(lds_dep, lds_cell, nbuf, [&](int32_t key, double v) {
        if (Ali && key < 0) unsafeAtomicAdd(&sdst[~key], v);
        else unsafeAtomicAdd(&dst[key], v);
    });
}

// Per-wave state that outlives one frequency: the LDS deposit ring and the
// statistics.
struct WaveTally {
    int nbuf = 0;          // deposits staged by this lane
    int since_flush = 0;   // wave-uniform
    unsigned long long n_pk = 0, n_st = 0, n_sc = 0, n_ru = 0;
    double e_em = 0.0, e_ab = 0.0, e_es = 0.0;
};

// Every package of one frequency's argument block A: ids from A.next_id in
// chunks, until the ids are used up and every lane of the wave has
// finished.  Deposits go through the lane's LDS ring to dst (sdst: the
// ALI self-absorption tally), keyed by brick_cell when A.brick is set.
template <bool Oct, bool Ali, typename AT>
__device__ __forceinline__ void mc_frequency(const AT &A, double *lds_dep, int32_t *lds_cell, double *dst,
                                             double *sdst, WaveTally &w)
{
    const int ring = (int)threadIdx.x * kRingStride;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const bool brick = A.brick;
    const int32_t hx = A.nx >> 1, hy = A.ny >> 1;
    const int64_t nroot = A.nroot;
    Pkg<float> p;
    Rng rng;
    bool active = false;   // lane holds a package
    bool pend = false;     // its last segment ended in a scattering whose new direction is not drawn yet
    bool first_step = false;   // its first step is still to come
    int32_t origin = -1;       // ALI: emitting cell of a dust package
    unsigned long long pool_next = 0, pool_end = 0;   // wave-uniform
    bool exhausted = false;                           // wave-uniform
    const float ks = A.ks_f, ka = A.ka_f;
    const HG<float> hg(A.g_f);
    int &nbuf = w.nbuf;
    int &since_flush = w.since_flush;
    for (;;) {
        // refill idle lanes from the wave's id pool
        const unsigned long long idle = __ballot(!active);
        const int nidle = __popcll(idle);
        if (!exhausted && nidle > 0 && (nidle >= A.refill_min || nidle == 64)) {
            const unsigned long long avail = pool_end - pool_next;
            unsigned long long grant = 0;   // first id of a new chunk from the global counter
            if (avail < (unsigned long long)nidle) {
                const int leader = __ffsll((long long)idle) - 1;
                unsigned long long b = 0;
                if (lane == leader) b = atomicAdd(A.next_id, (unsigned long long)A.chunk);
                grant = (unsigned long long)__shfl((long long)b, leader, 64);
            }
            if (!active) {
                const unsigned long long r = (unsigned long long)__popcll(idle & below);
                const unsigned long long id = r < avail ? pool_next + r : grant + (r - avail);
                if (id < A.n_total) {
                    uint32_t cls, pid;
                    double W0;
                    const bool ok = emit<float, Oct>(A, id, p, rng, cls, pid, W0);
                    w.n_pk += 1;
                    if (ok) w.e_em += W0;
                    active = ok;
                    first_step = ok;
                    if (Ali) origin = ok && cls == kClassDust ? p.c : -1;
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
        if (!__any(active)) {
            if (exhausted) break;
            continue;
        }
        // scatterings are drawn together once enough lanes wait for one
        // (or no lane could step otherwise)
        const unsigned long long pm = __ballot(pend);
        if (pm) {
            if (__popcll(pm) >= A.scatter_min || __ballot(active && !pend) == 0) {
                if (pend) {
                    scatter_new_direction<float>(p, rng, A, hg);
                    pend = false;
                }
            }
        }
        if ((since_flush + 1) * A.inner_steps > kDepSlots) {
            flush_deposits<Ali>(dst, sdst, lds_dep, lds_cell, nbuf);
            nbuf = 0;
            since_flush = 0;
        }
        ++since_flush;
        for (int s = 0; s < A.inner_steps; ++s) {
            const bool stepping = active && !pend;
            StepOut o;
            o.cell = 0;
            o.event = kEvCross;
            o.dep = 0.0;
            // the cell before the step; a root cell (every cell of a regular
            // grid) by its brick index
            const int32_t bcell = brick ? (p.c < nroot ? brick_cell(p.cx, p.cy, p.cz, hx, hy) : p.c) : 0;
            if (stepping) {
                float d;
                o = step<float, Oct>(p, A, ks, ka, d);
                w.n_st += 1;
                w.e_ab += o.dep;
            }
            // Packages refilled together often start in the same cell (the
            // luminosity-weighted emission puts consecutive ids in the
            // brightest cells): the first deposits of the lanes that share
            // the cell of the lowest such lane are summed in registers and
            // staged once, which spares the memory-side atomic unit a burst
            // of same-address adds.
            double dep = o.dep;
            const int32_t tcell = brick ? bcell : o.cell;
            const int32_t key = (Ali && o.cell == origin) ? ~tcell : tcell;
            const bool first = stepping && first_step && dep != 0.0;
            if (stepping) first_step = false;
            const unsigned long long fm = __ballot(first);
            if (fm & (fm - 1)) {   // at least two lanes
                const int leader = __ffsll((long long)fm) - 1;
                const int c0 = __shfl(key, leader, 64);
                const bool in = first && key == c0;
                const unsigned long long gm = __ballot(in);
                if (gm & (gm - 1)) {
                    double v = in ? dep : 0.0;
                    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
                    if (in) dep = lane == leader ? v : 0.0;
                }
            }
            // A segment that ends in a scattering is followed by one in the
            // same cell: consecutive deposits of a lane into one cell share
            // a ring slot, so each scattering saves one atomic.
            if (dep != 0.0) {
                if (nbuf > 0 && lds_cell[ring + nbuf - 1] == key) {
                    lds_dep[ring + nbuf - 1] += dep;
                } else {
                    lds_dep[ring + nbuf] = dep;
                    lds_cell[ring + nbuf] = key;
                    ++nbuf;
                }
            }
            if (stepping) {
                if (o.event == kEvScatter) {
                    pend = true;
                    w.n_sc += 1;
                } else if (o.event != kEvCross) {
                    active = false;
                    if (o.event == kEvEscape) w.e_es += p.W;
                    if (o.event == kEvRunaway) w.n_ru += 1;
                }
            }
        }
    }
}

template <bool Oct, bool Ali>
__device__ __forceinline__ void mc_body(const McArgs &A)
{
    extern __shared__ double lds_dep[];   // [blockDim.x][kRingStride] deposits, then cells
    int32_t *lds_cell = (int32_t *)(lds_dep + kRingStride * blockDim.x);
    double *const dst = A.priv ? A.priv + (size_t)priv_index() * (size_t)A.ncells : A.absorbed;
    double *const sdst = A.priv_self ? A.priv_self + (size_t)priv_index() * (size_t)A.ncells : A.ali_self;
    WaveTally w;
    mc_frequency<Oct, Ali>(A, lds_dep, lds_cell, dst, sdst, w);
    flush_deposits<Ali>(dst, sdst, lds_dep, lds_cell, w.nbuf);
    flush_stats(A, w.n_pk, w.n_st, w.n_sc, w.n_ru, w.e_em, w.e_ab, w.e_es);
}

template <bool Oct>
__global__ __launch_bounds__(kMcMaxBlock) void mc_kernel(McArgs A)
{
    mc_body<Oct, false>(A);
}

// The same with the diagonal-ALI tallies (Sect. 2.1.2).
template <bool Oct>
__global__ __launch_bounds__(kMcMaxBlock) void mc_ali_kernel(McArgs A)
{
    mc_body<Oct, true>(A);
}

// Several frequencies of one grid in one persistent launch (the argument
// blocks in device memory, one package-id counter each, all deposits into
// one tally): a wave works through the frequencies in a rotation and moves
// on when its current one has no ids left and its lanes are idle, so only
// the last frequencies leave a tail, not every one.  The rotation starts
// at the wave's own index (spread: the waves divide over the frequencies)
// or at 0 (all waves on one frequency, the next one filling in as it
// ends).  With Ali, a dust package's deposits in its emitting cell go to
// the self-absorption tally, as in mc_ali_kernel.
template <bool Oct, bool Ali>
__global__ __launch_bounds__(kMcMaxBlock) void mc_multi_kernel(MultiArgs M)
{
    extern __shared__ double lds_dep[];   // [blockDim.x][kRingStride] deposits, then cells
    int32_t *lds_cell = (int32_t *)(lds_dep + kRingStride * blockDim.x);
    // the argument blocks do not change during the launch: read them through
    // the constant address space, so that their fields are scalar loads
    const __attribute__((address_space(4))) McArgs *args = (const __attribute__((address_space(4))) McArgs *)M.args;
    const McArgs &A0 = M.args[0];
    double *const dst = A0.priv ? A0.priv + (size_t)priv_index() * (size_t)A0.ncells : A0.absorbed;
    double *const sdst = !Ali ? nullptr
                              : (A0.priv_self ? A0.priv_self + (size_t)priv_index() * (size_t)A0.ncells : A0.ali_self);
    WaveTally w;
    const int wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int k0 = M.spread ? wave % M.K : 0;
    for (int j = 0; j < M.K; ++j) {
        const int k = __builtin_amdgcn_readfirstlane((k0 + j) % M.K);
        mc_frequency<Oct, Ali>(args[k], lds_dep, lds_cell, dst, sdst, w);
    }
    flush_deposits<Ali>(dst, sdst, lds_dep, lds_cell, w.nbuf);
    flush_stats(A0, w.n_pk, w.n_st, w.n_sc, w.n_ru, w.e_em, w.e_ab, w.e_es);
}

hipError_t launch_mc_multi(const MultiArgs &m, int nlevels, bool ali, int blocks, int threads, hipStream_t s)
{
    const size_t lds = (size_t)kRingStride * threads * (sizeof(double) + sizeof(int32_t));
    if (nlevels > 1 && ali) hipLaunchKernelGGL((mc_multi_kernel<true, true>), dim3(blocks), dim3(threads), lds, s, m);
    else if (nlevels > 1) hipLaunchKernelGGL((mc_multi_kernel<true, false>), dim3(blocks), dim3(threads), lds, s, m);
    else if (ali) hipLaunchKernelGGL((mc_multi_kernel<false, true>), dim3(blocks), dim3(threads), lds, s, m);
    else hipLaunchKernelGGL((mc_multi_kernel<false, false>), dim3(blocks), dim3(threads), lds, s, m);
    return hipGetLastError();
}

hipError_t launch_mc(const McArgs &a, int blocks, int threads, hipStream_t s)
{
    const size_t lds = (size_t)kRingStride * threads * (sizeof(double) + sizeof(int32_t));
    const bool ali = a.ali_self != nullptr;
    if (a.nlevels > 1 && ali) hipLaunchKernelGGL(mc_ali_kernel<true>, dim3(blocks), dim3(threads), lds, s, a);
    else if (ali) hipLaunchKernelGGL(mc_ali_kernel<false>, dim3(blocks), dim3(threads), lds, s, a);
    else if (a.nlevels > 1) hipLaunchKernelGGL(mc_kernel<true>, dim3(blocks), dim3(threads), lds, s, a);
    else hipLaunchKernelGGL(mc_kernel<false>, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ traces
template <typename R, bool Oct>
__global__ __launch_bounds__(256) void trace_kernel(McArgs A, TraceArgs T)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T.n) return;
    const uint32_t id = T.ids[i];
    const uint64_t nps_tot = (uint64_t)A.n_ps * A.n_ps_pk;
    uint64_t gid;
    if (T.cls == kClassBg) gid = id;
    else if (T.cls == kClassDust) gid = A.n_bg + nps_tot + id;
    else gid = A.n_bg + (uint64_t)(T.cls - kClassPs0) * A.n_ps_pk + id;
    Pkg<R> p;
    Rng rng;
    uint32_t cls, pid;
    double W0;
    int32_t ns = 0;
    const R ks = sizeof(R) == 8 ? (R)A.ks_d : (R)A.ks_f;
    const R ka = sizeof(R) == 8 ? (R)A.ka_d : (R)A.ka_f;
    const HG<R> hg(sizeof(R) == 8 ? (R)A.g_d : (R)A.g_f);
    SegmentDev *out = T.out + (int64_t)i * T.max_seg;
    if (emit<R, Oct>(A, gid, p, rng, cls, pid, W0)) {
        for (;;) {
            R d;
            const StepOut o = step<R, Oct>(p, A, ks, ka, d);
            if (ns < T.max_seg) {
                out[ns].cell = o.cell;
                out[ns].ds = (double)d;
                out[ns].event = o.event;
                out[ns].pad = 0;
            }
            ++ns;
            if (o.event == kEvScatter) scatter_new_direction<R>(p, rng, A, hg);
            else if (o.event != kEvCross) break;
        }
    }
    T.nseg[i] = ns;
}

hipError_t launch_trace(const McArgs &a, const TraceArgs &t, int precision, hipStream_t s)
{
    const int threads = 64;
    const int blocks = (t.n + threads - 1) / threads;
    const bool oct = a.nlevels > 1;
    if (precision == 1 && oct) hipLaunchKernelGGL((trace_kernel<double, true>), dim3(blocks), dim3(threads), 0, s, a, t);
    else if (precision == 1) hipLaunchKernelGGL((trace_kernel<double, false>), dim3(blocks), dim3(threads), 0, s, a, t);
    else if (oct) hipLaunchKernelGGL((trace_kernel<float, true>), dim3(blocks), dim3(threads), 0, s, a, t);
    else hipLaunchKernelGGL((trace_kernel<float, false>), dim3(blocks), dim3(threads), 0, s, a, t);
    return hipGetLastError();
}

}  // namespace soc
