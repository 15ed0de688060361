// batch.hip -- many independent Monte Carlo problems in one persistent
// launch: every (cloud model, frequency) pair is cut into tiles of package
// ids, and waves pull tiles from one queue.  A wave works on one tile at a
// time: its lanes are refilled from the tile's id range (wave ballot and
// lane rank, as in the single-problem kernel), and once the range is used
// up and every lane has finished, the wave flushes its LDS deposit ring
// into that model's tally and takes the next tile.  The tally is the
// model's array or, with private copies on, a brick-ordered scratch copy
// of it (neighbouring cells in one 64-byte line, so that the transposed
// flush merges their adds), added into the array after the launch by
// batch_fold_kernel.  Pair parameters are read as wave-uniform (scalar)
// data at each tile switch.
//
// Pairs of small grids come first and differently: a workgroup takes a
// whole pair, keeps that grid's absorbed array in LDS, and its waves add
// every deposit there (LDS atomics: ~25x the rate of the memory-side
// global atomics that bound the rest); when the pair is done the
// workgroup adds the LDS array to the model's array, one coalesced add
// per cell.  Then the same LDS serves as the deposit ring of the tiles.
#include <algorithm>

#include "soc_device.h"

namespace soc {

__device__ inline unsigned long long wsum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += (unsigned long long)__shfl_xor((long long)v, o, 64);
    return v;
}
__device__ inline double wsum_f64(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline void batch_add_stats(DevStats *t, unsigned long long pk, unsigned long long st,
                                       unsigned long long sc, unsigned long long ru, double em, double ab, double es)
{
    atomicAdd(&t->packages, pk);
    atomicAdd(&t->steps, st);
    atomicAdd(&t->scatterings, sc);
    atomicAdd(&t->runaways, ru);
    unsafeAtomicAdd(&t->emitted, em);
    unsafeAtomicAdd(&t->absorbed, ab);
    unsafeAtomicAdd(&t->escaped, es);
}

// The pair-invariant fields of the view, and the pair's own fields.
__device__ inline void view_base(BatchView &A, uint32_t iteration, int64_t step_cap)
{
    A.parent = nullptr;
    A.nlevels = 1;
    A.nroot = 0;
    A.level_offset = nullptr;
    A.n_dust = 0;
    A.dust_mode = 1;
    A.dust_L = nullptr;
    A.dust_S = nullptr;
    A.dust_cap = 0.0;
    A.dust_cell = nullptr;
    A.leaves = nullptr;
    A.per_leaf = 1;
    A.iteration = iteration;
    A.step_cap = step_cap;
}

__device__ inline void view_pair(BatchView &A, const PairDev &P)
{
    A.words = P.words;
    A.nx = P.nx; A.ny = P.ny; A.nz = P.nz;
    A.ncells = P.ncells;
    A.n_bg = P.n_bg; A.n_ps_pk = P.n_ps_pk; A.n_total = P.n_total; A.n_ps = P.n_ps;
    A.W_bg = P.W_bg;
    for (int k = 0; k < 6; ++k) A.face_cum[k] = P.face_cum[k];
    A.face_tot = P.face_tot;
    A.ps = P.ps;
    A.key0 = P.key0; A.key1 = P.key1; A.freq_index = P.freq_index;
}

__global__ __launch_bounds__(kMcMaxBlock) void mc_batch_kernel(BatchArgs B)
{
    extern __shared__ double lds_dep[];   // LDS phase: a grid's tally; tiles: [blockDim.x][kRingStride] deposits, then cells
    int32_t *lds_cell = (int32_t *)(lds_dep + kRingStride * blockDim.x);
    __shared__ int32_t sh_pair;                // pair of the LDS phase, workgroup-uniform
    __shared__ unsigned long long sh_next;     // its next unassigned package id
    const int tid = threadIdx.x;
    const int bd = blockDim.x;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t iteration = __builtin_amdgcn_readfirstlane(*B.iteration);
    unsigned long long n_pk = 0, n_st = 0, n_sc = 0, n_ru = 0;
    double e_em = 0.0, e_ab = 0.0, e_es = 0.0;

    // ---- small grids: one whole pair per workgroup, tallied in LDS
    if (B.n_lds_pairs > 0) {
        BatchView A;
        view_base(A, iteration, B.step_cap);
        for (;;) {
            __syncthreads();   // the previous pair's LDS array has been added out
            if (tid == 0) {
                sh_pair = (int32_t)atomicAdd(B.next_lds, 1u);
                sh_next = 0ull;
            }
            __syncthreads();
            const int32_t q = sh_pair;
            if (q >= B.n_lds_pairs) break;
            const PairDev &P = B.pairs[B.lds_pairs[q]];
            view_pair(A, P);
            const int32_t nc = (int32_t)P.ncells;
            for (int32_t c = tid; c < nc; c += bd) lds_dep[c] = 0.0;
            __syncthreads();
            const float ks = P.ks_f, ka = P.ka_f;
            const HG<float> hg(P.g_f);
            Pkg<float> p;
            Rng rng;
            bool active = false, pend = false, exhausted = false;
            unsigned long long pool_next = 0, pool_end = 0;   // wave-uniform
            for (;;) {
                const unsigned long long idle = __ballot(!active);
                const int nidle = __popcll(idle);
                if (!exhausted && nidle > 0 && (nidle >= B.refill_min || nidle == 64)) {
                    const unsigned long long avail = pool_end - pool_next;
                    unsigned long long grant = 0;
                    if (avail < (unsigned long long)nidle) {
                        const int leader = __ffsll((long long)idle) - 1;
                        unsigned long long g0 = 0;
                        if (lane == leader) g0 = atomicAdd(&sh_next, (unsigned long long)B.chunk);
                        grant = (unsigned long long)__shfl((long long)g0, leader, 64);
                    }
                    if (!active) {
                        const unsigned long long r = (unsigned long long)__popcll(idle & below);
                        const unsigned long long id = r < avail ? pool_next + r : grant + (r - avail);
                        if (id < A.n_total) {
                            uint32_t cls, pid;
                            double W0;
                            const bool ok = emit<float, false>(A, id, p, rng, cls, pid, W0);
                            n_pk += 1;
                            if (ok) e_em += W0;
                            active = ok;
                        }
                    }
                    if (avail < (unsigned long long)nidle) {
                        pool_next = grant + ((unsigned long long)nidle - avail);
                        pool_end = grant + (unsigned long long)B.chunk;
                    } else {
                        pool_next += (unsigned long long)nidle;
                    }
                    if (pool_next >= A.n_total) exhausted = true;
                }
                if (!__any(active)) {
                    if (exhausted) break;
                    continue;
                }
                const unsigned long long pm = __ballot(pend);
                if (pm) {
                    if (__popcll(pm) >= B.scatter_min || __ballot(active && !pend) == 0) {
                        if (pend) {
                            scatter_new_direction<float>(p, rng, A, hg);
                            pend = false;
                        }
                    }
                }
                for (int s = 0; s < B.inner_steps; ++s) {
                    if (active && !pend) {
                        float d;
                        const StepOut o = step<float, false>(p, A, ks, ka, d);
                        n_st += 1;
                        if (o.dep != 0.0) {
                            unsafeAtomicAdd(&lds_dep[o.cell], o.dep);
                            e_ab += o.dep;
                        }
                        if (o.event == kEvScatter) {
                            pend = true;
                            n_sc += 1;
                        } else if (o.event != kEvCross) {
                            active = false;
                            if (o.event == kEvEscape) e_es += p.W;
                            if (o.event == kEvRunaway) n_ru += 1;
                        }
                    }
                }
            }
            __syncthreads();   // every wave has finished the pair
            for (int32_t c = tid; c < nc; c += bd) {
                const double v = lds_dep[c];
                if (v != 0.0) unsafeAtomicAdd(&P.absorbed[c], v);
            }
        }
    }

    // ---- tiles of the other pairs, wave by wave, LDS as the deposit ring
    BatchView A;
    view_base(A, iteration, B.step_cap);
    double *tally = nullptr;   // the pair's tile tally: brick-ordered scratch or the model's array
    bool brick = false;
    int32_t hx = 0, hy = 0;
    float ks = 0.0f, ka = 0.0f, gg = 0.0f;

    Pkg<float> p;
    Rng rng;
    bool active = false, pend = false;
    unsigned long long pool_next = 0, pool_end = 0;   // wave-uniform: the current tile's remaining ids
    int nbuf = 0, since_flush = 0;

    for (;;) {
        if (pool_next >= pool_end && !__any(active)) {
            // tile finished: flush its deposits, take the next tile
            flush_rings(lds_dep, lds_cell, nbuf, [&](int32_t c, double v) { unsafeAtomicAdd(&tally[c], v); });
            nbuf = 0;
            since_flush = 0;
            unsigned int t = 0;
            if (lane == 0) t = atomicAdd(B.next_tile, 1u);
            t = __builtin_amdgcn_readfirstlane(__shfl((int)t, 0, 64));
            if ((int32_t)t >= B.n_tiles) break;
            const TileDev tile = B.tiles[t];
            const int32_t pi = __builtin_amdgcn_readfirstlane(tile.pair);
            const PairDev &P = B.pairs[pi];
            view_pair(A, P);
            tally = P.tally;
            brick = P.brick != 0;
            hx = P.nx >> 1;
            hy = P.ny >> 1;
            ks = P.ks_f; ka = P.ka_f; gg = P.g_f;
            pool_next = __builtin_amdgcn_readfirstlane(tile.begin);
            pool_end = __builtin_amdgcn_readfirstlane(tile.end);
            continue;
        }
        const unsigned long long idle = __ballot(!active);
        const int nidle = __popcll(idle);
        if (pool_next < pool_end && nidle > 0 && (nidle >= B.refill_min || nidle == 64)) {
            if (!active) {
                const unsigned long long id = pool_next + (unsigned long long)__popcll(idle & below);
                if (id < pool_end) {
                    uint32_t cls, pid;
                    double W0;
                    const bool ok = emit<float, false>(A, id, p, rng, cls, pid, W0);
                    n_pk += 1;
                    if (ok) e_em += W0;
                    active = ok;
                }
            }
            pool_next += (unsigned long long)nidle;
            if (pool_next > pool_end) pool_next = pool_end;
        }
        if (!__any(active)) continue;
        const HG<float> hg(gg);
        const unsigned long long pm = __ballot(pend);
        if (pm) {
            if (__popcll(pm) >= B.scatter_min || __ballot(active && !pend) == 0) {
                if (pend) {
                    scatter_new_direction<float>(p, rng, A, hg);
                    pend = false;
                }
            }
        }
        if ((since_flush + 1) * B.inner_steps > kDepSlots) {
            flush_rings(lds_dep, lds_cell, nbuf, [&](int32_t c, double v) { unsafeAtomicAdd(&tally[c], v); });
            nbuf = 0;
            since_flush = 0;
        }
        ++since_flush;
        for (int s = 0; s < B.inner_steps; ++s) {
            if (active && !pend) {
                float d;
                const int32_t bcell = brick ? brick_cell(p.cx, p.cy, p.cz, hx, hy) : 0;   // the cell before the step
                const StepOut o = step<float, false>(p, A, ks, ka, d);
                n_st += 1;
                if (o.dep != 0.0) {
                    lds_dep[tid * kRingStride + nbuf] = o.dep;
                    lds_cell[tid * kRingStride + nbuf] = brick ? bcell : o.cell;
                    ++nbuf;
                    e_ab += o.dep;
                }
                if (o.event == kEvScatter) {
                    pend = true;
                    n_sc += 1;
                } else if (o.event != kEvCross) {
                    active = false;
                    if (o.event == kEvEscape) e_es += p.W;
                    if (o.event == kEvRunaway) n_ru += 1;
                }
            }
        }
    }
    n_pk = wsum_u64(n_pk);
    n_st = wsum_u64(n_st);
    n_sc = wsum_u64(n_sc);
    n_ru = wsum_u64(n_ru);
    e_em = wsum_f64(e_em);
    e_ab = wsum_f64(e_ab);
    e_es = wsum_f64(e_es);
    if (lane == 0) {
        batch_add_stats(B.st_call, n_pk, n_st, n_sc, n_ru, e_em, e_ab, e_es);
        batch_add_stats(B.st_total, n_pk, n_st, n_sc, n_ru, e_em, e_ab, e_es);
    }
}

hipError_t launch_mc_batch(const BatchArgs &a, int blocks, int threads, int64_t lds_cells, hipStream_t s)
{
    const size_t ring = (size_t)kRingStride * threads * (sizeof(double) + sizeof(int32_t));
    const size_t tally = a.n_lds_pairs > 0 ? (size_t)lds_cells * sizeof(double) : 0;
    hipLaunchKernelGGL(mc_batch_kernel, dim3(blocks), dim3(threads), ring > tally ? ring : tally, s, a);
    return hipGetLastError();
}

// Brick-ordered tallies into their arrays: blockIdx.y is the tally, the
// x dimension strides over its entries (brick order as fold_copies_kernel).
__global__ void batch_fold_kernel(const BrickFold *folds)
{
    const BrickFold f = folds[blockIdx.y];
    const int32_t hx = f.nx >> 1, hy = f.ny >> 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.ncells;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = f.tally[i];
        if (v == 0.0) continue;
        f.tally[i] = 0.0;
        const int64_t b = i >> 3, bx = b % hx, t = b / hx, by = t % hy, bz = t / hy;
        const int64_t c = ((2 * bz + ((i >> 2) & 1)) * (2 * hy) + 2 * by + ((i >> 1) & 1)) * (2 * hx) + 2 * bx + (i & 1);
        f.absorbed[c] += v;
    }
}

hipError_t launch_batch_fold(const BrickFold *folds, int32_t n, int64_t max_cells, hipStream_t s)
{
    const int64_t bx = std::max<int64_t>(std::min<int64_t>((max_cells + 255) / 256, 256), 1);
    for (int32_t f0 = 0; f0 < n; f0 += 65535) {   // the grid's y dimension holds at most 65535 tallies
        const int32_t nf = std::min<int32_t>(65535, n - f0);
        hipLaunchKernelGGL(batch_fold_kernel, dim3((unsigned)bx, (unsigned)nf), dim3(256), 0, s, folds + f0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// mode 0: set the iteration word to value; mode 1: advance it by one
__global__ void advance_iteration_kernel(uint32_t *it, int32_t mode, uint32_t value)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *it = mode ? *it + 1u : value;
}

hipError_t launch_advance_iteration(uint32_t *it, int32_t mode, uint32_t value, hipStream_t s)
{
    hipLaunchKernelGGL(advance_iteration_kernel, dim3(1), dim3(64), 0, s, it, mode, value);
    return hipGetLastError();
}

}  // namespace soc
