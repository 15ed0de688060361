// unet.hip -- BF16 MFMA kernels and runtime of the 3-D U-Net surrogate.
//
// Every convolution of the network, forward and backward-data alike, is one
// implicit GEMM: rows are the positions of a "row grid", columns the output
// channels, and the reduction runs over (tap, input channel) pairs.  A
// layer kind only changes how a row maps to input and output positions:
//   3^3 convolution        rows = grid,        input = row + tap - 1,   output = row
//   stride-2 2^3 (down)    rows = coarse grid, input = 2 row + tap,     output = row
//   transposed 2^3 (up)    rows = coarse grid, input = row,             output = 2 row + phase
// (a transposed convolution is eight independent phase GEMMs).  The
// backward-data pass of each kind is again one of these forms with the
// weights re-laid out (flipped taps for the 3^3 convolution, phases and taps
// exchanged between the up and down convolutions).
//
// Each wave computes a 32-row x 32*NT-column tile with
// v_mfma_f32_32x32x16_bf16 (8 BF16 of A and B per lane, 16 FP32 results
// per lane); operands are loaded straight from channels-last tensors as
// 16-byte vectors: 8 consecutive input channels of one position (A) and 8
// consecutive reduction entries of one output channel (B, weights stored
// output-channel-major).  The epilogue adds the bias, applies the leaky
// ReLU, or -- in backward-data passes -- multiplies by the leaky ReLU
// derivative taken from the sign of the stored activation and adds a
// second gradient (the skip connection), then rounds to BF16.
//
// Weight gradients contract over positions: each workgroup reduces a chunk
// of positions for one tap and a 32 x 32 (input, output channel) tile,
// transposing the channels-last tiles through LDS, and writes a partial sum;
// a second kernel adds the partials in a fixed order, so training is
// bit-reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "unet.h"

namespace soc {
namespace unet {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr float kLeak = 0.1f;

__device__ __host__ inline uint16_t f2bf(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __host__ inline float bf2f(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__device__ inline bf16x8_t ld8(const uint16_t *p)
{
    return __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4 *>(p));
}

__device__ inline bf16x8_t zero8()
{
    return __builtin_bit_cast(bf16x8_t, u32x4{0u, 0u, 0u, 0u});
}

// ------------------------------------------------------------------ conv
struct ConvArgs {
    const uint16_t *x;
    int32_t x_cs, x_co, cin;        // input view; cin channels per tap (multiple of 16)
    int32_t iz, iy, ix;             // input grid of one sample
    int32_t mz, my, mx, batch;      // row grid of one sample, samples
    int32_t k, s_in, pad;           // taps per axis, input stride, padding
    int32_t nph, s_out;             // output phases (1 or 8), output stride
    int32_t oz, oy, ox;             // output grid of one sample
    const uint16_t *w;              // [nph][npad][k^3 * cin]
    int32_t npad;
    const float *bias;              // NULL: none
    int32_t cout;                   // columns stored (n < cout)
    int32_t act;                    // 1: leaky ReLU after the bias
    const uint16_t *slope;          // NULL, or multiply by the leaky ReLU derivative at the sign of this tensor
    int32_t sl_cs, sl_co;
    const uint16_t *add;            // NULL, or add this tensor
    int32_t ad_cs, ad_co;
    uint16_t *y;                    // BF16 output view, or
    int32_t y_cs, y_co;
    float *yf;                      // FP32 output (when y is NULL)
    int32_t yf_cs;
};

template <int NT>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int r = lane & 31;
    const uint32_t mtot = (uint32_t)a.batch * a.mz * a.my * a.mx;
    const uint32_t tile = (blockIdx.x * 4u + wave) * 32u;
    const int ph = blockIdx.z;
    const int n0 = blockIdx.y * 32 * NT;
    if (tile >= mtot) return;

    // A operand: this lane's row
    const uint32_t m = tile + r;
    const bool mval = m < mtot;
    int b = 0, qz = 0, qy = 0, qx = 0;
    if (mval) {
        uint32_t t = m;
        qx = t % a.mx;
        t /= a.mx;
        qy = t % a.my;
        t /= a.my;
        qz = t % a.mz;
        b = t / a.mz;
    }
    const int K = a.k * a.k * a.k * a.cin;
    const uint16_t *wrow[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) wrow[s] = a.w + (size_t)(ph * a.npad + n0 + 32 * s + r) * K + 8 * half;

    f32x16_t acc[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s)
        for (int v = 0; v < 16; ++v) acc[s][v] = 0.0f;

    int tap = 0;
    for (int tz = 0; tz < a.k; ++tz)
        for (int ty = 0; ty < a.k; ++ty)
            for (int tx = 0; tx < a.k; ++tx, ++tap) {
                const int zz = a.s_in * qz + tz - a.pad;
                const int yy = a.s_in * qy + ty - a.pad;
                const int xx = a.s_in * qx + tx - a.pad;
                const bool ok = mval && zz >= 0 && zz < a.iz && yy >= 0 && yy < a.iy && xx >= 0 && xx < a.ix;
                const uint16_t *xrow =
                    ok ? a.x + (size_t)(((b * a.iz + zz) * a.iy + yy) * a.ix + xx) * a.x_cs + a.x_co + 8 * half
                       : nullptr;
                const int kb = tap * a.cin;
                for (int c = 0; c < a.cin; c += 16) {
                    const bf16x8_t A = ok ? ld8(xrow + c) : zero8();
#pragma unroll
                    for (int s = 0; s < NT; ++s) {
                        const bf16x8_t B = ld8(wrow[s] + kb + c);
                        acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[s], 0, 0, 0);
                    }
                }
            }

    // epilogue: lane holds column n0 + 32 s + r and rows 8 (v / 4) + 4 half + v % 4
    const int ez = (ph >> 2) & 1, ey = (ph >> 1) & 1, ex = ph & 1;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const uint32_t row = tile + 8 * (v >> 2) + 4 * half + (v & 3);
        if (row >= mtot) continue;
        uint32_t t = row;
        const int px = t % a.mx;
        t /= a.mx;
        const int py = t % a.my;
        t /= a.my;
        const int pz = t % a.mz;
        const int pb = t / a.mz;
        const size_t op =
            (size_t)((pb * a.oz + a.s_out * pz + ez) * a.oy + a.s_out * py + ey) * a.ox + a.s_out * px + ex;
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            const int n = n0 + 32 * s + r;
            if (n >= a.cout) continue;
            float val = acc[s][v];
            if (a.bias) val += a.bias[n];
            if (a.act) val = val > 0.0f ? val : kLeak * val;
            if (a.slope && !(bf2f(a.slope[op * a.sl_cs + a.sl_co + n]) > 0.0f)) val *= kLeak;
            if (a.add) val += bf2f(a.add[op * a.ad_cs + a.ad_co + n]);
            if (a.y)
                a.y[op * a.y_cs + a.y_co + n] = f2bf(val);
            else
                a.yf[op * a.yf_cs + n] = val;
        }
    }
}

// 3^3 convolutions (stride 1, padding 1) -- most of the network's work --
// with the input staged in LDS: a workgroup owns a 4 x 8 x 8 brick of
// output positions (256 rows); for every chunk of 32 input channels it
// loads the 6 x 10 x 10 halo of the brick once (zero outside the volume)
// and all 27 taps read their A fragments from LDS.  Each wave computes two
// 32-row tiles (half z-planes of the brick) x 32*NT columns, so every B
// fragment, shared by the four waves through L1, feeds two MFMAs.
constexpr int kBZ = 4, kBY = 8, kBX = 8;
constexpr int kHZ = kBZ + 2, kHY = kBY + 2, kHX = kBX + 2;
constexpr int kHalo = kHZ * kHY * kHX;   // 600 positions
constexpr int kCC = 32;                  // input channels per LDS chunk
constexpr int kHS = kCC + 8;             // padded position stride in the halo (elements)

template <int NT>
__global__ __launch_bounds__(256) void conv3_lds_kernel(ConvArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t halo[kHalo * kHS];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int half = lane >> 5;
    const int r = lane & 31;
    const int nbx = (a.mx + kBX - 1) / kBX, nby = (a.my + kBY - 1) / kBY, nbz = (a.mz + kBZ - 1) / kBZ;
    int bid = blockIdx.x;
    const int bxi = bid % nbx;
    bid /= nbx;
    const int byi = bid % nby;
    bid /= nby;
    const int bzi = bid % nbz;
    const int b = bid / nbz;
    const int z0 = bzi * kBZ, y0 = byi * kBY, x0 = bxi * kBX;
    const int n0 = blockIdx.y * 32 * NT;
    const int K = 27 * a.cin;

    // this lane's two rows (row tiles 2 wave and 2 wave + 1 of the brick)
    int lz[2], ly[2];
    const int lx = r & 7;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int rt = 2 * wave + t;
        lz[t] = rt >> 1;
        ly[t] = (rt & 1) * 4 + (r >> 3);
    }
    const uint16_t *wrow[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) wrow[s] = a.w + (size_t)(n0 + 32 * s + r) * K + 8 * half;

    f32x16_t acc[2][NT];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int s = 0; s < NT; ++s)
            for (int v = 0; v < 16; ++v) acc[t][s][v] = 0.0f;

    for (int c0 = 0; c0 < a.cin; c0 += kCC) {
        const int cc = min(kCC, a.cin - c0);   // 16 or 32
        const int groups = cc >> 3;
        __syncthreads();   // the previous chunk has been consumed
        for (int i = tid; i < kHalo * groups; i += 256) {
            const int pos = i / groups, g = i - pos * groups;
            const int hx = pos % kHX, hy = (pos / kHX) % kHY, hz = pos / (kHX * kHY);
            const int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (zz >= 0 && zz < a.iz && yy >= 0 && yy < a.iy && xx >= 0 && xx < a.ix)
                v = *reinterpret_cast<const u32x4 *>(
                    a.x + (size_t)(((b * a.iz + zz) * a.iy + yy) * a.ix + xx) * a.x_cs + a.x_co + c0 + 8 * g);
            *reinterpret_cast<u32x4 *>(&halo[pos * kHS + 8 * g]) = v;
        }
        __syncthreads();
        int tap = 0;
        for (int tz = 0; tz < 3; ++tz)
            for (int ty = 0; ty < 3; ++ty)
                for (int tx = 0; tx < 3; ++tx, ++tap) {
                    const int h0 = ((lz[0] + tz) * kHY + ly[0] + ty) * kHX + lx + tx;
                    const int h1 = ((lz[1] + tz) * kHY + ly[1] + ty) * kHX + lx + tx;
                    const int kb = tap * a.cin + c0;
                    for (int cg = 0; cg < cc; cg += 16) {
                        const bf16x8_t A0 =
                            __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4 *>(&halo[h0 * kHS + cg + 8 * half]));
                        const bf16x8_t A1 =
                            __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4 *>(&halo[h1 * kHS + cg + 8 * half]));
#pragma unroll
                        for (int s = 0; s < NT; ++s) {
                            const bf16x8_t B = ld8(wrow[s] + kb + cg);
                            acc[0][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, B, acc[0][s], 0, 0, 0);
                            acc[1][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, B, acc[1][s], 0, 0, 0);
                        }
                    }
                }
    }

    // epilogue: lane holds column n0 + 32 s + r and, in row tile t, the rows
    // 8 (v / 4) + 4 half + v % 4 (= 8 y-rows of 8 x in brick order)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int rt = 2 * wave + t;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = 8 * (v >> 2) + 4 * half + (v & 3);   // 0..31 within the tile
            const int pz = z0 + (rt >> 1), py = y0 + (rt & 1) * 4 + (row >> 3), px = x0 + (row & 7);
            if (pz >= a.mz || py >= a.my || px >= a.mx) continue;
            const size_t op = (size_t)((b * a.oz + pz) * a.oy + py) * a.ox + px;
#pragma unroll
            for (int s = 0; s < NT; ++s) {
                const int n = n0 + 32 * s + r;
                if (n >= a.cout) continue;
                float val = acc[t][s][v];
                if (a.bias) val += a.bias[n];
                if (a.act) val = val > 0.0f ? val : kLeak * val;
                if (a.slope && !(bf2f(a.slope[op * a.sl_cs + a.sl_co + n]) > 0.0f)) val *= kLeak;
                if (a.add) val += bf2f(a.add[op * a.ad_cs + a.ad_co + n]);
                if (a.y)
                    a.y[op * a.y_cs + a.y_co + n] = f2bf(val);
                else
                    a.yf[op * a.yf_cs + n] = val;
            }
        }
    }
}

// The same 3^3 convolution for large grids: an 8 x 8 x 8 brick per
// workgroup (512 rows, halo 10^3 = 1.95x instead of 2.34x), 16 input
// channels per LDS chunk, and four 32-row tiles per wave (two z-planes),
// so every B fragment feeds four MFMAs per column tile.  The x-taps and
// the per-tap channel groups are unrolled so that the weight loads of a
// tap row are issued before its MFMAs.  A halo position is its 16
// channels (32 bytes, two 16-byte units) and a halo row of 10 positions
// is padded to 21 units: the 16 lanes of an operand read that the LDS
// serves together (two x-rows of 8 positions) then fall on 16 different
// units of a 256-byte window, the even ones for one row and the odd ones
// for the other, so the reads are free of bank conflicts; the halo takes
// 33.6 KB, and with at most 128 registers four workgroups share a CU.
constexpr int kB3 = 8;
constexpr int kH3 = kB3 + 2;             // 10
constexpr int kHalo3 = kH3 * kH3 * kH3;  // 1000 positions
constexpr int kCC3 = 16;                 // 32 bytes per position, unpadded
constexpr int kRow3 = kH3 * kCC3 + 8;    // 168 elements per halo row: an odd number of 16-byte units

template <int NT>
__global__ __launch_bounds__(256, 4) void conv3_big_kernel(ConvArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t halo[kH3 * kH3 * kRow3];   // 33600 B
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int half = lane >> 5;
    const int r = lane & 31;
    const int nbx = (a.mx + kB3 - 1) / kB3, nby = (a.my + kB3 - 1) / kB3, nbz = (a.mz + kB3 - 1) / kB3;
    int bid = blockIdx.x;
    const int bxi = bid % nbx;
    bid /= nbx;
    const int byi = bid % nby;
    bid /= nby;
    const int bzi = bid % nbz;
    const int b = bid / nbz;
    const int z0 = bzi * kB3, y0 = byi * kB3, x0 = bxi * kB3;
    const int n0 = blockIdx.y * 32 * NT;
    const int K = 27 * a.cin;

    // row tile t of this wave: z-plane 2 wave + t / 2, y-rows 4 (t % 2) .. +3, x = r % 8
    const int lx = r & 7;
    int hbase[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int lz = 2 * wave + (t >> 1), ly = (t & 1) * 4 + (r >> 3);
        hbase[t] = (lz * kH3 + ly) * kRow3 + lx * kCC3 + 8 * half;
    }
    const uint16_t *wrow[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) wrow[s] = a.w + (size_t)(n0 + 32 * s + r) * K + 8 * half;

    f32x16_t acc[4][NT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < NT; ++s)
            for (int v = 0; v < 16; ++v) acc[t][s][v] = 0.0f;

    for (int c0 = 0; c0 < a.cin; c0 += kCC3) {
        __syncthreads();   // the previous chunk has been consumed
        for (int i = tid; i < kHalo3 * 2; i += 256) {
            const int pos = i >> 1, g = i & 1;
            const int hx = pos % kH3, hy = (pos / kH3) % kH3, hz = pos / (kH3 * kH3);
            const int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (zz >= 0 && zz < a.iz && yy >= 0 && yy < a.iy && xx >= 0 && xx < a.ix)
                v = *reinterpret_cast<const u32x4 *>(
                    a.x + (size_t)(((b * a.iz + zz) * a.iy + yy) * a.ix + xx) * a.x_cs + a.x_co + c0 + 8 * g);
            *reinterpret_cast<u32x4 *>(&halo[(hz * kH3 + hy) * kRow3 + hx * kCC3 + 8 * g]) = v;
        }
        __syncthreads();
        for (int tzy = 0; tzy < 9; ++tzy) {
            const int tz = tzy / 3, ty = tzy % 3;
            const int hoff = (tz * kH3 + ty) * kRow3;
            bf16x8_t B[3][NT];
#pragma unroll
            for (int tx = 0; tx < 3; ++tx)
#pragma unroll
                for (int s = 0; s < NT; ++s) B[tx][s] = ld8(wrow[s] + (tzy * 3 + tx) * a.cin + c0);
#pragma unroll
            for (int tx = 0; tx < 3; ++tx) {
                bf16x8_t A[4];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    A[t] = __builtin_bit_cast(
                        bf16x8_t, *reinterpret_cast<const u32x4 *>(&halo[hbase[t] + hoff + tx * kCC3]));
#pragma unroll
                for (int s = 0; s < NT; ++s)
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[t][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[t], B[tx][s], acc[t][s], 0, 0, 0);
            }
        }
    }

#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = 8 * (v >> 2) + 4 * half + (v & 3);   // 0..31 within the tile: 4 y-rows of 8
            const int pz = z0 + 2 * wave + (t >> 1), py = y0 + (t & 1) * 4 + (row >> 3), px = x0 + (row & 7);
            if (pz >= a.mz || py >= a.my || px >= a.mx) continue;
            const size_t op = (size_t)((b * a.oz + pz) * a.oy + py) * a.ox + px;
#pragma unroll
            for (int s = 0; s < NT; ++s) {
                const int n = n0 + 32 * s + r;
                if (n >= a.cout) continue;
                float val = acc[t][s][v];
                if (a.bias) val += a.bias[n];
                if (a.act) val = val > 0.0f ? val : kLeak * val;
                if (a.slope && !(bf2f(a.slope[op * a.sl_cs + a.sl_co + n]) > 0.0f)) val *= kLeak;
                if (a.add) val += bf2f(a.add[op * a.ad_cs + a.ad_co + n]);
                if (a.y)
                    a.y[op * a.y_cs + a.y_co + n] = f2bf(val);
                else
                    a.yf[op * a.yf_cs + n] = val;
            }
        }
    }
}

// ------------------------------------------------------------------ weight gradient
struct WgradArgs {
    const uint16_t *x;
    int32_t x_cs, x_co, x_c;        // forward input view (x_c channels present, multiple of 8)
    int32_t iz, iy, ix;
    int32_t mz, my, mx, batch;
    int32_t k, s_in, pad;
    int32_t nph, s_out, oz, oy, ox;
    const uint16_t *dy;             // gradient of the pre-activation output
    int32_t dy_cs, dy_co, dy_c;
    int32_t cin, cout;              // real channel counts (stored)
    uint32_t chunk;                 // rows per workgroup (multiple of 256)
    float *part;                    // [chunks][slots][cin][cout]
};

constexpr int kWgStep = 64;   // rows per wave and step

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t xs[4][kWgStep][32];
    __shared__ __attribute__((aligned(16))) uint16_t ds[4][kWgStep][32];
    __shared__ float red[3][64][17];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int r = lane & 31;
    const int ntile_o = (a.cout + 31) / 32;
    const int i0 = (blockIdx.y / ntile_o) * 32;
    const int o0 = (blockIdx.y % ntile_o) * 32;
    const int slot = blockIdx.z;
    const int tap = a.nph > 1 ? 0 : slot;
    const int ph = a.nph > 1 ? slot : 0;
    const int tz = tap / (a.k * a.k), ty = (tap / a.k) % a.k, tx = tap % a.k;
    const int ez = (ph >> 2) & 1, ey = (ph >> 1) & 1, ex = ph & 1;
    const uint32_t mtot = (uint32_t)a.batch * a.mz * a.my * a.mx;
    const uint32_t c_begin = blockIdx.x * a.chunk;
    const uint32_t c_end = min(c_begin + a.chunk, mtot);
    const int cg = (lane & 3) * 8;

    f32x16_t acc;
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;

    for (uint32_t base = c_begin; base < c_end; base += 4 * kWgStep) {
#pragma unroll
        for (int j = 0; j < kWgStep / 16; ++j) {
            const int rr = (lane >> 2) + 16 * j;
            const uint32_t m = base + wave * kWgStep + rr;
            u32x4 vx = {0u, 0u, 0u, 0u}, vd = {0u, 0u, 0u, 0u};
            if (m < c_end) {
                uint32_t t = m;
                const int qx = t % a.mx;
                t /= a.mx;
                const int qy = t % a.my;
                t /= a.my;
                const int qz = t % a.mz;
                const int b = t / a.mz;
                const int zz = a.s_in * qz + tz - a.pad, yy = a.s_in * qy + ty - a.pad, xx = a.s_in * qx + tx - a.pad;
                if (i0 + cg < a.x_c && zz >= 0 && zz < a.iz && yy >= 0 && yy < a.iy && xx >= 0 && xx < a.ix)
                    vx = *reinterpret_cast<const u32x4 *>(
                        a.x + (size_t)(((b * a.iz + zz) * a.iy + yy) * a.ix + xx) * a.x_cs + a.x_co + i0 + cg);
                if (o0 + cg < a.dy_c) {
                    const size_t op = (size_t)((b * a.oz + a.s_out * qz + ez) * a.oy + a.s_out * qy + ey) * a.ox +
                                      a.s_out * qx + ex;
                    vd = *reinterpret_cast<const u32x4 *>(a.dy + op * a.dy_cs + a.dy_co + o0 + cg);
                }
            }
            *reinterpret_cast<u32x4 *>(&xs[wave][rr][cg]) = vx;
            *reinterpret_cast<u32x4 *>(&ds[wave][rr][cg]) = vd;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kWgStep / 16; ++kk) {
            u32x4 pa, pb;
            for (int j = 0; j < 4; ++j) {
                const int q0 = kk * 16 + 8 * half + 2 * j;
                pa[j] = (uint32_t)xs[wave][q0][r] | ((uint32_t)xs[wave][q0 + 1][r] << 16);
                pb[j] = (uint32_t)ds[wave][q0][r] | ((uint32_t)ds[wave][q0 + 1][r] << 16);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, pa),
                                                          __builtin_bit_cast(bf16x8_t, pb), acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // reduce the four waves' tiles in a fixed order
    if (wave > 0)
        for (int v = 0; v < 16; ++v) red[wave - 1][lane][v] = acc[v];
    __syncthreads();
    if (wave == 0) {
        for (int w = 0; w < 3; ++w)
            for (int v = 0; v < 16; ++v) acc[v] += red[w][lane][v];
        const int slots = a.nph > 1 ? a.nph : a.k * a.k * a.k;
        float *out = a.part + ((size_t)blockIdx.x * slots + slot) * a.cin * a.cout;
        for (int v = 0; v < 16; ++v) {
            const int i = i0 + 8 * (v >> 2) + 4 * half + (v & 3);
            const int o = o0 + r;
            if (i < a.cin && o < a.cout) out[(size_t)i * a.cout + o] = acc[v];
        }
    }
}

// Weight gradients of 3^3 convolutions, all 27 taps per workgroup.  The
// workgroup owns a 32 x 32 (input, output channel) tile and a chunk of
// 2 x 8 x 8 position bricks; per brick it stages dy and the 4 x 10 x 10
// input halo in LDS as they are in memory, channels last (one 16-byte
// write per 8 channels of a position).  The MFMA reduction runs over
// positions: one K-step is 16 positions (two x-rows of 8).  Its operands
// need 8 positions of one channel per lane, which the LDS transpose read
// (ds_read_b64_tr_b16) delivers from the channels-last tiles: within each
// group of 16 lanes, lane s gives the address of 4 channels (4 (s mod 4)
// onwards) at position s / 4, and lane i receives channel i at the 4
// positions.  Wave w takes the taps with tz = w; a tap's x-shift is an
// offset of the positions read.
constexpr int kGZ = 2, kGY = 8, kGX = 8;                 // brick
constexpr int kGHZ = kGZ + 2, kGHY = kGY + 2, kGHX = 16;  // halo (x padded to 16)

typedef short s16x4 __attribute__((ext_vector_type(4)));

// 4 positions (pos0 .. pos0 + 3, row stride 32 channels) of the lane's
// channel c0 + (lane mod 16), read transposed from a channels-last tile.
__device__ inline uint2 tr_read4(const uint16_t *tile, int pos0, int c0, int lane)
{
    const int s = lane & 15;
    const uint16_t *p = tile + (pos0 + (s >> 2)) * 32 + c0 + 4 * (s & 3);
    const s16x4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4 *)p);
    return __builtin_bit_cast(uint2, v);
}

__global__ __launch_bounds__(192, 2) void wgrad3_kernel(WgradArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t xL[kGHZ * kGHY * kGHX * 32];   // 40 KB, [hz][hy][hx][ch]
    __shared__ __attribute__((aligned(16))) uint16_t dL[kGZ * kGY * kGX * 32];      // 8 KB, [lz][ly][lx][ch]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int tz = tid >> 6;   // wave = z-tap
    const int half = lane >> 5;
    const int r = lane & 31;
    const int cg = 16 * ((lane >> 4) & 1);   // channel group of the lane's 16-lane group
    const int ntile_o = (a.cout + 31) / 32;
    const int i0 = (blockIdx.y / ntile_o) * 32;
    const int o0 = (blockIdx.y % ntile_o) * 32;
    const int nbx = (a.mx + kGX - 1) / kGX, nby = (a.my + kGY - 1) / kGY, nbz = (a.mz + kGZ - 1) / kGZ;
    const uint32_t nb = (uint32_t)a.batch * nbz * nby * nbx;
    const uint32_t b_begin = blockIdx.x * a.chunk, b_end = min(b_begin + a.chunk, nb);

    // workgroups of the first input-channel tile also sum dy per output
    // channel (the bias gradient): thread (o = tid % 32, part = tid / 32)
    // adds the staged positions part, part + 6, ...
    const bool want_bias = i0 == 0;
    float bsum = 0.0f;

    f32x16_t acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q)
        for (int v = 0; v < 16; ++v) acc[q][v] = 0.0f;

    // The next brick's input halo (the larger tile) is loaded into registers
    // while the current brick is multiplied: 9 16-byte loads per thread
    // (1600 items over 192 threads); the dy tile is loaded when staged.
    constexpr int kDyItems = kGZ * kGY * kGX * 4, kHaloItems = kGHZ * kGHY * 10 * 4;
    constexpr int kHaloPer = (kHaloItems + 191) / 192;
    u32x4 ph[kHaloPer];
    struct Brick { int b, z0, y0, x0; };
    auto brick = [&](uint32_t bi) {
        uint32_t t = bi;
        const int bxi = t % nbx;
        t /= nbx;
        const int byi = t % nby;
        t /= nby;
        const int bzi = t % nbz;
        return Brick{(int)(t / nbz), bzi * kGZ, byi * kGY, bxi * kGX};
    };
    auto load_halo = [&](const Brick &k) {
#pragma unroll
        for (int j = 0; j < kHaloPer; ++j) {
            const int e = tid + 192 * j;
            ph[j] = u32x4{0u, 0u, 0u, 0u};
            const int pos = e >> 2, g = e & 3;
            const int hx = pos % 10, hy = (pos / 10) % kGHY, hz = pos / (10 * kGHY);
            const int zz = k.z0 + hz - 1, yy = k.y0 + hy - 1, xx = k.x0 + hx - 1;
            if (e < kHaloItems && zz >= 0 && zz < a.iz && yy >= 0 && yy < a.iy && xx >= 0 && xx < a.ix &&
                i0 + 8 * g < a.x_c)
                ph[j] = *reinterpret_cast<const u32x4 *>(
                    a.x + (size_t)(((k.b * a.iz + zz) * a.iy + yy) * a.ix + xx) * a.x_cs + a.x_co + i0 + 8 * g);
        }
    };
    if (b_begin < b_end) load_halo(brick(b_begin));
    for (uint32_t bi = b_begin; bi < b_end; ++bi) {
        const Brick k = brick(bi);
        __syncthreads();   // previous brick consumed
        for (int e = tid; e < kDyItems; e += 192) {
            const int pos = e >> 2, g = e & 3;
            const int lx = pos & 7, ly = (pos >> 3) & 7, lz = pos >> 6;
            const int zz = k.z0 + lz, yy = k.y0 + ly, xx = k.x0 + lx;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (zz < a.mz && yy < a.my && xx < a.mx && o0 + 8 * g < a.dy_c)
                v = *reinterpret_cast<const u32x4 *>(
                    a.dy + (size_t)(((k.b * a.oz + zz) * a.oy + yy) * a.ox + xx) * a.dy_cs + a.dy_co + o0 + 8 * g);
            *reinterpret_cast<u32x4 *>(&dL[pos * 32 + 8 * g]) = v;
        }
#pragma unroll
        for (int j = 0; j < kHaloPer; ++j) {
            const int e = tid + 192 * j;
            const int pos = e >> 2;
            const int hx = pos % 10, hy = (pos / 10) % kGHY, hz = pos / (10 * kGHY);
            if (e < kHaloItems) *reinterpret_cast<u32x4 *>(&xL[((hz * kGHY + hy) * kGHX + hx) * 32 + 8 * (e & 3)]) = ph[j];
        }
        __syncthreads();
        if (bi + 1 < b_end) load_halo(brick(bi + 1));
        if (want_bias)
            for (int pos = tid >> 5; pos < kGZ * kGY * kGX; pos += 6) bsum += bf2f(dL[pos * 32 + (tid & 31)]);
        // (the row loop stays rolled: unrolled, the hoisted transpose reads
        // need 336 registers, one wave per SIMD; rolled, 188)
#pragma unroll
        for (int lz = 0; lz < kGZ; ++lz)
#pragma unroll 1
            for (int m = 0; m < kGY / 2; ++m) {
                const int ly = 2 * m + half;   // this lane's x-row of the K-step
                const int drow = (lz * kGY + ly) * kGX;
                const uint2 b0 = tr_read4(dL, drow, cg, lane), b1 = tr_read4(dL, drow + 4, cg, lane);
                const bf16x8_t B = __builtin_bit_cast(bf16x8_t, u32x4{b0.x, b0.y, b1.x, b1.y});
#pragma unroll
                for (int ty = 0; ty < 3; ++ty) {
                    const int xrow = ((lz + tz) * kGHY + ly + ty) * kGHX;
#pragma unroll
                    for (int tx = 0; tx < 3; ++tx) {
                        const uint2 a0 = tr_read4(xL, xrow + tx, cg, lane), a1 = tr_read4(xL, xrow + tx + 4, cg, lane);
                        const bf16x8_t A = __builtin_bit_cast(bf16x8_t, u32x4{a0.x, a0.y, a1.x, a1.y});
                        acc[3 * ty + tx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[3 * ty + tx], 0, 0, 0);
                    }
                }
            }
    }
    // bias partials of this chunk, after all weight partials: the six parts
    // of each output channel added in order
    if (want_bias) {
        __shared__ float bred[6][32];
        bred[tid >> 5][tid & 31] = bsum;
        __syncthreads();
        if (tid < 32 && o0 + tid < a.cout) {
            float t = 0.0f;
            for (int q = 0; q < 6; ++q) t += bred[q][tid];
            const size_t row = (size_t)27 * a.cin * a.cout + a.cout;   // a chunk's weight partials, then its bias partials
            a.part[(size_t)blockIdx.x * row + (size_t)27 * a.cin * a.cout + o0 + tid] = t;
        }
    }
    // partials of this chunk: rows = input channels, columns = output channels
    float *out = a.part + (size_t)blockIdx.x * ((size_t)27 * a.cin * a.cout + a.cout);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int tap = tz * 9 + q;
        for (int v = 0; v < 16; ++v) {
            const int i = i0 + 8 * (v >> 2) + 4 * half + (v & 3);
            const int o = o0 + r;
            if (i < a.cin && o < a.cout) out[((size_t)tap * a.cin + i) * a.cout + o] = acc[q][v];
        }
    }
}

// Sum the chunk partials: g[e] = sum_c part[c][e].  A workgroup takes 32
// consecutive elements; its 8 chunk lanes sum the chunks c = lane mod 8 and
// are then added in lane order, so the result does not depend on timing.
constexpr int kSumElems = 32, kSumLanes = 8;

__global__ __launch_bounds__(256) void sum_chunks_kernel(const float *part, int32_t chunks, int64_t n, float *g)
{
    __shared__ float red[kSumLanes][kSumElems + 1];
    const int ex = threadIdx.x % kSumElems, cl = threadIdx.x / kSumElems;
    const int64_t e = (int64_t)blockIdx.x * kSumElems + ex;
    float s = 0.0f;
    if (e < n)
        for (int c = cl; c < chunks; c += kSumLanes) s += part[(size_t)c * n + e];
    red[cl][ex] = s;
    __syncthreads();
    if (cl == 0 && e < n) {
        float t = 0.0f;
        for (int k = 0; k < kSumLanes; ++k) t += red[k][ex];
        g[e] = t;
    }
}

// Column sums of a channels-last BF16 view over npos positions (bias
// gradients): partial[block][c], then a fixed-order sum.
constexpr int kColBlocks = 512;

__global__ __launch_bounds__(256) void colsum_kernel(const uint16_t *x, int32_t cs, int32_t co, int32_t C,
                                                     uint32_t npos, float *part)
{
    __shared__ float red[256];
    const uint32_t per = (npos + gridDim.x - 1) / gridDim.x;
    const uint32_t p0 = min(blockIdx.x * per, npos), p1 = min(p0 + per, npos);
    if (C <= 256 && 256 % C == 0) {
        // 256 / C position lanes per channel, then a fixed-order sum over them
        const int rows = 256 / C;
        const int c = threadIdx.x % C, rsub = threadIdx.x / C;
        float s = 0.0f;
        for (uint32_t p = p0 + rsub; p < p1; p += rows) s += bf2f(x[(size_t)p * cs + co + c]);
        red[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < C) {
            float t = 0.0f;
            for (int q = 0; q < rows; ++q) t += red[q * C + threadIdx.x];
            part[(size_t)blockIdx.x * C + threadIdx.x] = t;
        }
    } else {
        for (int c = threadIdx.x; c < C; c += 256) {
            float s = 0.0f;
            for (uint32_t p = p0; p < p1; ++p) s += bf2f(x[(size_t)p * cs + co + c]);
            part[(size_t)blockIdx.x * C + c] = s;
        }
    }
}

// ------------------------------------------------------------------ elementwise
// Weight layouts for the GEMMs from the FP32 master weights W[slot][cin][cout]:
//   out[ph][n][t][c], with slot = ph (phase layouts) or t (flipped: T-1-t),
//   value W[slot][c][n] (forward) or W[slot][n][c] (transposed, backward-data).
struct PrepArgs {
    const float *W;
    int32_t cin, cout, nslots;
    uint16_t *out;
    int32_t nph, taps, npad, crow;
    int32_t transposed, flip;
};

// Every layout job of the network in one launch: blockIdx.y is the job,
// the x dimension strides over its elements.
__global__ void prep_weights_kernel(const PrepArgs *jobs)
{
    const PrepArgs a = jobs[blockIdx.y];
    const int64_t total = (int64_t)a.nph * a.npad * a.taps * a.crow;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = e;
        const int c = t % a.crow;
        t /= a.crow;
        const int tap = t % a.taps;
        t /= a.taps;
        const int n = t % a.npad;
        const int ph = t / a.npad;
        const int slot = a.nph > 1 ? ph : (a.flip ? a.nslots - 1 - tap : tap);
        float v = 0.0f;
        if (a.transposed) {
            if (n < a.cin && c < a.cout) v = a.W[((size_t)slot * a.cin + n) * a.cout + c];
        } else {
            if (c < a.cin && n < a.cout) v = a.W[((size_t)slot * a.cin + c) * a.cout + n];
        }
        a.out[e] = f2bf(v);
    }
}

// FP32 [npos][c] -> BF16 [npos][cpad], zero padded.
__global__ void to_bf16_padded_kernel(const float *x, int32_t c, int32_t cpad, int64_t npos, uint16_t *out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npos * cpad) return;
    const int64_t p = e / cpad;
    const int ch = (int)(e % cpad);
    out[e] = ch < c ? f2bf(x[p * c + ch]) : (uint16_t)0;
}

// dy = 2 (y - t) / count, and per-block FP64 partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void mse_kernel(const float *y, const float *t, int64_t count, float *dy,
                                                  double *part)
{
    __shared__ double red[256];
    double s = 0.0;
    const float scale = (float)(2.0 / (double)count);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const float d = y[e] - t[e];
        s += (double)d * d;
        if (dy) dy[e] = scale * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_f64_kernel(const double *part, int32_t n, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        out[0] = s;
    }
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, float lr_t, float b1, float b2,
                            float eps)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr_t * me / (sqrtf(ve) + eps);
}

// He-normal initialisation from a counter hash (splitmix64) and Box-Muller.
__device__ inline uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void init_normal_kernel(float *p, int64_t n, float stddev, uint64_t seed, int64_t offset)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)(offset + e)));
    const double u1 = ((h >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((splitmix64(h) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    p[e] = (float)(stddev * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

__global__ void fill_f32_kernel(float *p, int64_t n, float v)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void fill_u16_kernel(uint16_t *p, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0;
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ------------------------------------------------------------------ runtime
namespace {

int32_t round_up(int32_t v, int32_t m) { return (v + m - 1) / m * m; }
int32_t npad_for(int32_t rows) { return rows >= 64 ? round_up(rows, 64) : round_up(rows, 32); }
int taps_of(Layer::Kind k) { return k == Layer::CONV3 ? 27 : 8; }

}  // namespace

int64_t Net::positions(int level, int32_t n) const
{
    return (int64_t)n * (nz_ >> level) * (ny_ >> level) * (nx_ >> level);
}

// Split-K plan of a layer's weight gradient for a batch of n: 3^3 layers
// reduce bricks of 2 x 8 x 8 positions with all 27 taps per workgroup
// (about 768 workgroups in all); the other kinds reduce rows per tap with
// the generic kernel (about 4096 workgroups).  chunks x taps x cin x cout
// partial sums are written.
Net::WgradPlan Net::plan_wgrad(const Layer &L, int32_t n) const
{
    WgradPlan p;
    const int64_t ctiles = (int64_t)((L.cin + 31) / 32) * ((L.cout + 31) / 32);
    if (L.kind == Layer::CONV3) {
        const int l = L.level_out;
        const int64_t nb = (int64_t)n * (((nz_ >> l) + kGZ - 1) / kGZ) * (((ny_ >> l) + kGY - 1) / kGY) *
                           (((nx_ >> l) + kGX - 1) / kGX);
        // about 512 workgroups in all: two per CU resident at once, one round
        // (measured 4 x 64^3 step: 6.05 ms; 384: 6.22, 768: 6.59, 1024: 6.62)
        int64_t chunks = std::min<int64_t>(nb, std::max<int64_t>(1, 512 / ctiles));
        p.chunk = (uint32_t)((nb + chunks - 1) / chunks);
        p.chunks = (nb + p.chunk - 1) / p.chunk;
        p.bricks = true;
    } else {
        const int64_t rows = L.kind == Layer::UP2 ? positions(L.level_in, n) : positions(L.level_out, n);
        const int64_t tiles = ctiles * taps_of(L.kind);
        int64_t chunks = std::min<int64_t>((rows + 1023) / 1024, std::max<int64_t>(1, 4096 / tiles));
        uint32_t chunk = (uint32_t)((rows + chunks - 1) / chunks);
        p.chunk = (chunk + 255) / 256 * 256;
        p.chunks = (rows + p.chunk - 1) / p.chunk;
        p.bricks = false;
    }
    return p;
}

// The forward and backward-data layout jobs of every layer.
static std::vector<PrepArgs> prep_jobs(const std::vector<Layer> &layers, float *params)
{
    std::vector<PrepArgs> jobs;
    for (const auto &L : layers) {
        const int taps = taps_of(L.kind);
        PrepArgs f{params + L.w_off, L.cin, L.cout, taps, L.wf, 1, taps, L.npad_f, L.cin_buf, 0, 0};
        PrepArgs b{params + L.w_off, L.cin, L.cout, taps, L.wb, 1, taps, L.npad_b, L.cout_buf, 1, 0};
        if (L.kind == Layer::CONV3) {
            b.flip = 1;
        } else if (L.kind == Layer::UP2) {
            f.nph = 8;   // forward: eight phase GEMMs over the input channels
            f.taps = 1;
        } else {
            b.nph = 8;   // down2 backward-data: eight phase GEMMs
            b.taps = 1;
        }
        jobs.push_back(f);
        jobs.push_back(b);
    }
    return jobs;
}

Net::Status Net::create(int dev, int32_t cin, int32_t cout, int32_t base, int32_t levels, int32_t nmax, int32_t nz,
                        int32_t ny, int32_t nx, uint64_t seed, hipStream_t s)
{
    device = dev;
    if (cin < 1 || cout < 1 || base < 16 || base % 16 || levels < 1 || levels > 6 || nmax < 1 || nz < 1 || ny < 1 ||
        nx < 1)
        return {BAD_SHAPE, "bad network shape (base must be a positive multiple of 16, 1 <= levels <= 6)"};
    const int32_t div = 1 << (levels - 1);
    if (nz % div || ny % div || nx % div) return {BAD_SHAPE, "grid dimensions must be divisible by 2^(levels-1)"};
    if ((int64_t)nmax * nz * ny * nx >= (1ll << 31)) return {BAD_SHAPE, "batch x cells must stay below 2^31"};
    if ((int64_t)base << (levels - 1) > 4096) return {BAD_SHAPE, "more than 4096 channels"};
    cin_ = cin;
    cout_ = cout;
    base_ = base;
    levels_ = levels;
    nmax_ = nmax;
    nz_ = nz;
    ny_ = ny;
    nx_ = nx;
    cin_pad_ = round_up(cin, 16);
    cout_pad_ = round_up(cout, 16);
    std::vector<int32_t> ch(levels);
    for (int l = 0; l < levels; ++l) ch[l] = base << l;

    // layers in parameter order
    auto add = [&](Layer::Kind k, const std::string &name, int32_t ci, int32_t co, int32_t ci_buf, int32_t co_buf,
                   int lin, int lout) {
        Layer L;
        L.kind = k;
        L.name = name;
        L.cin = ci;
        L.cout = co;
        L.cin_buf = ci_buf;
        L.cout_buf = co_buf;
        L.level_in = lin;
        L.level_out = lout;
        L.nw = (int64_t)taps_of(k) * ci * co;
        L.w_off = nparam_;
        L.b_off = nparam_ + L.nw;
        nparam_ += L.nw + co;
        layers_.push_back(L);
    };
    int32_t c = cin;
    int32_t cbuf = cin_pad_;
    for (int l = 0; l < levels; ++l) {
        add(Layer::CONV3, "e" + std::to_string(l) + "a", c, ch[l], cbuf, ch[l], l, l);
        add(Layer::CONV3, "e" + std::to_string(l) + "b", ch[l], ch[l], ch[l], ch[l], l, l);
        if (l < levels - 1) {
            add(Layer::DOWN2, "d" + std::to_string(l), ch[l], ch[l + 1], ch[l], ch[l + 1], l, l + 1);
            c = cbuf = ch[l + 1];
        }
    }
    for (int l = levels - 2; l >= 0; --l) {
        add(Layer::UP2, "u" + std::to_string(l), ch[l + 1], ch[l], ch[l + 1], ch[l], l + 1, l);
        add(Layer::CONV3, "q" + std::to_string(l) + "a", 2 * ch[l], ch[l], 2 * ch[l], ch[l], l, l);
        add(Layer::CONV3, "q" + std::to_string(l) + "b", ch[l], ch[l], ch[l], ch[l], l, l);
    }
    add(Layer::CONV3, "out", ch[0], cout, ch[0], cout_pad_, 0, 0);

    auto alloc = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) return nullptr;
        allocs_.push_back(p);
        return p;
    };
#define ALLOC(ptr, type, count)                                              \
    do {                                                                     \
        ptr = (type *)alloc(sizeof(type) * (size_t)(count));                 \
        if (!ptr) return {NO_MEMORY, "device allocation failed"};          \
    } while (0)

    ALLOC(d_params_, float, nparam_);
    ALLOC(d_grads_, float, nparam_);
    ALLOC(d_m_, float, nparam_);
    ALLOC(d_v_, float, nparam_);
    for (auto &L : layers_) {
        const int taps = taps_of(L.kind);
        L.npad_f = npad_for(L.cout);
        L.npad_b = npad_for(L.cin);
        // forward: conv3 and down2 are tap GEMMs, up2 is a phase GEMM; backward the other way round
        ALLOC(L.wf, uint16_t, (size_t)L.npad_f * taps * L.cin_buf);
        ALLOC(L.wb, uint16_t, (size_t)L.npad_b * taps * L.cout_buf);
    }
    ALLOC(d_loss_part_, double, 1024 + 1);
    ALLOC(d_xin_, uint16_t, positions(0, nmax) * cin_pad_);
    ALLOC(d_gy_, uint16_t, positions(0, nmax) * cout_pad_);
    ha_.assign(levels, nullptr);
    cat_.assign(levels, nullptr);
    hd_.assign(levels, nullptr);
    hqa_.assign(levels, nullptr);
    hqb_.assign(levels, nullptr);
    g1_.assign(levels, nullptr);
    g2_.assign(levels, nullptr);
    gcat_.assign(levels, nullptr);
    for (int l = 0; l < levels; ++l) {
        const int64_t P = positions(l, nmax);
        ALLOC(ha_[l], uint16_t, P * ch[l]);
        ALLOC(g1_[l], uint16_t, P * ch[l]);
        ALLOC(g2_[l], uint16_t, P * ch[l]);
        if (l > 0) ALLOC(hd_[l], uint16_t, P * ch[l]);
        if (l < levels - 1) {
            ALLOC(cat_[l], uint16_t, P * 2 * ch[l]);
            ALLOC(gcat_[l], uint16_t, P * 2 * ch[l]);
            ALLOC(hqa_[l], uint16_t, P * ch[l]);
            ALLOC(hqb_[l], uint16_t, P * ch[l]);
        }
    }
    ALLOC(hbot_, uint16_t, positions(levels - 1, nmax) * ch[levels - 1]);
    // split-K partials: the largest chunks x taps x cin x cout of any layer
    // (chunk counts do not decrease with the batch, so nmax bounds them)
    cap_part_ = 0;
    for (auto &L : layers_) cap_part_ = std::max(cap_part_, plan_wgrad(L, nmax).chunks * (L.nw + L.cout));
    ALLOC(d_part_, float, std::max<int64_t>(cap_part_, kColBlocks * 4096));
    {
        const std::vector<PrepArgs> jobs = prep_jobs(layers_, d_params_);
        ALLOC(d_prep_, PrepArgs, jobs.size());
        if (hipMemcpy(d_prep_, jobs.data(), sizeof(PrepArgs) * jobs.size(), hipMemcpyHostToDevice) != hipSuccess)
            return {HIP_ERROR, "weight-layout table upload failed"};
        n_prep_ = (int32_t)jobs.size();
        max_prep_ = 0;
        for (const auto &j : jobs) max_prep_ = std::max<int64_t>(max_prep_, (int64_t)j.nph * j.npad * j.taps * j.crow);
    }
#undef ALLOC

    // He-normal weights, zero biases, zero optimiser state
    for (auto &L : layers_) {
        const float sd = (float)std::sqrt(2.0 / ((double)taps_of(L.kind) * L.cin));
        hipLaunchKernelGGL(init_normal_kernel, dim3(nblk(L.nw)), dim3(256), 0, s, d_params_ + L.w_off, L.nw, sd, seed,
                           L.w_off);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(nblk(L.cout)), dim3(256), 0, s, d_params_ + L.b_off,
                           (int64_t)L.cout, 0.0f);
    }
    hipLaunchKernelGGL(fill_f32_kernel, dim3(nblk(nparam_)), dim3(256), 0, s, d_m_, nparam_, 0.0f);
    hipLaunchKernelGGL(fill_f32_kernel, dim3(nblk(nparam_)), dim3(256), 0, s, d_v_, nparam_, 0.0f);
    hipLaunchKernelGGL(fill_f32_kernel, dim3(nblk(nparam_)), dim3(256), 0, s, d_grads_, nparam_, 0.0f);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = prep_weights(s);
    if (e != hipSuccess) return {HIP_ERROR, hipGetErrorString(e)};
    return {OK, ""};
}

void Net::destroy()
{
    for (void *p : allocs_) (void)hipFree(p);
    allocs_.clear();
    layers_.clear();
}

hipError_t Net::prep_weights(hipStream_t s)
{
    if (n_prep_ == 0) return hipSuccess;
    const int64_t gx = std::min<int64_t>(nblk(max_prep_), 1024);
    hipLaunchKernelGGL(prep_weights_kernel, dim3((unsigned)gx, (unsigned)n_prep_), dim3(256), 0, s,
                       (const PrepArgs *)d_prep_);
    return hipGetLastError();
}

static hipError_t launch_conv(const ConvArgs &a, hipStream_t s)
{
    const uint32_t mtot = (uint32_t)a.batch * a.mz * a.my * a.mx;
    const int nt = a.npad % 64 == 0 ? 2 : 1;
    if (a.k == 3 && a.s_in == 1 && a.pad == 1 && a.nph == 1 && a.s_out == 1 && a.cin % 16 == 0) {
        const unsigned big = (unsigned)a.batch * ((a.mz + kB3 - 1) / kB3) * ((a.my + kB3 - 1) / kB3) *
                             ((a.mx + kB3 - 1) / kB3);
        if (big >= 256) {   // enough 8^3 bricks to fill the device
            // one 32-column tile per wave: with two, the four row tiles'
            // accumulators and operands need ~275 registers, one wave per
            // SIMD, and the step was 2.6% slower
            const dim3 grid(big, a.npad / 32, 1);
            hipLaunchKernelGGL(conv3_big_kernel<1>, grid, dim3(256), 0, s, a);
            return hipGetLastError();
        }
        const unsigned bricks = (unsigned)a.batch * ((a.mz + kBZ - 1) / kBZ) * ((a.my + kBY - 1) / kBY) *
                                ((a.mx + kBX - 1) / kBX);
        // small grids: 32-column tiles give twice the workgroups
        const int ntl = (nt == 2 && bricks * (unsigned)(a.npad / 64) < 512) ? 1 : nt;
        const dim3 grid(bricks, a.npad / (32 * ntl), 1);
        if (ntl == 2)
            hipLaunchKernelGGL(conv3_lds_kernel<2>, grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL(conv3_lds_kernel<1>, grid, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const dim3 grid((mtot + 127) / 128, a.npad / (32 * nt), a.nph);
    if (nt == 2)
        hipLaunchKernelGGL(conv_kernel<2>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(conv_kernel<1>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t Net::conv_fwd(const Layer &L, int32_t n, const View &x, const View &y, float *yf, int32_t yf_cs,
                         hipStream_t s)
{
    ConvArgs a{};
    const int lin = L.level_in, lout = L.level_out;
    a.x = x.p;
    a.x_cs = x.cs;
    a.x_co = x.co;
    a.cin = L.cin_buf;
    a.iz = nz_ >> lin;
    a.iy = ny_ >> lin;
    a.ix = nx_ >> lin;
    a.oz = nz_ >> lout;
    a.oy = ny_ >> lout;
    a.ox = nx_ >> lout;
    a.batch = n;
    if (L.kind == Layer::CONV3) {
        a.mz = a.oz, a.my = a.oy, a.mx = a.ox;
        a.k = 3, a.s_in = 1, a.pad = 1, a.nph = 1, a.s_out = 1;
    } else if (L.kind == Layer::DOWN2) {
        a.mz = a.oz, a.my = a.oy, a.mx = a.ox;
        a.k = 2, a.s_in = 2, a.pad = 0, a.nph = 1, a.s_out = 1;
    } else {
        a.mz = a.iz, a.my = a.iy, a.mx = a.ix;
        a.k = 1, a.s_in = 1, a.pad = 0, a.nph = 8, a.s_out = 2;
    }
    a.w = L.wf;
    a.npad = L.npad_f;
    a.bias = d_params_ + L.b_off;
    a.cout = L.cout;
    a.act = yf ? 0 : 1;
    a.y = yf ? nullptr : y.p;
    a.y_cs = y.cs;
    a.y_co = y.co;
    a.yf = yf;
    a.yf_cs = yf_cs;
    return launch_conv(a, s);
}

hipError_t Net::conv_bwd_data(const Layer &L, int32_t n, const View &dy, const View &slope, const View *add,
                              const View &dx, hipStream_t s)
{
    ConvArgs a{};
    const int lin = L.level_in, lout = L.level_out;
    // the pass reads the output-side gradient and writes the input side
    a.x = dy.p;
    a.x_cs = dy.cs;
    a.x_co = dy.co;
    a.cin = L.cout_buf;
    a.iz = nz_ >> lout;
    a.iy = ny_ >> lout;
    a.ix = nx_ >> lout;
    a.oz = nz_ >> lin;
    a.oy = ny_ >> lin;
    a.ox = nx_ >> lin;
    a.batch = n;
    if (L.kind == Layer::CONV3) {
        a.mz = a.oz, a.my = a.oy, a.mx = a.ox;
        a.k = 3, a.s_in = 1, a.pad = 1, a.nph = 1, a.s_out = 1;
    } else if (L.kind == Layer::DOWN2) {   // dx[2q + e] = dy[q] W[e]^T
        a.mz = a.iz, a.my = a.iy, a.mx = a.ix;
        a.k = 1, a.s_in = 1, a.pad = 0, a.nph = 8, a.s_out = 2;
    } else {                               // dx[q] = sum_e dy[2q + e] W[e]^T
        a.mz = a.oz, a.my = a.oy, a.mx = a.ox;
        a.k = 2, a.s_in = 2, a.pad = 0, a.nph = 1, a.s_out = 1;
    }
    a.w = L.wb;
    a.npad = L.npad_b;
    a.bias = nullptr;
    a.cout = L.cin;
    a.act = 0;
    a.slope = slope.p;
    a.sl_cs = slope.cs;
    a.sl_co = slope.co;
    if (add) {
        a.add = add->p;
        a.ad_cs = add->cs;
        a.ad_co = add->co;
    }
    a.y = dx.p;
    a.y_cs = dx.cs;
    a.y_co = dx.co;
    return launch_conv(a, s);
}

hipError_t Net::conv_wgrad(const Layer &L, int32_t n, const View &x, const View &dy, hipStream_t s)
{
    WgradArgs a{};
    const int lin = L.level_in, lout = L.level_out;
    a.x = x.p;
    a.x_cs = x.cs;
    a.x_co = x.co;
    a.x_c = x.c;
    a.iz = nz_ >> lin;
    a.iy = ny_ >> lin;
    a.ix = nx_ >> lin;
    a.oz = nz_ >> lout;
    a.oy = ny_ >> lout;
    a.ox = nx_ >> lout;
    a.batch = n;
    if (L.kind == Layer::CONV3) {
        a.mz = a.oz, a.my = a.oy, a.mx = a.ox;
        a.k = 3, a.s_in = 1, a.pad = 1, a.nph = 1, a.s_out = 1;
    } else if (L.kind == Layer::DOWN2) {
        a.mz = a.oz, a.my = a.oy, a.mx = a.ox;
        a.k = 2, a.s_in = 2, a.pad = 0, a.nph = 1, a.s_out = 1;
    } else {
        a.mz = a.iz, a.my = a.iy, a.mx = a.ix;
        a.k = 1, a.s_in = 1, a.pad = 0, a.nph = 8, a.s_out = 2;
    }
    a.dy = dy.p;
    a.dy_cs = dy.cs;
    a.dy_co = dy.co;
    a.dy_c = dy.c;
    a.cin = L.cin;
    a.cout = L.cout;
    const int slots = taps_of(L.kind);
    const WgradPlan p = plan_wgrad(L, n);
    if (p.chunks * (L.nw + L.cout) > std::max<int64_t>(cap_part_, kColBlocks * 4096)) return hipErrorInvalidValue;
    a.chunk = p.chunk;
    a.part = d_part_;
    const unsigned ctiles = (unsigned)(((L.cin + 31) / 32) * ((L.cout + 31) / 32));
    if (p.bricks)
        hipLaunchKernelGGL(wgrad3_kernel, dim3((unsigned)p.chunks, ctiles, 1), dim3(192), 0, s, a);
    else
        hipLaunchKernelGGL(wgrad_kernel, dim3((unsigned)p.chunks, ctiles, (unsigned)slots), dim3(256), 0, s, a);
    if (p.bricks) {   // the 27-tap kernel's chunk rows hold the weight, then the bias partials (b_off = w_off + nw)
        hipLaunchKernelGGL(sum_chunks_kernel, dim3(nblk(L.nw + L.cout, kSumElems)), dim3(256), 0, s,
                           (const float *)d_part_, (int32_t)p.chunks, L.nw + L.cout, d_grads_ + L.w_off);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(nblk(L.nw, kSumElems)), dim3(256), 0, s, (const float *)d_part_,
                       (int32_t)p.chunks, L.nw, d_grads_ + L.w_off);
    // bias gradient: column sums of dy over the output positions
    const int64_t npos = positions(lout, n);
    hipLaunchKernelGGL(colsum_kernel, dim3(kColBlocks), dim3(256), 0, s, (const uint16_t *)dy.p, dy.cs, dy.co, L.cout,
                       (uint32_t)npos, d_part_);
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(nblk(L.cout, kSumElems)), dim3(256), 0, s, (const float *)d_part_,
                       (int32_t)kColBlocks, (int64_t)L.cout, d_grads_ + L.b_off);
    return hipGetLastError();
}

hipError_t Net::forward(int32_t n, const float *d_x, float *d_y, hipStream_t s)
{
    if (n < 1 || n > nmax_ || !d_x || !d_y) return hipErrorInvalidValue;
    n_last_ = n;
    const int Lv = levels_;
    std::vector<int32_t> ch(Lv);
    for (int l = 0; l < Lv; ++l) ch[l] = base_ << l;
    const int64_t P0 = positions(0, n);
    hipLaunchKernelGGL(to_bf16_padded_kernel, dim3(nblk(P0 * cin_pad_)), dim3(256), 0, s, d_x, cin_, cin_pad_, P0,
                       d_xin_);
    size_t li = 0;
    View h{d_xin_, cin_pad_, 0, cin_pad_};
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    };
    fin_.assign(layers_.size(), View{});
    fout_.assign(layers_.size(), View{});
    auto conv = [&](const View &x, const View &y, float *yf, int32_t yf_cs) {
        fin_[li] = x;
        fout_[li] = y;
        chk(conv_fwd(layers_[li], n, x, y, yf, yf_cs, s));
        ++li;
    };
    for (int l = 0; l < Lv; ++l) {
        const View a{ha_[l], ch[l], 0, ch[l]};
        conv(h, a, nullptr, 0);
        const View bo = l < Lv - 1 ? View{cat_[l], 2 * ch[l], 0, ch[l]} : View{hbot_, ch[l], 0, ch[l]};
        conv(a, bo, nullptr, 0);
        if (l < Lv - 1) {
            const View d{hd_[l + 1], ch[l + 1], 0, ch[l + 1]};
            conv(bo, d, nullptr, 0);
            h = d;
        }
    }
    View top{hbot_, ch[Lv - 1], 0, ch[Lv - 1]};
    for (int l = Lv - 2; l >= 0; --l) {
        const View uin = top;
        const View cat{cat_[l], 2 * ch[l], 0, 2 * ch[l]};
        conv(uin, cat.at(ch[l], ch[l]), nullptr, 0);
        const View qa{hqa_[l], ch[l], 0, ch[l]};
        conv(cat, qa, nullptr, 0);
        const View qb{hqb_[l], ch[l], 0, ch[l]};
        conv(qa, qb, nullptr, 0);
        top = qb;
    }
    conv(top, View{}, d_y, cout_);
    return e;
}

hipError_t Net::backward(const float *d_dy, hipStream_t s, int32_t stop_layer)
{
    const int32_t n = n_last_;
    if (n < 1 || !d_dy) return hipErrorInvalidValue;
    bdy_.assign(layers_.size(), View{});
    bdx_.assign(layers_.size(), View{});
    const int Lv = levels_;
    std::vector<int32_t> ch(Lv);
    for (int l = 0; l < Lv; ++l) ch[l] = base_ << l;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    };
    // parameter-order indices of the layers
    std::vector<size_t> ea(Lv), eb(Lv), dn(Lv), up(Lv), qa(Lv), qb(Lv);
    size_t li = 0;
    for (int l = 0; l < Lv; ++l) {
        ea[l] = li++;
        eb[l] = li++;
        if (l < Lv - 1) dn[l] = li++;
    }
    for (int l = Lv - 2; l >= 0; --l) {
        up[l] = li++;
        qa[l] = li++;
        qb[l] = li++;
    }
    const size_t out = li;

    // a layer is done once its weight gradient and (if any) backward-data
    // pass are enqueued; stop_layer ends the pass there (test hook)
    bool stop = false;
    auto wgrad = [&](size_t li, const View &x, const View &dy) {
        bdy_[li] = dy;
        chk(conv_wgrad(layers_[li], n, x, dy, s));
        if ((int32_t)li == stop_layer && li == ea[0]) stop = true;
    };
    auto bdata = [&](size_t li, const View &dy, const View &slope, const View *add, const View &dx) {
        bdx_[li] = dx;
        chk(conv_bwd_data(layers_[li], n, dy, slope, add, dx, s));
        if ((int32_t)li == stop_layer) stop = true;
    };
    const int64_t P0 = positions(0, n);
    hipLaunchKernelGGL(to_bf16_padded_kernel, dim3(nblk(P0 * cout_pad_)), dim3(256), 0, s, d_dy, cout_, cout_pad_,
                       P0, d_gy_);
    const View top = Lv == 1 ? View{hbot_, ch[0], 0, ch[0]} : View{hqb_[0], ch[0], 0, ch[0]};
    const View gy{d_gy_, cout_pad_, 0, cout_pad_};
    wgrad(out, top, gy);
    View g{g1_[0], ch[0], 0, ch[0]};
    bdata(out, gy, top, nullptr, g);
    if (stop) return e;
    for (int l = 0; l < Lv - 1; ++l) {
        const View hqa{hqa_[l], ch[l], 0, ch[l]};
        const View cat{cat_[l], 2 * ch[l], 0, 2 * ch[l]};
        const View uin = l == Lv - 2 ? View{hbot_, ch[l + 1], 0, ch[l + 1]} : View{hqb_[l + 1], ch[l + 1], 0, ch[l + 1]};
        wgrad(qb[l], hqa, g);
        const View g2{g2_[l], ch[l], 0, ch[l]};
        bdata(qb[l], g, hqa, nullptr, g2);
        if (stop) return e;
        wgrad(qa[l], cat, g2);
        const View gc{gcat_[l], 2 * ch[l], 0, 2 * ch[l]};
        bdata(qa[l], g2, cat, nullptr, gc);
        if (stop) return e;
        const View gu = gc.at(ch[l], ch[l]);
        wgrad(up[l], uin, gu);
        const View gn{g1_[l + 1], ch[l + 1], 0, ch[l + 1]};
        bdata(up[l], gu, uin, nullptr, gn);
        if (stop) return e;
        g = gn;
    }
    for (int l = Lv - 1; l >= 0; --l) {
        const View ha{ha_[l], ch[l], 0, ch[l]};
        wgrad(eb[l], ha, g);
        const View ga{g2_[l], ch[l], 0, ch[l]};
        bdata(eb[l], g, ha, nullptr, ga);
        if (stop) return e;
        const View in = l == 0 ? View{d_xin_, cin_pad_, 0, cin_pad_} : View{hd_[l], ch[l], 0, ch[l]};
        wgrad(ea[l], in, ga);
        if (stop) return e;
        if (l > 0) {
            const View gd{g1_[l], ch[l], 0, ch[l]};
            bdata(ea[l], ga, in, nullptr, gd);
            if (stop) return e;
            const View skip{cat_[l - 1], 2 * ch[l - 1], 0, ch[l - 1]};
            wgrad(dn[l - 1], skip, gd);
            const View gskip{gcat_[l - 1], 2 * ch[l - 1], 0, ch[l - 1]};
            const View gp{g1_[l - 1], ch[l - 1], 0, ch[l - 1]};
            bdata(dn[l - 1], gd, skip, &gskip, gp);
            if (stop) return e;
            g = gp;
        }
    }
    return e;
}

Net::Status Net::read(int32_t layer, int32_t which, float *h, int64_t count, hipStream_t s)
{
    if (layer < 0 || layer >= (int32_t)layers_.size() || which < 0 || which > 3 || !h || n_last_ < 1)
        return {BAD_SHAPE, "bad layer, tensor or state"};
    const Layer &L = layers_[layer];
    const std::vector<View> &vs = which == 0 ? fin_ : which == 1 ? fout_ : which == 2 ? bdy_ : bdx_;
    if ((size_t)layer >= vs.size() || !vs[layer].p) return {BAD_SHAPE, "tensor not stored"};
    const View v = vs[layer];
    // input-side tensors (forward input, backward-data result) live at the
    // input level with cin channels, output-side ones at the output level
    const bool in_side = which == 0 || which == 3;
    const int32_t c = in_side ? L.cin : L.cout;
    const int64_t npos = positions(in_side ? L.level_in : L.level_out, n_last_);
    if (c > v.c || count != npos * c) return {BAD_SHAPE, "count does not match the tensor"};
    std::vector<uint16_t> tmp((size_t)(npos * v.cs));
    hipError_t e = hipMemcpyAsync(tmp.data(), v.p, tmp.size() * sizeof(uint16_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return {HIP_ERROR, hipGetErrorString(e)};
    for (int64_t p = 0; p < npos; ++p)
        for (int32_t j = 0; j < c; ++j) {
            const uint32_t bits = (uint32_t)tmp[(size_t)(p * v.cs + v.co + j)] << 16;
            float f;
            std::memcpy(&f, &bits, sizeof f);
            h[p * c + j] = f;
        }
    return {OK, ""};
}

hipError_t Net::mse(int32_t n, const float *d_y, const float *d_t, float *d_dy, double *h_loss, hipStream_t s)
{
    if (n < 1 || n > nmax_ || !d_y || !d_t) return hipErrorInvalidValue;
    const int64_t count = positions(0, n) * cout_;
    const int blocks = 1024;
    hipLaunchKernelGGL(mse_kernel, dim3(blocks), dim3(256), 0, s, d_y, d_t, count, d_dy, d_loss_part_);
    hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(64), 0, s, (const double *)d_loss_part_, blocks,
                       d_loss_part_ + 1024);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !h_loss) return e;
    double sum = 0.0;
    e = hipMemcpyAsync(&sum, d_loss_part_ + 1024, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    *h_loss = sum / (double)count;
    return e;
}

hipError_t Net::adam(float lr, float beta1, float beta2, float eps, int32_t step, hipStream_t s)
{
    if (step < 1) return hipErrorInvalidValue;
    const double c1 = 1.0 - std::pow((double)beta1, step);
    const double c2 = 1.0 - std::pow((double)beta2, step);
    // bias-corrected step size; eps scaled so that the update equals m_hat / (sqrt(v_hat) + eps)
    const float lr_t = (float)(lr * std::sqrt(c2) / c1);
    const float eps_t = (float)(eps * std::sqrt(c2));
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(nparam_)), dim3(256), 0, s, d_params_, (const float *)d_grads_, d_m_,
                       d_v_, nparam_, lr_t, beta1, beta2, eps_t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return prep_weights(s);
}

hipError_t Net::zero_grads(hipStream_t s)
{
    hipLaunchKernelGGL(fill_f32_kernel, dim3(nblk(nparam_)), dim3(256), 0, s, d_grads_, nparam_, 0.0f);
    return hipGetLastError();
}

hipError_t Net::set_params(const float *h, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(d_params_, h, sizeof(float) * nparam_, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    return prep_weights(s);
}

hipError_t Net::get_params(float *h, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(h, d_params_, sizeof(float) * nparam_, hipMemcpyDeviceToHost, s);
    return e != hipSuccess ? e : hipStreamSynchronize(s);
}

hipError_t Net::get_grads(float *h, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(h, d_grads_, sizeof(float) * nparam_, hipMemcpyDeviceToHost, s);
    return e != hipSuccess ? e : hipStreamSynchronize(s);
}

int64_t Net::flops_forward(int32_t n) const
{
    int64_t f = 0;
    for (auto &L : layers_) {
        const int64_t rows = positions(L.level_out, n);   // an up convolution: 8 phases x coarse rows
        const int64_t k = L.kind == Layer::CONV3 ? 27 * (int64_t)L.cin : L.kind == Layer::DOWN2 ? 8 * (int64_t)L.cin
                                                                                                 : (int64_t)L.cin;
        f += 2 * rows * k * L.cout;
    }
    return f;
}

}  // namespace unet
}  // namespace soc
