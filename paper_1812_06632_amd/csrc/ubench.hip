// ubench.hip -- micro-benchmarks that measure the ceilings the Monte Carlo
// kernel is bounded by on this device: FP64 atomic adds (random addresses
// in an array shared by all XCDs or in one private slice per XCD chosen by
// the hardware XCC id, wave-coalesced blocks, or an LDS array), dependent
// random 4-byte gathers, and a plain streaming copy (the reference for HBM
// traffic counters).
#include <hip/hip_runtime.h>

#include "soc_device.h"

namespace soc {

__device__ inline uint32_t mix32(uint32_t x)
{
    // integer hash (xorshift-multiply), a cheap address scrambler
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// mode 0: random addresses in one array shared by every XCD;
// mode 1: random addresses in slice xcd_index() of 8 (per-XCD private copies);
// mode 2: wave-coalesced, every wave updating the 64 consecutive doubles of
//         one random 64-double block (n >= 64);
// mode 3: random addresses in a 4096-double LDS array of the workgroup
//         (the LDS sum is folded into a[0..4095] at the end; n >= 4096);
// mode 4: random FP32 atomic adds into n floats;
// mode 5: random 64-bit integer atomic adds into n words;
// mode 6: random 32-bit integer atomic adds into n words.
constexpr int kUbLds = 4096;

__global__ void ubench_atomic_kernel(double *a, uint32_t n, int32_t per_thread, int32_t mode)
{
    __shared__ double lds[kUbLds];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u;
    double *base = mode == 1 ? a + (size_t)xcd_index() * n : a;
    if (mode == 3) {
        for (int i = threadIdx.x; i < kUbLds; i += blockDim.x) lds[i] = 0.0;
        __syncthreads();
    }
    uint32_t h = tid * 0x9E3779B9u + 1u;
    for (int i = 0; i < per_thread; ++i) {
        h = mix32(h + (uint32_t)i);
        if (mode == 2) {
            const uint32_t blk = __builtin_amdgcn_readfirstlane(h) % (n >> 6);
            unsafeAtomicAdd(&base[blk * 64u + lane], 1.0);
        } else if (mode == 3) {
            unsafeAtomicAdd(&lds[h & (kUbLds - 1)], 1.0);
        } else if (mode == 4) {
            unsafeAtomicAdd(&((float *)a)[h % n], 1.0f);
        } else if (mode == 5) {
            atomicAdd(&((unsigned long long *)a)[h % n], 1ull);
        } else if (mode == 6) {
            atomicAdd(&((unsigned int *)a)[h % n], 1u);
        } else {
            unsafeAtomicAdd(&base[h % n], 1.0);
        }
    }
    if (mode == 3) {
        __syncthreads();
        for (int i = threadIdx.x; i < kUbLds; i += blockDim.x) unsafeAtomicAdd(&a[i], lds[i]);
    }
}

__global__ void ubench_gather_kernel(const uint32_t *w, uint32_t n, int32_t per_thread, uint32_t *out)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t h = mix32(tid + 12345u) % n;
    uint32_t acc = 0;
    for (int i = 0; i < per_thread; ++i) {
        const uint32_t v = w[h];
        acc += v;
        h = mix32(h ^ v) % n;   // dependent chain: the next address needs this load
    }
    if (acc == 0xFFFFFFFFu) out[0] = acc;
}

__global__ void ubench_copy_kernel(const float4 *src, float4 *dst, size_t n4)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_ubench(int32_t which, void *buf, void *buf2, uint64_t n, int32_t per_thread, int32_t mode,
                         int blocks, int threads, hipStream_t s)
{
    if (which == 0)
        hipLaunchKernelGGL(ubench_atomic_kernel, dim3(blocks), dim3(threads), 0, s, (double *)buf, (uint32_t)n,
                           per_thread, mode);
    else if (which == 1)
        hipLaunchKernelGGL(ubench_gather_kernel, dim3(blocks), dim3(threads), 0, s, (const uint32_t *)buf,
                           (uint32_t)n, per_thread, (uint32_t *)buf2);
    else
        hipLaunchKernelGGL(ubench_copy_kernel, dim3(blocks), dim3(threads), 0, s, (const float4 *)buf,
                           (float4 *)buf2, (size_t)(n / 16));
    return hipGetLastError();
}

}  // namespace soc
