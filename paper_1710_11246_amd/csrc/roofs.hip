// Microbenchmarks of the slab hash's memory access patterns (random slab reads, random 64-bit
// compare-and-swaps, and a slab read followed by a compare-and-swap into it), measuring the
// ceilings the operation kernels run against. Every address is slab * 32 + word with
// slab < slabs and word < 32, inside the caller's buffer.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "slabhash_roofs.h"

namespace {

constexpr uint32_t kBlock = 256;

__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ uint64_t load_coherent(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t cas(uint64_t *p, uint64_t expected, uint64_t desired)
{
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return expected;
}

// Keeps the loaded values live without a store the compiler could drop; the condition never
// holds for the values these kernels see in practice, and then writes word 0 of the buffer.
__device__ __forceinline__ void sink(uint64_t *buf, uint64_t acc)
{
    if (acc == 0x5EED5EED5EED5EEDull)
        buf[0] = acc;
}

// Two operations per wavefront iteration: lanes 0..31 read slab of op 2p, lanes 32..63 of 2p+1.
template <bool Cas>
__global__ __launch_bounds__(kBlock) void slab_kernel(uint64_t *buf, uint32_t slabs, uint32_t n,
                                                      uint32_t seed)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t pairs = (uint32_t)(((uint64_t)n + 1) / 2);
    uint64_t acc = 0;
    for (uint32_t p = wave; p < pairs; p += nwaves) {
        const uint32_t op = 2 * p + (lane >> 5);
        const bool live = op < n;
        const uint32_t s = __umulhi(mix(seed + op), slabs);
        uint64_t *slab = buf + (size_t)s * 32;
        const uint64_t w = load_coherent(slab + (lane & 31u));
        acc += w;
        if constexpr (Cas) {
            const uint64_t m = __ballot(w == ~0ull);
            const uint32_t hm = (uint32_t)(m >> (lane & 32u)) & 0x7FFFFFFFu;
            if (live && (lane & 31u) == 0)
                acc += cas(slab + (hm ? __builtin_ctz(hm) : 0u), ~0ull, (uint64_t)op);
        }
    }
    sink(buf, acc);
}

// One compare-and-swap per lane per iteration.
__global__ __launch_bounds__(kBlock) void cas_kernel(uint64_t *buf, uint32_t slabs, uint32_t n,
                                                     uint32_t seed)
{
    const uint32_t nt = gridDim.x * blockDim.x;
    uint64_t acc = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nt) {
        const uint32_t h = mix(seed + i);
        uint64_t *p = buf + (size_t)__umulhi(h, slabs) * 32 + (mix(h) & 31u);
        acc += cas(p, ~0ull, (uint64_t)i);
    }
    sink(buf, acc);
}

} // namespace

extern "C" sh_status_t sh_roof_run(int kind, void *d_buf, size_t bytes, uint64_t n_ops,
                                   uint32_t waves_per_cu, uint32_t seed, void *stream)
{
    if (kind < SH_ROOF_SLAB_LOAD || kind > SH_ROOF_LOAD_CAS || !d_buf ||
        (reinterpret_cast<uintptr_t>(d_buf) & 255u) || bytes < 256 || (bytes & 255u) ||
        bytes / 256 > 0xFFFFFFFFull || n_ops >= (1ull << 32) || waves_per_cu > 64)
        return SH_EINVAL;
    if (n_ops == 0)
        return SH_OK;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
        return SH_EHIP;
    const uint32_t wpc = waves_per_cu ? waves_per_cu : 32u;
    const uint32_t blocks = ((uint32_t)ncu * wpc + 3u) / 4u; // four wavefronts per block
    uint64_t *buf = static_cast<uint64_t *>(d_buf);
    const uint32_t slabs = (uint32_t)(bytes / 256), n = (uint32_t)n_ops;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (kind == SH_ROOF_SLAB_LOAD)
        hipLaunchKernelGGL(slab_kernel<false>, dim3(blocks), dim3(kBlock), 0, s, buf, slabs, n,
                           seed);
    else if (kind == SH_ROOF_LOAD_CAS)
        hipLaunchKernelGGL(slab_kernel<true>, dim3(blocks), dim3(kBlock), 0, s, buf, slabs, n,
                           seed);
    else
        hipLaunchKernelGGL(cas_kernel, dim3(blocks), dim3(kBlock), 0, s, buf, slabs, n, seed);
    return hipGetLastError() == hipSuccess ? SH_OK : SH_EHIP;
}
