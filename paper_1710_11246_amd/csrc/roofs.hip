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

// P op pairs per wavefront iteration: lanes 0..31 read the slab of op 2p, lanes 32..63 that of
// op 2p+1, for the P pairs p of a group; all P loads are issued before any is used (then, with
// Cas, one swap per op), so P pairs' reads are in flight per wavefront.
template <bool Cas, int P>
__global__ __launch_bounds__(kBlock) void slab_kernel(uint64_t *buf, uint32_t slabs, uint32_t n,
                                                      uint32_t seed)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t pairs = (uint32_t)(((uint64_t)n + 1) / 2);
    const uint32_t groups = (pairs + P - 1) / P;
    uint64_t acc = 0;
    for (uint32_t g = wave; g < groups; g += nwaves) {
        uint64_t w[P];
        uint32_t s[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint32_t op = 2 * (g * P + j) + (lane >> 5); // < 2 * groups * P <= n + 2 P
            s[j] = __umulhi(mix(seed + op), slabs);
            w[j] = load_coherent(buf + (size_t)s[j] * 32 + (lane & 31u));
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            acc += w[j];
            if constexpr (Cas) {
                const uint32_t op = 2 * (g * P + j) + (lane >> 5);
                const uint64_t m = __ballot(w[j] == ~0ull);
                const uint32_t hm = (uint32_t)(m >> (lane & 32u)) & 0x7FFFFFFFu;
                if (op < n && (lane & 31u) == 0)
                    acc += cas(buf + (size_t)s[j] * 32 + (hm ? __builtin_ctz(hm) : 0u), ~0ull,
                               (uint64_t)op);
            }
        }
    }
    sink(buf, acc);
}

// P compare-and-swaps per lane per iteration (ops i, i + nt, ..., issued back to back).
template <int P>
__global__ __launch_bounds__(kBlock) void cas_kernel(uint64_t *buf, uint32_t slabs, uint32_t n,
                                                     uint32_t seed)
{
    const uint32_t nt = gridDim.x * blockDim.x;
    uint64_t acc = 0;
    for (uint64_t i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += (uint64_t)nt * P) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint64_t i = i0 + (uint64_t)j * nt;
            if (i < n) {
                const uint32_t h = mix(seed + (uint32_t)i);
                uint64_t *p = buf + (size_t)__umulhi(h, slabs) * 32 + (mix(h) & 31u);
                acc += cas(p, ~0ull, i);
            }
        }
    }
    sink(buf, acc);
}

template <int P>
void launch_pattern(int kind, dim3 grid, hipStream_t s, uint64_t *buf, uint32_t slabs, uint32_t n,
                    uint32_t seed)
{
    if (kind == SH_ROOF_SLAB_LOAD)
        hipLaunchKernelGGL((slab_kernel<false, P>), grid, dim3(kBlock), 0, s, buf, slabs, n, seed);
    else if (kind == SH_ROOF_LOAD_CAS)
        hipLaunchKernelGGL((slab_kernel<true, P>), grid, dim3(kBlock), 0, s, buf, slabs, n, seed);
    else
        hipLaunchKernelGGL((cas_kernel<P>), grid, dim3(kBlock), 0, s, buf, slabs, n, seed);
}

} // namespace

extern "C" sh_status_t sh_roof_run(int kind, void *d_buf, size_t bytes, uint64_t n_ops,
                                   uint32_t waves_per_cu, uint32_t depth, uint32_t seed,
                                   void *stream)
{
    if (kind < SH_ROOF_SLAB_LOAD || kind > SH_ROOF_LOAD_CAS || !d_buf ||
        (reinterpret_cast<uintptr_t>(d_buf) & 255u) || bytes < 256 || (bytes & 255u) ||
        bytes / 256 > 0xFFFFFFFFull || n_ops >= (1ull << 32) - 64 || waves_per_cu > 64 ||
        (depth != 0 && depth != 1 && depth != 4 && depth != 8 && depth != 16))
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
    switch (depth ? depth : 8u) {
    case 1:
        launch_pattern<1>(kind, dim3(blocks), s, buf, slabs, n, seed);
        break;
    case 4:
        launch_pattern<4>(kind, dim3(blocks), s, buf, slabs, n, seed);
        break;
    case 8:
        launch_pattern<8>(kind, dim3(blocks), s, buf, slabs, n, seed);
        break;
    default:
        launch_pattern<16>(kind, dim3(blocks), s, buf, slabs, n, seed);
        break;
    }
    return hipGetLastError() == hipSuccess ? SH_OK : SH_EHIP;
}
