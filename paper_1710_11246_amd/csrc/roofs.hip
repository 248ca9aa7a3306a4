// Microbenchmarks of the slab hash's memory access patterns (random slab reads, random 64-bit
// compare-and-swaps, a slab read followed by a compare-and-swap into it, and a search and an
// insert whose lists are all one slab long, with their input and result streams), measuring
// the ceilings the operation kernels run against.
// Every address is slab * 32 + word with slab < slabs and word < 32, inside the caller's
// buffer.
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

// A search whose every list is one slab: 2P ops per wavefront iteration. Lanes 0..2P-1 load the
// iteration's keys (one coalesced load); op 2j + h's slab, chosen by a fixed mix of its key, is
// read through the caches by half h (lanes 32h..32h+31) for each pair j, all P loads issued
// before any is used; each half votes on slots 0..30 for its key, and lane 2j + h of the
// iteration writes op 2j + h's value (the high word of the first matching slot, else all ones)
// and found flag, so the results leave in one coalesced store each.
template <int P>
__global__ __launch_bounds__(kBlock) void search_kernel(const uint64_t *__restrict__ buf,
                                                        uint32_t slabs,
                                                        const uint32_t *__restrict__ keys,
                                                        uint32_t n, uint32_t *__restrict__ vout,
                                                        uint8_t *__restrict__ found)
{
    constexpr uint32_t G = 2 * P; // ops per iteration, at most 32
    const uint32_t lane = threadIdx.x & 63u, half = lane >> 5, slot = lane & 31u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t groups = (uint32_t)(((uint64_t)n + G - 1) / G);
    for (uint32_t g = wave; g < groups; g += nwaves) {
        const uint64_t base = (uint64_t)g * G;
        const bool in = lane < G && base + lane < n;
        const uint32_t k = in ? keys[base + lane] : 0u;
        uint64_t w[P];
        uint32_t kq[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            kq[j] = (uint32_t)__shfl((int)k, 2 * j + (int)half, 64);
            const uint32_t s = __umulhi(mix(kq[j]), slabs);
            w[j] = buf[(size_t)s * 32 + slot];
        }
        uint32_t my_v = ~0u, my_f = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint64_t m = __ballot(slot < 31 && (uint32_t)w[j] == kq[j]);
            const uint32_t hm = (uint32_t)(m >> (lane & 32u));
            const uint32_t src = (lane & 32u) | (hm ? (uint32_t)__builtin_ctz(hm) : 0u);
            const uint32_t hv = (uint32_t)__shfl((int)(uint32_t)(w[j] >> 32), (int)src, 64);
            const uint32_t v = hm ? hv : ~0u;
            // lane 2j + h takes half h's result: v is uniform within each half
            const uint32_t vv = (uint32_t)__shfl((int)v, (int)((lane & 1u) << 5), 64);
            const uint32_t ff = (uint32_t)__shfl((int)(hm != 0), (int)((lane & 1u) << 5), 64);
            if ((lane >> 1) == (uint32_t)j) {
                my_v = vv;
                my_f = ff;
            }
        }
        if (in) {
            vout[base + lane] = my_v;
            found[base + lane] = (uint8_t)my_f;
        }
    }
}

// An insert whose key is absent and whose base slab has room, with its input and status
// streams: 2P ops per wavefront iteration. Lanes 0..2P-1 load the iteration's keys and values;
// op 2j + h's slab, chosen by a fixed mix of its key, is read by half h with device-coherent
// loads for each pair j, all P loads issued before any is used; the half's first lane swaps the
// pair into the first all-ones slot of 0..30 (slot 0 if none), and lane 2j + h of the iteration
// writes the op's status (1 if its swap won, else 0).
template <int P>
__global__ __launch_bounds__(kBlock) void insert_kernel(uint64_t *buf, uint32_t slabs,
                                                        const uint32_t *__restrict__ keys,
                                                        const uint32_t *__restrict__ vals,
                                                        uint32_t n, uint8_t *__restrict__ status)
{
    constexpr uint32_t G = 2 * P; // ops per iteration, at most 32
    const uint32_t lane = threadIdx.x & 63u, half = lane >> 5, slot = lane & 31u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t groups = (uint32_t)(((uint64_t)n + G - 1) / G);
    for (uint32_t g = wave; g < groups; g += nwaves) {
        const uint64_t base = (uint64_t)g * G;
        const bool in = lane < G && base + lane < n;
        const uint32_t k = in ? keys[base + lane] : 0u;
        const uint32_t v = in ? vals[base + lane] : 0u;
        uint64_t w[P];
        uint32_t s[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint32_t kq = (uint32_t)__shfl((int)k, 2 * j + (int)half, 64);
            s[j] = __umulhi(mix(kq), slabs);
            w[j] = load_coherent(buf + (size_t)s[j] * 32 + slot);
        }
        uint32_t my_st = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint32_t op = 2 * j + half; // this half's op in the iteration
            const uint64_t m = __ballot(w[j] == ~0ull);
            const uint32_t hm = (uint32_t)(m >> (lane & 32u)) & 0x7FFFFFFFu;
            const uint32_t kq = (uint32_t)__shfl((int)k, (int)op, 64);
            const uint32_t vq = (uint32_t)__shfl((int)v, (int)op, 64);
            uint32_t won = 0;
            if (slot == 0 && base + op < n) {
                const uint64_t pair = ((uint64_t)vq << 32) | kq;
                won = cas(buf + (size_t)s[j] * 32 + (hm ? __builtin_ctz(hm) : 0u), ~0ull, pair) ==
                      ~0ull;
            }
            // lane 2j + h takes half h's status
            const uint32_t st = (uint32_t)__shfl((int)won, (int)((lane & 1u) << 5), 64);
            if ((lane >> 1) == (uint32_t)j)
                my_st = st;
        }
        if (in)
            status[base + lane] = (uint8_t)my_st;
    }
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

extern "C" sh_status_t sh_roof_search(const void *d_buf, size_t bytes, const uint32_t *d_keys,
                                      uint64_t n_ops, uint32_t *d_vals_out, uint8_t *d_found,
                                      uint32_t waves_per_cu, uint32_t depth, void *stream)
{
    if (!d_buf || (reinterpret_cast<uintptr_t>(d_buf) & 255u) || bytes < 256 || (bytes & 255u) ||
        bytes / 256 > 0xFFFFFFFFull || n_ops >= (1ull << 32) - 64 || waves_per_cu > 64 ||
        (depth != 0 && depth != 1 && depth != 4 && depth != 8 && depth != 16) ||
        (n_ops && (!d_keys || !d_vals_out || !d_found)))
        return SH_EINVAL;
    if (n_ops == 0)
        return SH_OK;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
        return SH_EHIP;
    const uint32_t wpc = waves_per_cu ? waves_per_cu : 32u;
    const dim3 grid(((uint32_t)ncu * wpc + 3u) / 4u); // four wavefronts per block
    const uint64_t *buf = static_cast<const uint64_t *>(d_buf);
    const uint32_t slabs = (uint32_t)(bytes / 256), n = (uint32_t)n_ops;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    switch (depth ? depth : 8u) {
    case 1:
        hipLaunchKernelGGL(search_kernel<1>, grid, dim3(kBlock), 0, s, buf, slabs, d_keys, n,
                           d_vals_out, d_found);
        break;
    case 4:
        hipLaunchKernelGGL(search_kernel<4>, grid, dim3(kBlock), 0, s, buf, slabs, d_keys, n,
                           d_vals_out, d_found);
        break;
    case 8:
        hipLaunchKernelGGL(search_kernel<8>, grid, dim3(kBlock), 0, s, buf, slabs, d_keys, n,
                           d_vals_out, d_found);
        break;
    default:
        hipLaunchKernelGGL(search_kernel<16>, grid, dim3(kBlock), 0, s, buf, slabs, d_keys, n,
                           d_vals_out, d_found);
        break;
    }
    return hipGetLastError() == hipSuccess ? SH_OK : SH_EHIP;
}

extern "C" sh_status_t sh_roof_insert(void *d_buf, size_t bytes, const uint32_t *d_keys,
                                      const uint32_t *d_vals, uint64_t n_ops, uint8_t *d_status,
                                      uint32_t waves_per_cu, uint32_t depth, void *stream)
{
    if (!d_buf || (reinterpret_cast<uintptr_t>(d_buf) & 255u) || bytes < 256 || (bytes & 255u) ||
        bytes / 256 > 0xFFFFFFFFull || n_ops >= (1ull << 32) - 64 || waves_per_cu > 64 ||
        (depth != 0 && depth != 1 && depth != 4 && depth != 8 && depth != 16) ||
        (n_ops && (!d_keys || !d_vals || !d_status)))
        return SH_EINVAL;
    if (n_ops == 0)
        return SH_OK;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
        return SH_EHIP;
    const uint32_t wpc = waves_per_cu ? waves_per_cu : 32u;
    const dim3 grid(((uint32_t)ncu * wpc + 3u) / 4u); // four wavefronts per block
    uint64_t *buf = static_cast<uint64_t *>(d_buf);
    const uint32_t slabs = (uint32_t)(bytes / 256), n = (uint32_t)n_ops;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    switch (depth ? depth : 8u) {
    case 1:
        hipLaunchKernelGGL(insert_kernel<1>, grid, dim3(kBlock), 0, s, buf, slabs, d_keys, d_vals,
                           n, d_status);
        break;
    case 4:
        hipLaunchKernelGGL(insert_kernel<4>, grid, dim3(kBlock), 0, s, buf, slabs, d_keys, d_vals,
                           n, d_status);
        break;
    case 8:
        hipLaunchKernelGGL(insert_kernel<8>, grid, dim3(kBlock), 0, s, buf, slabs, d_keys, d_vals,
                           n, d_status);
        break;
    default:
        hipLaunchKernelGGL(insert_kernel<16>, grid, dim3(kBlock), 0, s, buf, slabs, d_keys, d_vals,
                           n, d_status);
        break;
    }
    return hipGetLastError() == hipSuccess ? SH_OK : SH_EHIP;
}
