// gfx950 kernels of libko beyond the simulator: writing sampled launch orders,
// and selecting the smallest values of large device arrays (the orders a
// surrogate scores best; the makespan at a given rank of a full enumeration).
//
// Selection is radix selection on order-preserving unsigned keys: each pass
// counts, among the keys that share the digits fixed so far, how many fall on
// each value of the next 8-bit digit (workgroup-private LDS counters flushed
// with one atomic per nonzero bin); the host walks the counts to fix that
// digit.  After the last pass the k-th smallest key is known exactly.

#include <hip/hip_runtime.h>

#include "ko_device.h"
#include "ko_orders.h"
#include "ko_select.h"

namespace ko {

// ------------------------------------------------------------------ orders

__global__ __launch_bounds__(256) void sample_orders_kernel(uint32_t n, uint32_t set, uint64_t seed,
                                                            uint64_t first, const uint64_t *indices,
                                                            uint64_t count, uint8_t *orders,
                                                            uint8_t *positions)
{
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count)
        return;
    const uint64_t i = indices ? indices[b] : first + b;
    const uint64_t rank = sampled_rank(seed, set, i, n);
    unrank_thread(rank, n, orders ? orders + b * n : nullptr, positions ? positions + b * n : nullptr);
}

// ------------------------------------------------------------------ keys

// float -> unsigned key with the same order (negative values reversed)
__device__ __forceinline__ uint32_t f32_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_f32(uint32_t k)
{
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(u);
}

// int64 -> unsigned key with the same order
__device__ __forceinline__ uint64_t i64_key(int64_t v) { return (uint64_t)v ^ 0x8000000000000000ull; }

template <typename T>
__device__ __forceinline__ uint64_t key_of(const T *src, uint64_t i);

template <>
__device__ __forceinline__ uint64_t key_of<float>(const float *src, uint64_t i)
{
    return f32_key(src[i]);
}

template <>
__device__ __forceinline__ uint64_t key_of<int64_t>(const int64_t *src, uint64_t i)
{
    return i64_key(src[i]);
}

// bins[d] += #{i : (key_i & mask) == prefix and digit (key_i >> shift) & 255 == d}
template <typename T>
__global__ __launch_bounds__(256) void radix_hist_kernel(const T *src, uint64_t count, uint32_t shift,
                                                         uint64_t mask, uint64_t prefix,
                                                         unsigned long long *bins)
{
    __shared__ uint32_t local[256];
    local[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t k = key_of<T>(src, i);
        if ((k & mask) == prefix)
            atomicAdd(&local[(uint32_t)(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t c = local[threadIdx.x];
    if (c)
        atomicAdd(&bins[threadIdx.x], (unsigned long long)c);
}

// Candidates of a float top-k: every index whose key is <= the k-th smallest,
// as (key << 32) | index, appended through an atomic cursor (order arbitrary;
// the caller sorts).  Entries beyond `cap` are counted but not written.
__global__ __launch_bounds__(256) void gather_f32_kernel(const float *src, uint64_t count,
                                                         uint32_t kth_key, uint64_t *out, uint64_t cap,
                                                         unsigned long long *cursor)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint32_t k = f32_key(src[i]);
        if (k <= kth_key) {
            const uint64_t slot = atomicAdd(cursor, 1ull);
            if (slot < cap)
                out[slot] = ((uint64_t)k << 32) | i;
        }
    }
}

__global__ void fill_u64_kernel(uint64_t *p, uint64_t from, uint64_t to, uint64_t value)
{
    const uint64_t i = from + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < to)
        p[i] = value;
}

// One compare-exchange stage (j, k) of the bitonic sorting network over
// keys[0, n), n a power of two: ascending overall.
__global__ void bitonic_stage_kernel(uint64_t *keys, uint64_t n, uint64_t j, uint64_t k)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t l = i ^ j;
    if (l <= i)
        return;
    const uint64_t a = keys[i], b = keys[l];
    const bool up = (i & k) == 0;
    if (up ? (a > b) : (a < b)) {
        keys[i] = b;
        keys[l] = a;
    }
}

__global__ void unpack_topk_kernel(const uint64_t *keys, uint32_t k, int64_t *idx, float *val)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k)
        return;
    const uint64_t c = keys[i];
    if (idx)
        idx[i] = (int64_t)(c & 0xFFFFFFFFull);
    if (val)
        val[i] = key_f32((uint32_t)(c >> 32));
}

// ------------------------------------------------------------------ launchers

namespace {
unsigned blocks_for(uint64_t count, uint64_t cap)
{
    uint64_t b = (count + 255) / 256;
    if (b > cap)
        b = cap;
    return (unsigned)(b ? b : 1);
}
}  // namespace

int launch_sample_orders(uint32_t n, uint32_t set, uint64_t seed, uint64_t first,
                         const uint64_t *indices, uint64_t count, uint8_t *orders, uint8_t *positions,
                         void *stream)
{
    if (count == 0)
        return 0;
    hipLaunchKernelGGL(sample_orders_kernel, dim3(blocks_for(count, 1ull << 31)), dim3(256), 0,
                       (hipStream_t)stream, n, set, seed, first, indices, count, orders, positions);
    return (int)hipGetLastError();
}

int launch_radix_hist_f32(const float *src, uint64_t count, uint32_t shift, uint64_t mask,
                          uint64_t prefix, unsigned long long *bins, int grid_cap, void *stream)
{
    hipLaunchKernelGGL(radix_hist_kernel<float>, dim3(blocks_for(count, (uint64_t)grid_cap)), dim3(256),
                       0, (hipStream_t)stream, src, count, shift, mask, prefix, bins);
    return (int)hipGetLastError();
}

int launch_radix_hist_i64(const int64_t *src, uint64_t count, uint32_t shift, uint64_t mask,
                          uint64_t prefix, unsigned long long *bins, int grid_cap, void *stream)
{
    hipLaunchKernelGGL(radix_hist_kernel<int64_t>, dim3(blocks_for(count, (uint64_t)grid_cap)),
                       dim3(256), 0, (hipStream_t)stream, src, count, shift, mask, prefix, bins);
    return (int)hipGetLastError();
}

int launch_gather_f32(const float *src, uint64_t count, uint32_t kth_key, uint64_t *out, uint64_t cap,
                      unsigned long long *cursor, int grid_cap, void *stream)
{
    hipLaunchKernelGGL(gather_f32_kernel, dim3(blocks_for(count, (uint64_t)grid_cap)), dim3(256), 0,
                       (hipStream_t)stream, src, count, kth_key, out, cap, cursor);
    return (int)hipGetLastError();
}

int launch_bitonic_sort_u64(uint64_t *keys, uint64_t used, uint64_t n_pow2, void *stream)
{
    if (n_pow2 > used) {
        hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n_pow2 - used, 1ull << 31)), dim3(256), 0,
                           (hipStream_t)stream, keys, used, n_pow2, ~0ull);
        int e = (int)hipGetLastError();
        if (e)
            return e;
    }
    for (uint64_t k = 2; k <= n_pow2; k <<= 1)
        for (uint64_t j = k >> 1; j > 0; j >>= 1) {
            hipLaunchKernelGGL(bitonic_stage_kernel, dim3(blocks_for(n_pow2, 1ull << 31)), dim3(256), 0,
                               (hipStream_t)stream, keys, n_pow2, j, k);
            int e = (int)hipGetLastError();
            if (e)
                return e;
        }
    return 0;
}

int launch_unpack_topk(const uint64_t *keys, uint32_t k, int64_t *idx, float *val, void *stream)
{
    if (k == 0)
        return 0;
    hipLaunchKernelGGL(unpack_topk_kernel, dim3((k + 255) / 256), dim3(256), 0, (hipStream_t)stream, keys,
                       k, idx, val);
    return (int)hipGetLastError();
}

}  // namespace ko
