// stream.hip -- streaming kernels of exactly known traffic: a copy (every
// byte read once and written once), a read-only pass (XOR checksums of 8 KiB
// blocks, so the loads cannot be dropped; its writes are 1/512 of its reads)
// and a write-only fill, all with 128-bit accesses. They measure the HBM
// bandwidth a kernel can attain on the device, against which the step
// kernels are judged, and they calibrate the profiler's byte counters (a
// launch of known size).
//
// Shape: one 16-byte word per thread (two for the read pass) over a flat grid
// of as many workgroups as the data needs. Measured on the MI355X with 2 GiB
// buffers: copy 6.1 TB/s, read 6.8 TB/s; grid-stride loops over a persistent
// grid of 4-16 workgroups per compute unit reached only 4.4-4.9 (copy) and
// 5.3-6.2 TB/s (read), unrolled 2-16 deep, with or without non-temporal hints.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cdi.h"
#include "cdi_internal.h"

namespace cdi {

namespace {

constexpr int kStreamThreads = 256;
constexpr int kReadWords = 2;  // 16-byte words per thread of the read pass: 8 KiB per workgroup

__device__ inline uint4 xor4(uint4 a, uint4 b) { return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w); }

__global__ __launch_bounds__(kStreamThreads) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                              uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * kStreamThreads + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(kStreamThreads) void fill_kernel16(uint4 *__restrict__ dst, uint64_t n, uint32_t value)
{
    const uint64_t i = (uint64_t)blockIdx.x * kStreamThreads + threadIdx.x;
    if (i < n) dst[i] = make_uint4(value, value, value, value);
}

// dst[b] = XOR of the words of block b (kReadWords * kStreamThreads words).
__global__ __launch_bounds__(kStreamThreads) void xor_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                             uint64_t n)
{
    __shared__ uint4 part[kStreamThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * (kReadWords * kStreamThreads) + threadIdx.x;
    uint4 v[kReadWords];
#pragma unroll
    for (int u = 0; u < kReadWords; ++u) {
        const uint64_t i = base + (uint64_t)u * kStreamThreads;
        v[u] = i < n ? src[i] : make_uint4(0, 0, 0, 0);
    }
    uint4 acc = v[0];
#pragma unroll
    for (int u = 1; u < kReadWords; ++u) acc = xor4(acc, v[u]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc.x ^= __shfl_xor(acc.x, off, 64);
        acc.y ^= __shfl_xor(acc.y, off, 64);
        acc.z ^= __shfl_xor(acc.z, off, 64);
        acc.w ^= __shfl_xor(acc.w, off, 64);
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint4 s = part[0];
#pragma unroll
        for (int w = 1; w < kStreamThreads / 64; ++w) s = xor4(s, part[w]);
        dst[blockIdx.x] = s;
    }
}

}  // namespace

hipError_t launch_stream(int mode, void *dst, const void *src, uint64_t bytes, uint32_t value, hipStream_t s)
{
    const uint64_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const uint4 *in = reinterpret_cast<const uint4 *>(src);
    uint4 *out = reinterpret_cast<uint4 *>(dst);
    const uint64_t per = mode == kStreamRead ? (uint64_t)kReadWords * kStreamThreads : kStreamThreads;
    const uint64_t blocks = (n + per - 1) / per;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    switch (mode) {
    case kStreamCopy: copy_kernel<<<(unsigned)blocks, kStreamThreads, 0, s>>>(in, out, n); break;
    case kStreamRead: xor_kernel<<<(unsigned)blocks, kStreamThreads, 0, s>>>(in, out, n); break;
    default: fill_kernel16<<<(unsigned)blocks, kStreamThreads, 0, s>>>(out, n, value); break;
    }
    return hipGetLastError();
}

}  // namespace cdi
