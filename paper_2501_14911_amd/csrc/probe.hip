// Streaming probes for roofline context: a plain read (non-temporal; each
// wavefront reads 2 KB per access, every load instruction one contiguous
// kilobyte; folded into one word per workgroup so nothing is optimised away)
// and a plain copy.  They give the measured streaming
// bandwidth of the device next to its rated peak, and a kernel of known
// traffic against which hardware byte counters are scaled.
#include "common.hpp"
#include "kernels.hpp"

namespace p2o {

__global__ __launch_bounds__(256) void k_probe_read(const uint8_t* __restrict__ src, long long n32,
                                                    uint32_t* __restrict__ sink) {
    uint32_t acc = 0;
    const long long nchunk = n32 / 64;                    // 2 KB chunks
    const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
    const int lane = threadIdx.x & 63;
    for (long long c = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < nchunk; c += waves) {
        const Raw32 r = load32_split(src + c * 2048 + lane * 16, true, true);
        acc ^= r.a.x ^ r.a.y ^ r.a.z ^ r.a.w ^ r.b.x ^ r.b.y ^ r.b.z ^ r.b.w;
    }
    __shared__ uint32_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] ^= red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_probe_copy(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst,
                                                    long long n16) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
}

hipError_t launch_probe(int mode, const void* src, void* dst, size_t bytes, int blocks, hipStream_t st) {
    if (mode == 0) {
        hipLaunchKernelGGL(k_probe_read, dim3(blocks), dim3(256), 0, st, (const uint8_t*)src, (long long)(bytes / 32),
                           (uint32_t*)dst);
    } else {
        hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, st, (const uint8_t*)src, (uint8_t*)dst,
                           (long long)(bytes / 16));
    }
    return hipGetLastError();
}

}  // namespace p2o
