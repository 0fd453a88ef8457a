// Measurement probes: a plain streaming copy (the HBM roofline and the
// calibration run for the FETCH_SIZE / WRITE_SIZE counters) and a random
// segment gather over a working set of a given size (the roofline of the
// dependent, scattered row reads the NS sampler issues).
#include "sgpm_internal.h"

namespace sgpm {

namespace {

__global__ __launch_bounds__(256) void copy_kernel(const uint4* __restrict__ in, uint4* __restrict__ out, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

__device__ __forceinline__ uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Each group of seg/4 lanes reads one random seg-byte segment (coalesced
// within the segment); rounds dependent reads per group chain the next
// segment index on the data just read, like a walk.
__global__ __launch_bounds__(256) void gather_kernel(const int32_t* __restrict__ a, uint64_t nseg, int lanes_per_seg,
                                                     int rounds, uint64_t seed, unsigned long long* __restrict__ sink) {
    const int lane = (int)(threadIdx.x & 63);
    const int gl = lane % lanes_per_seg;
    const uint64_t gid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / (uint64_t)lanes_per_seg;
    uint64_t h = mix(seed ^ (gid * 0x9E3779B97F4A7C15ull));
    unsigned long long acc = 0;
    for (int r = 0; r < rounds; ++r) {
        const uint64_t s = __umul64hi(h, nseg);
        const int32_t x = a[s * (uint64_t)lanes_per_seg + (uint64_t)gl];
        acc += (unsigned long long)(uint32_t)x;
        h = mix(h + (uint64_t)(uint32_t)__shfl(x, lane - gl));
    }
    if (acc == 0x123456789ull) sink[0] = acc;  // keeps the loads alive
}

}  // namespace

hipError_t probe_copy(const void* in, void* out, uint64_t bytes, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (const uint4*)in, (uint4*)out,
                       bytes / 16);
    return hipGetLastError();
}

hipError_t probe_gather(const int32_t* a, uint64_t words, int seg_bytes, int rounds, int blocks, uint64_t seed,
                        unsigned long long* sink, hipStream_t st) {
    const int lps = seg_bytes / 4;
    const uint64_t nseg = words / (uint64_t)lps;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a, nseg, lps, rounds, seed, sink);
    return hipGetLastError();
}

}  // namespace sgpm
