// Measurement hooks: LDS and global-memory atomic throughput of this device,
// the references the histogram kernels' binning rates are reported against.
// Every lane adds 1 to pseudo-random bins of a histogram (32-bit atomics),
// per workgroup in LDS or shared by the whole grid in device memory, from
// indices held in registers so that address arithmetic, not the
// random-number generator, accompanies each atomic.
#include "internal.hpp"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeStreams = 8;  // independent index streams per lane

__global__ void __launch_bounds__(kProbeBlock) lds_atomic_probe_kernel(int mask, int iters,
                                                                       unsigned* out)
{
    extern __shared__ unsigned h[];
    for (int b = threadIdx.x; b <= mask; b += kProbeBlock) h[b] = 0u;
    __syncthreads();
    // a fixed odd stride per stream walks every bin; starts differ per lane
    unsigned x = (blockIdx.x * kProbeBlock + threadIdx.x) * 2654435761u;
    unsigned idx[kProbeStreams];
#pragma unroll
    for (int s = 0; s < kProbeStreams; ++s) {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        idx[s] = x;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int s = 0; s < kProbeStreams; ++s) {
            atomicAdd(&h[idx[s] & (unsigned)mask], 1u);
            idx[s] += 2 * s + 40503u;
        }
    }
    __syncthreads();
    unsigned sum = 0;
    for (int b = threadIdx.x; b <= mask; b += kProbeBlock) sum += h[b];
    if (sum) atomicAdd(out, sum);
}

// Global atomics without return value into hist[0 .. mask] (device memory).
__global__ void __launch_bounds__(kProbeBlock) global_atomic_probe_kernel(unsigned mask, int iters,
                                                                          unsigned* hist)
{
    unsigned x = (blockIdx.x * kProbeBlock + threadIdx.x) * 2654435761u + 12345u;
    unsigned idx[kProbeStreams];
#pragma unroll
    for (int s = 0; s < kProbeStreams; ++s) {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        idx[s] = x;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int s = 0; s < kProbeStreams; ++s) {
            atomicAdd(&hist[idx[s] & mask], 1u);
            idx[s] += 2 * s + 40503u;
        }
    }
}

}  // namespace

extern "C" int ppa_probe_lds_atomics(int32_t log2_bins, int32_t iters, int32_t blocks,
                                     uint32_t* out_dev, hipStream_t stream)
{
    if (log2_bins < 1 || log2_bins > 14 || iters < 1 || blocks < 1 || !out_dev)
        return ppa::set_error(PPA_EINVAL, "need 1 <= log2_bins <= 14, iters >= 1, blocks >= 1");
    const int mask = (1 << log2_bins) - 1;
    hipLaunchKernelGGL(lds_atomic_probe_kernel, dim3(blocks), dim3(kProbeBlock),
                       sizeof(unsigned) * (size_t)(mask + 1), stream, mask, iters,
                       (unsigned*)out_dev);
    return ppa::hip_check(hipGetLastError(), "kernel launch");
}

extern "C" int ppa_probe_global_atomics(int32_t log2_words, int32_t iters, int32_t blocks,
                                        uint32_t* hist_dev, hipStream_t stream)
{
    if (log2_words < 1 || log2_words > 28 || iters < 1 || blocks < 1 || !hist_dev)
        return ppa::set_error(PPA_EINVAL, "need 1 <= log2_words <= 28, iters >= 1, blocks >= 1");
    const unsigned mask = (1u << log2_words) - 1u;
    hipLaunchKernelGGL(global_atomic_probe_kernel, dim3(blocks), dim3(kProbeBlock), 0, stream, mask,
                       iters, (unsigned*)hist_dev);
    return ppa::hip_check(hipGetLastError(), "kernel launch");
}
