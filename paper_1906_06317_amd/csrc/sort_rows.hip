// Rows of a NeighborList ordered by neighbour index (the paper's promise of
// sorted neighbour order in the Python API, "Implementation"; the analyses do
// not need it, so it is an option of the query).
//
// One wavefront per row, rows dealt to wavefronts in turn.  A row of at
// most kSortLds entries is staged in LDS (indices and distances); each
// entry's place is the number of entries of the row with a smaller index
// (indices are distinct within a row), and the wavefront writes the row back
// in that order.  Longer rows are sorted in place in global memory by a
// bitonic network whose comparators all put the smaller key first, so the
// missing entries of the padded power-of-two length (taken as +infinity)
// never move into the row.
#include "internal.hpp"

namespace ppa {

namespace {

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / kWave;
constexpr int kSortLds = 256;  // entries a wavefront stages in LDS

__device__ __forceinline__ void sort_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Orders a, b (positions in the row, b > a) so the smaller index comes first.
__device__ __forceinline__ void compare_swap(int32_t* idx, float* dist, long long a, long long b)
{
    const int ka = idx[a], kb = idx[b];
    if (kb < ka) {
        idx[a] = kb;
        idx[b] = ka;
        if (dist) {
            const float da = dist[a];
            dist[a] = dist[b];
            dist[b] = da;
        }
    }
}

// In-place bitonic sort of row [e0, e0 + L) in global memory.  For each
// merge size k: first every element of the lower half of a block meets its
// mirror image in the upper half, then half-cleaners at distances k/4 ... 1.
// Partners past the end of the row are +infinity and stay where they are.
__device__ void bitonic_row(int32_t* idx, float* dist, long long e0, long long L, int lane)
{
    int lp = 0;  // P = 2^lp >= L
    while ((1LL << lp) < L) ++lp;
    const long long pairs = 1LL << (lp - 1);
    int32_t* ri = idx + e0;
    float* rd = dist ? dist + e0 : nullptr;
    for (int lk = 1; lk <= lp; ++lk) {  // merge size k = 2^lk
        const long long k = 1LL << lk, hmask = (k >> 1) - 1;
        for (long long t = lane; t < pairs; t += kWave) {
            const long long blk = (t >> (lk - 1)) << lk;
            const long long a = blk + (t & hmask);
            const long long b = blk + (k - 1 - (t & hmask));
            if (b < L) compare_swap(ri, rd, a, b);
        }
        // stores of this step are read by other lanes in the next one
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        for (int lj = lk - 2; lj >= 0; --lj) {  // half-cleaners at distance 2^lj
            const long long j = 1LL << lj;
            for (long long t = lane; t < pairs; t += kWave) {
                const long long a = ((t >> lj) << (lj + 1)) + (t & (j - 1));
                const long long b = a + j;
                if (b < L) compare_swap(ri, rd, a, b);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

__global__ void __launch_bounds__(kSortBlock) sort_rows_kernel(const int64_t* __restrict__ offsets,
                                                               int64_t nq, int32_t* idx,
                                                               float* dist, int64_t capacity)
{
    __shared__ alignas(16) int s_key[kSortWaves][kSortLds];
    __shared__ float s_val[kSortWaves][kSortLds];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    int* key = s_key[wv];
    float* val = s_val[wv];
    const long long nwaves = (long long)gridDim.x * kSortWaves;
    for (long long row = (long long)blockIdx.x * kSortWaves + wv; row < nq; row += nwaves) {
        const long long e0 = offsets[row], e1 = offsets[row + 1];
        // rows the list could not hold (capacity exceeded) stay as they are
        if (e0 < 0 || e1 < e0 || e1 > capacity) continue;
        const long long L = e1 - e0;
        if (L < 2) continue;
        if (L > kSortLds) {
            bitonic_row(idx, dist, e0, L, lane);
            continue;
        }
        const int n = (int)L;
        const int n4 = (n + 3) & ~3;
        for (int e = lane; e < n4; e += kWave) {
            key[e] = e < n ? idx[e0 + e] : 0x7fffffff;  // padding sorts last
            if (dist && e < n) val[e] = dist[e0 + e];
        }
        sort_wave_sync();
        for (int e = lane; e < n; e += kWave) {
            const int mine = key[e];
            int r = 0;
            for (int u = 0; u < n4; u += 4) {
                const int4 v = *reinterpret_cast<const int4*>(&key[u]);
                r += (v.x < mine) + (v.y < mine) + (v.z < mine) + (v.w < mine);
            }
            idx[e0 + r] = mine;
            if (dist) dist[e0 + r] = val[e];
        }
        sort_wave_sync();  // the next row reuses the buffers
    }
}

}  // namespace

void launch_sort_rows(const int64_t* offsets, int64_t nq, int32_t* idx, float* dist,
                      int64_t capacity, hipStream_t s)
{
    if (nq <= 0 || !idx) return;
    const int cus = device_cus();
    long long blocks = (nq + kSortWaves - 1) / kSortWaves;
    const long long cap = 16LL * cus;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(sort_rows_kernel, dim3((unsigned)blocks), dim3(kSortBlock), 0, s, offsets,
                       nq, idx, dist, capacity);
}

}  // namespace ppa
