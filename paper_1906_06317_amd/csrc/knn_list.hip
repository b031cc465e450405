// k nearest neighbours selected from a stored ball NeighborList (the paper's
// reuse of a NeighborList across analyses, "Implementation"): each row of the
// list keeps its k entries of smallest (distance, point index), in that
// order.  When every row of a ball list with cutoff r_max holds at least k
// entries, this is the k-nearest query itself (no point outside the ball
// can be nearer); otherwise it is the k-nearest query with a guard at r_max.
//
// One wavefront per list row; the wavefronts take consecutive rows, so a
// row's threshold guess is the previous row's k-th distance.  A threshold T
// with want <= #{d < T} <= 64 (256 when many distances tie) is found by
// counting ballots over the row (held in registers up to 256 entries,
// re-read from cache per refinement beyond), the entries under T are compacted into LDS as 64-bit keys (distance bits,
// index) — non-negative float distances order like their bit patterns — and
// each lane ranks its keys among them.
#include "internal.hpp"

namespace ppa {

namespace {

constexpr int kKlBlock = 256;
constexpr int kKlWaves = kKlBlock / kWave;
constexpr int kKlBuf = 256;  // keys a row may leave under its threshold
constexpr int kKlIter = 40;  // threshold refinements before giving up
constexpr unsigned long long kNoKey = ~0ull;

__device__ __forceinline__ unsigned long long kl_key(float d, int id)
{
    return ((unsigned long long)__float_as_uint(d) << 32) | (unsigned)id;
}

// Number of row entries with distance below T (uniform across the wave).
__device__ __forceinline__ int kl_count(const float* __restrict__ dist, long long e0, int L,
                                        float T, int lane)
{
    int c = 0;
    for (int b = 0; b < L; b += kWave) {
        const int e = b + lane;
        const bool h = e < L && dist[e0 + e] < T;
        c += __popcll(__ballot(h));
    }
    return c;
}

// Next threshold of the refinement: up when too few entries lie below T,
// down when too many (bisection once both sides are known).
__device__ __forceinline__ float kl_refine(int cnt, int want, float& lo, float& hi, float T)
{
    if (cnt < want) {
        lo = T;
        return hi < INFINITY ? 0.5f * (T + hi) : (T > 0.f ? 2.f * T : 1.f);
    }
    hi = T;
    return 0.5f * (lo + T);
}

template <int NS>
__device__ __forceinline__ void kl_row(const KnnListArgs& a, long long row, long long e0, int L,
                                       int want, float& guess, unsigned long long* key, int lane)
{
    // the row in registers (NS > 0: rows of up to 64 NS entries), else re-read
    float d[NS > 0 ? NS : 1];
    int id[NS > 0 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int e = s * kWave + lane;
        d[s] = INFINITY;
        id[s] = 0;
        if (e < L) {
            d[s] = a.dist[e0 + e];
            id[s] = a.idx[e0 + e];
        }
    }
    auto count = [&](float T) {
        int c = 0;
        if (NS > 0) {
#pragma unroll
            for (int s = 0; s < NS; ++s) c += __popcll(__ballot(d[s] < T));
        } else {
            c = kl_count(a.dist, e0, L, T, lane);
        }
        return c;
    };
    // threshold: every entry of a row of at most 64, else refine T until
    // want <= #{d < T} <= 64 (after kKlIter / 2 tries, <= kKlBuf, for rows
    // with many equal distances)
    float T = INFINITY;
    if (L > kWave) {
        float lo = 0.f, hi = INFINITY;
        if (guess > 0.f) {
            T = guess * 1.05f;
        } else {
            // no previous row: start from half the row's largest distance
            float m = 0.f;
            for (int b = lane; b < L; b += kWave) m = fmaxf(m, a.dist[e0 + b]);
            for (int sh = 32; sh > 0; sh >>= 1) m = fmaxf(m, __shfl_xor(m, sh));
            T = m > 0.f ? 0.5f * m : 1.f;
        }
        bool ok = false;
        for (int it = 0; it < kKlIter; ++it) {
            const int cnt = count(T);
            const int cap = it < kKlIter / 2 ? kWave : kKlBuf;
            if (cnt >= want && cnt <= cap) {
                ok = true;
                break;
            }
            T = kl_refine(cnt, want, lo, hi, T);
        }
        if (!ok) {  // more than kKlBuf entries tie at the k-th distance
            if (lane == 0) {
                atomicOr(a.status, kStatusTies);
                a.row_len[row] = 0;
            }
            return;
        }
    }
    // compact the keys under T (from the registers, or re-read)
    int nb = 0;
    auto compact = [&](float dv, int iv) {
        const bool h = dv < T;
        const unsigned long long m = __ballot(h);
        if (h) {
            const unsigned below = __builtin_amdgcn_mbcnt_hi(
                (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            key[nb + (int)below] = kl_key(dv, iv);
        }
        nb += __popcll(m);
    };
    if constexpr (NS > 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) compact(d[s], id[s]);
    } else {
        for (int b = 0; b < L; b += kWave) {
            const int e = b + lane;
            compact(e < L ? a.dist[e0 + e] : INFINITY, e < L ? a.idx[e0 + e] : 0);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // each lane ranks its keys (lane, lane + 64, ...) among the nb keys
    unsigned long long kth = kNoKey;
    for (int t = lane; t < nb; t += kWave) {
        const unsigned long long mine = key[t];
        int r = 0;
        int u = 0;
        for (; u + 1 < nb; u += 2) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(&key[u]);
            r += (v.x < mine ? 1 : 0) + (v.y < mine ? 1 : 0);
        }
        if (u < nb) r += key[u] < mine ? 1 : 0;
        if (r < want) {
            const long long o = (long long)a.k * row + r;
            a.out_idx[o] = (int)(unsigned)mine;
            a.out_dist[o] = __uint_as_float((unsigned)(mine >> 32));
        }
        if (r == want - 1) kth = mine;
    }
    // the k-th distance seeds the next row's threshold
    unsigned long long kmin = kth;
    for (int sh = 32; sh > 0; sh >>= 1) {
        const unsigned long long o = __shfl_xor(kmin, sh);
        kmin = o < kmin ? o : kmin;
    }
    guess = __uint_as_float((unsigned)(kmin >> 32));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(kKlBlock) knn_list_kernel(const KnnListArgs a)
{
    __shared__ alignas(16) unsigned long long s_key[kKlWaves][kKlBuf];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    unsigned long long* key = s_key[wv];
    const long long nwaves = (long long)gridDim.x * kKlWaves;
    const long long w = (long long)blockIdx.x * kKlWaves + wv;
    const long long per = (a.nq + nwaves - 1) / nwaves;
    const long long r0 = w * per;
    const long long r1 = r0 + per < a.nq ? r0 + per : a.nq;
    float guess = 0.f;  // previous row's k-th distance (0: none yet)
    for (long long row = r0; row < r1; ++row) {
        long long e0 = a.offsets[row], e1 = a.offsets[row + 1];
        if (e0 < 0 || e1 < e0 || e1 > a.capacity || e1 - e0 > 0x7fffffffLL) {
            if (lane == 0) atomicOr(a.status, kStatusBadList);
            e0 = e1 = 0;
        }
        const int L = (int)(e1 - e0);
        const int want = L < a.k ? L : a.k;
        if (lane == 0) a.row_len[row] = want;
        if (want == 0) continue;
        if (L <= kWave)
            kl_row<1>(a, row, e0, L, want, guess, key, lane);
        else if (L <= 2 * kWave)
            kl_row<2>(a, row, e0, L, want, guess, key, lane);
        else if (L <= 4 * kWave)
            kl_row<4>(a, row, e0, L, want, guess, key, lane);
        else
            kl_row<0>(a, row, e0, L, want, guess, key, lane);
    }
}

__global__ void __launch_bounds__(256) kl_zero_kernel(unsigned* p, long long words)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < words;
         i += (long long)gridDim.x * 256)
        p[i] = 0u;
}

}  // namespace

void launch_zero_words(unsigned* p, long long words, hipStream_t s)
{
    if (words <= 0) return;
    long long b = (words + 255) / 256;
    if (b > 1024) b = 1024;
    hipLaunchKernelGGL(kl_zero_kernel, dim3((unsigned)b), dim3(256), 0, s, p, words);
}

int knn_list_workgroups(long long nq)
{
    const int cus = device_cus();
    // a few rows per wavefront keep the threshold guess warm; many
    // wavefronts hide the latency of each row's loads
    long long want = (nq + 4LL * kKlWaves - 1) / (4LL * kKlWaves);
    const long long cap = 32LL * cus;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    return (int)want;
}

void launch_knn_list(const KnnListArgs& a, int blocks, hipStream_t s)
{
    if (a.nq == 0) return;
    hipLaunchKernelGGL(knn_list_kernel, dim3(blocks), dim3(kKlBlock), 0, s, a);
}

}  // namespace ppa
