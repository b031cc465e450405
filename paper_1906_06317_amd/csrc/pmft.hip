// 2D potential of mean force and torque histogram (the paper's PMFT
// section): for every ball pair (i, j) the bond d = p_j - q_i (minimum
// image) is turned into the frame of the query point by its orientation,
//     x' =  cos(theta_i) d_x + sin(theta_i) d_y
//     y' = -sin(theta_i) d_x + cos(theta_i) d_y,
// and counted in a uniform 2D histogram on [-x_max, x_max) x [-y_max, y_max).
//
// The pairs come from the ball query's cell list, one wavefront per home
// cell, candidates in register slots, each query in scalar registers.  A
// query finds about 20 bonds among a slot's 64 candidates, so binning them
// where they are found would run the binning arithmetic for a wavefront
// two-thirds idle: instead each hit's rotated bond (x', y') is compacted
// (ballot + mbcnt) into a per-wavefront LDS buffer, and whenever it holds 64
// bonds one full-width pass bins them.  The
// histogram is privatised per workgroup in LDS, keeping only the bins a bond
// shorter than r_max can reach (the paper notes that multi-dimensional
// histograms outgrow the caches first): at 200 x 200 bins on [-3, 3)^2 with
// r_max = 3 that is 31,450 bins.  When it lets more workgroups share a CU,
// two 16-bit counters share an LDS word (63 KB instead of 126 KB there, two
// 1024-thread workgroups per CU instead of one); a counter that reaches 2^15
// hands 2^15 to the caller's count with one global atomic (the lane whose
// add took it there), so a counter never wraps.  Each workgroup writes its
// histogram to its own partial array and a second kernel sums the partials
// into the caller's counts.  Histograms too large for LDS use global atomics.
#include "pair_common.hpp"

namespace ppa {

namespace {

using namespace pair;

constexpr int kPmftBlock = 1024;
constexpr int kPmftWaves = kPmftBlock / kWave;
constexpr int kPmftChunk = 4;  // slots per chunk of a stencil beyond 4 slots

struct PmftLds {
    float4 off[9];
    StencilLds st[kPmftWaves];
    int lo[kPmftMaxRows];
    int base[kPmftMaxRows + 1];
};

constexpr int kBondBuf = 2 * kWave;  // rotated bonds buffered per wavefront

// Where the bins live: global atomics only, the LDS window with 32-bit
// counters, or the LDS window with two 16-bit counters per word.
enum { kHistGlobal = 0, kHistLds32 = 1, kHistLds16 = 2 };

// Bins one rotated bond (the calling lanes).
template <int MODE>
__device__ __forceinline__ void bin_rotated(const PmftArgs& a, const PmftLds& L, unsigned* hist,
                                            float xr, float yr)
{
    const float tx = (xr + a.x_max) * a.inv_dx;
    const float ty = (yr + a.y_max) * a.inv_dy;
    if (!(tx >= 0.f && tx < (float)a.nbx && ty >= 0.f && ty < (float)a.nby)) return;
    const int ix = min((int)tx, a.nbx - 1);
    const int iy = min((int)ty, a.nby - 1);
    if (MODE != kHistGlobal) {
        const int w = iy - L.lo[ix];
        const int b = L.base[ix];
        if (w >= 0 && w < L.base[ix + 1] - b) {
            if (MODE == kHistLds32) {
                atomicAdd(&hist[b + w], 1u);
                return;
            }
            // entry e is the low (even e) or high half of word e / 2; the add
            // that takes a half from 2^15 - 1 to 2^15 takes 2^15 back out and
            // into the global count, so a half stays below 2^15 plus the adds
            // in flight (fewer than a workgroup's lanes) and never wraps
            const int e = b + w;
            const unsigned sh = (unsigned)(e & 1) << 4;
            const unsigned old = atomicAdd(&hist[e >> 1], 1u << sh);
            if (((old >> sh) & 0xffffu) == 0x7fffu) {
                atomicSub(&hist[e >> 1], 0x8000u << sh);
                atomicAdd(&a.counts[ix * a.nby + iy], 0x8000u);
            }
            return;
        }
    }
    atomicAdd(&a.counts[ix * a.nby + iy], 1u);
}

// A wavefront's buffer of rotated bonds waiting to be binned.
template <int MODE>
struct BondBuf {
    float2* buf;  // [kBondBuf] in LDS
    int nb;       // bonds buffered
    int lane;

    // Adds the calling lanes' bonds (mask m of the wavefront's lanes).
    __device__ __forceinline__ void add(bool h, unsigned long long m, float xr, float yr)
    {
        if (h) buf[nb + (int)lane_prefix(m)] = make_float2(xr, yr);
        nb += __popcll(m);
    }
    // Bins 64 bonds when that many are buffered, keeping the rest.
    __device__ __forceinline__ void drain(const PmftArgs& a, const PmftLds& L, unsigned* hist)
    {
        if (nb < kWave) return;
        wave_sync();
        const float2 v = buf[lane];
        const bool more = lane < nb - kWave;
        float2 rest = make_float2(0.f, 0.f);
        if (more) rest = buf[kWave + lane];
        wave_sync();
        if (more) buf[lane] = rest;
        nb -= kWave;
        bin_rotated<MODE>(a, L, hist, v.x, v.y);
    }
    __device__ __forceinline__ void finish(const PmftArgs& a, const PmftLds& L, unsigned* hist)
    {
        wave_sync();
        if (lane < nb) {
            const float2 v = buf[lane];
            bin_rotated<MODE>(a, L, hist, v.x, v.y);
        }
        nb = 0;
        wave_sync();
    }
};

// The queries of one home cell against candidates [k0, k0 + 64 NS) of its
// stencil.
template <int NS, int MODE>
__device__ __forceinline__ void pmft_tile(const PmftArgs& a, const PairIn& in, const PmftLds& L,
                                          const StencilLds& S, unsigned* hist, BondBuf<MODE>& B,
                                          int C, int k0, int q0, int q1, int lane)
{
    const PairGeom& G = a.geom;
    Slots<2, NS> c;
    c.load(in, G, S, L.off, k0, C, lane);
    const float r2max = G.r2max;
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        QueryChunk Q;
        Q.load(in, c0, q1 - c0, lane);
        float sn = 0.f, cs = 1.f;
        if (lane < Q.n) sincosf(a.angles[Q.my_id()], &sn, &cs);
        for (int t = 0; t < Q.n; ++t) {
            const float qx = lane_off(Q.q.x, t), qy = lane_off(Q.q.y, t);
            const int qid = lane_of(Q.my_id(), t);
            const float ct = lane_off(cs, t), st = lane_off(sn, t);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float dx = c.x[s] - qx, dy = c.y[s] - qy;
                bool h = fmaf(dy, dy, dx * dx) < r2max;
                if (a.excl) h = h && c.id[s] != qid;
                // the bond in the query's frame, rotated by -theta
                const float xr = fmaf(ct, dx, st * dy);
                const float yr = fmaf(ct, dy, -(st * dx));
                B.add(h, __ballot(h), xr, yr);
                B.drain(a, L, hist);
            }
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(kPmftBlock) pmft_kernel(const PmftArgs a)
{
    constexpr bool LDS = MODE != kHistGlobal;
    extern __shared__ unsigned s_hist[];
    __shared__ PmftLds L;
    __shared__ float2 s_bonds[kPmftWaves][kBondBuf];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    const PairGeom& G = a.geom;
    BondBuf<MODE> B{s_bonds[wv], 0, lane};
    if (threadIdx.x < 9)
        L.off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1], 0.f, 0.f);
    if (LDS) {
        for (int i = threadIdx.x; i < a.nbx; i += kPmftBlock) L.lo[i] = a.table.lo[i];
        for (int i = threadIdx.x; i <= a.nbx; i += kPmftBlock) L.base[i] = a.table.base[i];
        for (int i = threadIdx.x; i < a.words; i += kPmftBlock) s_hist[i] = 0u;
    }
    __syncthreads();
    const PairIn in{a.cand, a.cand_start, a.qsorted, a.q_start};
    StencilLds& S = L.st[wv];
    int t0, t1, stride;
    wave_tiles_interleaved<kPmftWaves>(G.ncells, wv, t0, t1, stride);
    for (int tile = t0; tile < t1; tile += stride) {
        const int q0 = in.q_start[tile];
        const int q1 = in.q_start[tile + 1];
        if (q0 == q1) continue;
        const int C = stencil<2>(in, G, tile, lane, S);
        const int ns = (C + kWave - 1) / kWave;
        switch (ns) {
#define PPA_CASE(N) \
    case N: pmft_tile<N, MODE>(a, in, L, S, s_hist, B, C, 0, q0, q1, lane); break;
            PPA_CASE(0) PPA_CASE(1) PPA_CASE(2) PPA_CASE(3) PPA_CASE(4)
#undef PPA_CASE
        default:
            for (int k0 = 0; k0 < C; k0 += kPmftChunk * kWave)
                pmft_tile<kPmftChunk, MODE>(a, in, L, S, s_hist, B, C, k0, q0, q1, lane);
        }
    }
    B.finish(a, L, s_hist);
    if (LDS) {
        __syncthreads();
        unsigned* out = a.partial + (size_t)blockIdx.x * a.entries;
        if (MODE == kHistLds32) {
            for (int i = threadIdx.x; i < a.words; i += kPmftBlock) out[i] = s_hist[i];
        } else {
            for (int i = threadIdx.x; i < a.words; i += kPmftBlock) {
                const unsigned v = s_hist[i];
                out[2 * i] = v & 0xffffu;
                if (2 * i + 1 < a.entries) out[2 * i + 1] = v >> 16;
            }
        }
    }
}

// counts[ix][iy] += the first stage's sums (level2[gs][word]) of the
// workgroups' partial histograms.
__global__ void __launch_bounds__(256) pmft_reduce_kernel(const unsigned* __restrict__ level2,
                                                          int rows, int words, int nbx, int nby,
                                                          PmftTable table,
                                                          unsigned* __restrict__ counts)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nbx * nby) return;
    const int ix = b / nby, iy = b - ix * nby;
    const int w = iy - table.lo[ix];
    if (w < 0 || w >= table.base[ix + 1] - table.base[ix]) return;
    const int idx = table.base[ix] + w;
    unsigned sum = 0;
    for (int g = 0; g < rows; ++g) sum += level2[(size_t)g * words + idx];
    counts[b] += sum;
}

}  // namespace

// Resident workgroups per CU of the launch with `words` LDS words of
// histogram (0: the global-atomics kernel), 32- or 16-bit counters.
int pmft_blocks_per_cu(int words, int packed)
{
    const size_t lds = sizeof(unsigned) * (size_t)words;
    int per_cu = 0;
    hipError_t e;
    if (words <= 0)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pmft_kernel<kHistGlobal>,
                                                         kPmftBlock, 0);
    else if (packed)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pmft_kernel<kHistLds16>,
                                                         kPmftBlock, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pmft_kernel<kHistLds32>,
                                                         kPmftBlock, lds);
    return e != hipSuccess || per_cu < 1 ? 1 : per_cu;
}

// Workgroups of the LDS-histogram launch (as many as are resident at once),
// or of the global-atomics launch; a multiple of 8.
int pmft_workgroups(int words, int packed)
{
    return (device_cus() * pmft_blocks_per_cu(words, packed) + 7) / 8 * 8;
}

size_t pmft_lds_limit()
{
    // initialised once, thread-safely
    static const size_t limit = [] {
        int dev = 0, v = 0;
        size_t l = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            v > 0)
            l = (size_t)v;
        // the static part of the kernel's LDS
        return l - (sizeof(PmftLds) + sizeof(float2) * kBondBuf * kPmftWaves + 256);
    }();
    return limit;
}

void launch_pmft(const PmftArgs& a, int blocks, hipStream_t s)
{
    if (a.words > 0) {
        const size_t lds = sizeof(unsigned) * (size_t)a.words;
        const auto k = a.packed ? pmft_kernel<kHistLds16> : pmft_kernel<kHistLds32>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(k, dim3(blocks), dim3(kPmftBlock), lds, s, a);
        const int rows = partial_rows(blocks);
        hipLaunchKernelGGL(partial_sum_stage1<unsigned>, dim3((a.entries + 63) / 64, rows),
                           dim3(256), 0, s, a.partial, blocks, a.entries, kPartialRowsPer,
                           a.level2);
        const int nb = a.nbx * a.nby;
        hipLaunchKernelGGL(pmft_reduce_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, a.level2,
                           rows, a.entries, a.nbx, a.nby, a.table, a.counts);
    } else {
        hipLaunchKernelGGL(pmft_kernel<kHistGlobal>, dim3(blocks), dim3(kPmftBlock), 0, s, a);
    }
}

}  // namespace ppa
