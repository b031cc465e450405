// Ball query over the cell list, with the RDF histogram binned in the same
// pass (the paper's neighbor query with a distance cutoff and the density
// module's RDF, "General Utilities" and "Analysis Modules": finding pairs
// inside the analysis instead of materializing them first is the design the
// paper credits with a 2x speed-up).
//
// Work decomposition (one wavefront per home cell):
//   * every wavefront owns a contiguous run of home cells; workgroups are
//     renumbered so the cells of one XCD are contiguous and its L2 sees the
//     stencil overlap of neighbouring cells;
//   * for a home cell, the 27 (2D: 9) stencil cells are gathered into up to
//     kMaxSlots registers per lane, each candidate shifted by its stencil
//     offset so it is relative to the home cell's centre;
//   * each query point of the home cell (scalar registers) is tested against
//     every candidate slot; the query's own entry is removed from the ballot
//     with a scalar mask when points query themselves.
// The NeighborList takes two passes so rows land in query order without
// atomics: count_kernel writes row lengths, a scan turns them into CSR
// offsets, and fill_kernel compacts hits with ballot + mbcnt into a small
// per-wavefront LDS list (whole rows) that is flushed densely: sqrt, the
// histogram bin and coalesced stores for 64 hits per instruction.  The RDF
// alone (no list) needs only the fill pass.  Home cells with more candidates
// than fit in registers stream candidates from memory instead.
#include "internal.hpp"

namespace ppa {

namespace {

constexpr float kFar = 1.0e18f;
constexpr int kHitCap = 512;   // hits buffered per wavefront in the list-writing pass
constexpr int kRows = 64;      // rows buffered per wavefront

__device__ __forceinline__ unsigned lane_prefix(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float uniformf(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int DIM>
__device__ __forceinline__ float dist2(float dx, float dy, float dz)
{
    return DIM == 3 ? fmaf(dz, dz, fmaf(dy, dy, dx * dx)) : fmaf(dy, dy, dx * dx);
}

// Inputs shared by the pair kernels.
struct PairIn {
    const float4* __restrict__ cand;     // points sorted by cell (local xyz, index bits)
    const int* __restrict__ cand_start;  // [ncells + 1]
    const float4* __restrict__ qs;       // query points sorted by cell
    const int* __restrict__ q_start;     // [ncells + 1]
};

struct StencilLds {
    int pre[32];
    int start[32];
};

// Home cells of this wavefront: [t0, t1).
__device__ __forceinline__ void wave_tiles(int ncells, int wv, int& t0, int& t1)
{
    const int G = gridDim.x;
    const int lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    const long long gw = (long long)lb * kWavesPerBlock + wv;
    const long long nw = (long long)G * kWavesPerBlock;
    t0 = uniform((int)(gw * ncells / nw));
    t1 = uniform((int)((gw + 1) * ncells / nw));
}

// Stencil of home cell `tile`: per-offset starts and prefix counts in LDS;
// returns the candidate count C (uniform).
template <int DIM>
__device__ __forceinline__ int stencil(const PairIn& in, const PairGeom& G, int tile, int lane,
                                       StencilLds& S)
{
    const int cx = tile % G.n[0];
    const int rest = tile / G.n[0];
    const int cy = rest % G.n[1];
    const int cz = rest / G.n[1];
    int cnt = 0, st = 0;
    if (lane < G.nsten) {
        const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = DIM == 3 ? lane / 9 - 1 : 0;
        int x = cx + dx, y = cy + dy, z = cz + dz;
        x += x < 0 ? G.n[0] : 0;
        x -= x >= G.n[0] ? G.n[0] : 0;
        y += y < 0 ? G.n[1] : 0;
        y -= y >= G.n[1] ? G.n[1] : 0;
        z += z < 0 ? G.n[2] : 0;
        z -= z >= G.n[2] ? G.n[2] : 0;
        const int nc = (z * G.n[1] + y) * G.n[0] + x;
        st = in.cand_start[nc];
        cnt = in.cand_start[nc + 1] - st;
    }
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
    }
    if (lane < G.nsten) {
        S.pre[lane + 1] = incl;
        S.start[lane] = st;
    }
    if (lane == 0) S.pre[0] = 0;
    wave_sync();
    return uniform(__shfl(incl, G.nsten - 1));
}

// Candidate at flat stencil index k, relative to the home cell's centre.
template <int DIM>
__device__ __forceinline__ void fetch(const PairIn& in, const PairGeom& G, const StencilLds& S,
                                      const float4* off, int k, float& x, float& y, float& z,
                                      int& id)
{
    int j = 0;
#pragma unroll
    for (int step = 16; step > 0; step >>= 1)
        if (j + step < G.nsten && S.pre[j + step] <= k) j += step;
    const float4 v = in.cand[S.start[j] + (k - S.pre[j])];
    const float4 o = off[j];
    x = v.x + o.x;
    y = v.y + o.y;
    z = DIM == 3 ? v.z + o.z : 0.f;
    id = __float_as_int(v.w);
}

// Bit of the query's own entry among the candidates (self queries only):
// it is entry (qi - q0) of the centre cell.
__device__ __forceinline__ void self_bit(const StencilLds& S, const PairGeom& G, int qi, int q0,
                                        int& slot, unsigned long long& keep)
{
    const int k = uniform(S.pre[G.center] + (qi - q0));
    slot = k >> 6;
    keep = ~(1ull << (k & 63));
}

// ---------------------------------------------------------------------------
// Pass 1: row lengths.
// ---------------------------------------------------------------------------
template <int DIM, int EXCL>
__global__ void __launch_bounds__(kBlock) count_kernel(const PairIn in, const PairGeom G,
                                                       int32_t* __restrict__ counts)
{
    __shared__ float4 s_off[27];
    __shared__ StencilLds s_st[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    StencilLds& S = s_st[wv];
    if (threadIdx.x < 27)
        s_off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1],
                                         G.off[threadIdx.x][2], 0.f);
    __syncthreads();
    int t0, t1;
    wave_tiles(G.ncells, wv, t0, t1);
    const float r2max = G.r2max;
    for (int tile = t0; tile < t1; ++tile) {
        const int q0 = in.q_start[tile];
        const int q1 = in.q_start[tile + 1];
        if (q0 == q1) continue;
        const int C = stencil<DIM>(in, G, tile, lane, S);
        if (C <= kCandCap) {
            float rx[kMaxSlots], ry[kMaxSlots], rz[kMaxSlots];
            int rid[kMaxSlots];
#pragma unroll
            for (int s = 0; s < kMaxSlots; ++s) {
                rx[s] = ry[s] = rz[s] = kFar;
                rid[s] = -1;
                if (s * kWave < C) {
                    const int k = s * kWave + lane;
                    if (k < C) fetch<DIM>(in, G, S, s_off, k, rx[s], ry[s], rz[s], rid[s]);
                }
            }
            for (int qi = q0; qi < q1; ++qi) {
                const float4 q = in.qs[qi];
                const float qx = uniformf(q.x), qy = uniformf(q.y), qz = uniformf(q.z);
                const int qid = uniform(__float_as_int(q.w));
                int sslot = -1;
                unsigned long long keep = ~0ull;
                if (EXCL == 1) self_bit(S, G, qi, q0, sslot, keep);
                int c = 0;
#pragma unroll
                for (int s = 0; s < kMaxSlots; ++s) {
                    if (s * kWave < C) {
                        const float r2 = dist2<DIM>(rx[s] - qx, ry[s] - qy, rz[s] - qz);
                        bool hit = r2 < r2max;
                        if (EXCL == 2) hit = hit && rid[s] != qid;
                        unsigned long long m = __ballot(hit);
                        if (EXCL == 1) m &= (s == sslot) ? keep : ~0ull;
                        c += __popcll(m);
                    }
                }
                if (lane == 0) counts[qid] = c;
            }
        } else {
            for (int qi = q0; qi < q1; ++qi) {
                const float4 q = in.qs[qi];
                const float qx = uniformf(q.x), qy = uniformf(q.y), qz = uniformf(q.z);
                const int qid = uniform(__float_as_int(q.w));
                int c = 0;
                for (int k0 = 0; k0 < C; k0 += kWave) {
                    const int k = k0 + lane;
                    bool hit = false;
                    if (k < C) {
                        float x, y, z;
                        int id;
                        fetch<DIM>(in, G, S, s_off, k, x, y, z, id);
                        hit = dist2<DIM>(x - qx, y - qy, z - qz) < r2max &&
                              !(EXCL != 0 && id == qid);
                    }
                    c += __popcll(__ballot(hit));
                }
                if (lane == 0) counts[qid] = c;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 2 (or the only pass for the histogram alone): hits -> list / bins.
// ---------------------------------------------------------------------------
struct FillOut {
    const int64_t* __restrict__ offsets;  // CSR row pointer (NL)
    int32_t* point_idx;
    float* dist;
    int64_t capacity;
    unsigned* status;
    unsigned long long* hist;
    int bins;
    float r_min;
    float inv_dr;
};

template <bool NL>
struct FillLds {
    int id[NL ? kHitCap : 1];
    float r2[NL ? kHitCap : kCandCap];
    unsigned char row[NL ? kHitCap : 1];
    long long base[NL ? kRows : 1];   // offsets[q] - start of the row in the buffer
    StencilLds st;
};

template <int DIM, int EXCL, bool NL, bool HIST>
__global__ void __launch_bounds__(kBlock) fill_kernel(const PairIn in, const PairGeom G,
                                                      const FillOut O)
{
    extern __shared__ unsigned s_hist[];
    __shared__ float4 s_off[27];
    __shared__ FillLds<NL> s_w[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    FillLds<NL>& W = s_w[wv];
    StencilLds& S = W.st;
    const bool lds_hist = HIST && O.bins <= kMaxLdsBins;
    if (threadIdx.x < 27)
        s_off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1],
                                         G.off[threadIdx.x][2], 0.f);
    if (lds_hist)
        for (int b = threadIdx.x; b < O.bins; b += kBlock) s_hist[b] = 0u;
    __syncthreads();

    auto bin = [&](float r) {
        const float t = (r - O.r_min) * O.inv_dr;
        if (t >= 0.f) {
            int b = (int)t;
            b = b < O.bins ? b : O.bins - 1;
            if (lds_hist)
                atomicAdd(&s_hist[b], 1u);
            else
                atomicAdd(&O.hist[b], 1ull);
        }
    };
    auto emit = [&](long long dst, int id, float r) {
        if (dst < O.capacity) {
            O.point_idx[dst] = id;
            if (O.dist) O.dist[dst] = r;
            return false;
        }
        return true;
    };

    int t0, t1;
    wave_tiles(G.ncells, wv, t0, t1);
    const float r2max = G.r2max;
    int nh = 0, nrows = 0;
    bool over = false;

    auto flush = [&]() {
        wave_sync();
        for (int e = lane; e < nh; e += kWave) {
            const float r = __fsqrt_rn(W.r2[e]);
            if (NL) over |= emit(W.base[W.row[e]] + e, W.id[e], r);
            if (HIST) bin(r);
        }
        nh = 0;
        nrows = 0;
        wave_sync();
    };

    for (int tile = t0; tile < t1; ++tile) {
        const int q0 = in.q_start[tile];
        const int q1 = in.q_start[tile + 1];
        if (q0 == q1) continue;
        const int C = stencil<DIM>(in, G, tile, lane, S);
        if (C <= kCandCap) {
            float rx[kMaxSlots], ry[kMaxSlots], rz[kMaxSlots];
            int rid[kMaxSlots];
#pragma unroll
            for (int s = 0; s < kMaxSlots; ++s) {
                rx[s] = ry[s] = rz[s] = kFar;
                rid[s] = -1;
                if (s * kWave < C) {
                    const int k = s * kWave + lane;
                    if (k < C) fetch<DIM>(in, G, S, s_off, k, rx[s], ry[s], rz[s], rid[s]);
                }
            }
            for (int qi = q0; qi < q1; ++qi) {
                const float4 q = in.qs[qi];
                const float qx = uniformf(q.x), qy = uniformf(q.y), qz = uniformf(q.z);
                const int qid = uniform(__float_as_int(q.w));
                int sslot = -1;
                unsigned long long keep = ~0ull;
                if (EXCL == 1) self_bit(S, G, qi, q0, sslot, keep);
                long long rbase = 0;
                int len = C;
                if (NL) {
                    rbase = O.offsets[qid];
                    len = (int)(O.offsets[qid + 1] - rbase);
                }
                const int cap = NL ? kHitCap : kCandCap;
                const bool direct = len > cap;  // a row longer than the buffer: write it directly
                if (nh + len > cap || (NL && nrows == kRows) || (direct && nh > 0)) flush();
                const int rs = nh;
                int w = 0;
#pragma unroll
                for (int s = 0; s < kMaxSlots; ++s) {
                    if (s * kWave < C) {
                        const float r2 = dist2<DIM>(rx[s] - qx, ry[s] - qy, rz[s] - qz);
                        bool hit = r2 < r2max;
                        if (EXCL == 2) hit = hit && rid[s] != qid;
                        unsigned long long m = __ballot(hit);
                        if (EXCL == 1) m &= (s == sslot) ? keep : ~0ull;
                        const bool mine = (m >> lane) & 1ull;
                        if (!direct) {
                            if (mine) {
                                const int pos = nh + (int)lane_prefix(m);
                                W.r2[pos] = r2;
                                if (NL) {
                                    W.id[pos] = rid[s];
                                    W.row[pos] = (unsigned char)nrows;
                                }
                            }
                            nh += __popcll(m);
                        } else {
                            if (mine) {
                                const float r = __fsqrt_rn(r2);
                                if (NL) over |= emit(rbase + w + (int)lane_prefix(m), rid[s], r);
                                if (HIST) bin(r);
                            }
                            w += __popcll(m);
                        }
                    }
                }
                if (NL && !direct) {
                    if (lane == 0) W.base[nrows] = rbase - rs;
                    ++nrows;
                }
            }
        } else {
            // oversized stencil: stream the candidates from memory, writing directly
            if (nh > 0) flush();
            for (int qi = q0; qi < q1; ++qi) {
                const float4 q = in.qs[qi];
                const float qx = uniformf(q.x), qy = uniformf(q.y), qz = uniformf(q.z);
                const int qid = uniform(__float_as_int(q.w));
                const long long rbase = NL ? O.offsets[qid] : 0;
                int w = 0;
                for (int k0 = 0; k0 < C; k0 += kWave) {
                    const int k = k0 + lane;
                    bool hit = false;
                    float r2 = 0.f;
                    int id = -1;
                    if (k < C) {
                        float x, y, z;
                        fetch<DIM>(in, G, S, s_off, k, x, y, z, id);
                        r2 = dist2<DIM>(x - qx, y - qy, z - qz);
                        hit = r2 < r2max && !(EXCL != 0 && id == qid);
                    }
                    const unsigned long long m = __ballot(hit);
                    if (hit) {
                        const float r = __fsqrt_rn(r2);
                        if (NL) over |= emit(rbase + w + (int)lane_prefix(m), id, r);
                        if (HIST) bin(r);
                    }
                    w += __popcll(m);
                }
            }
        }
    }
    if (nh > 0) flush();
    if (NL && __ballot(over) && lane == 0) atomicOr(O.status, kStatusCapacity);

    __syncthreads();
    if (lds_hist)
        for (int b = threadIdx.x; b < O.bins; b += kBlock) {
            const unsigned v = s_hist[b];
            if (v) atomicAdd(&O.hist[b], (unsigned long long)v);
        }
}

__global__ void __launch_bounds__(256) hist_from_dist_kernel(const float* __restrict__ dist,
                                                             const int64_t* n_pairs,
                                                             int64_t capacity, int bins,
                                                             float r_min, float inv_dr,
                                                             unsigned long long* hist)
{
    extern __shared__ unsigned s_hist[];
    const bool lds_hist = bins <= kMaxLdsBins;
    if (lds_hist)
        for (int b = threadIdx.x; b < bins; b += blockDim.x) s_hist[b] = 0u;
    __syncthreads();
    int64_t np = *n_pairs;
    np = np < capacity ? np : capacity;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < np;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float t = (dist[e] - r_min) * inv_dr;
        if (t >= 0.f) {
            int b = (int)t;
            if (b < bins) {
                if (lds_hist)
                    atomicAdd(&s_hist[b], 1u);
                else
                    atomicAdd(&hist[b], 1ull);
            }
        }
    }
    __syncthreads();
    if (lds_hist)
        for (int b = threadIdx.x; b < bins; b += blockDim.x) {
            const unsigned v = s_hist[b];
            if (v) atomicAdd(&hist[b], (unsigned long long)v);
        }
}

template <int DIM, int EXCL>
void launch_count_t(const PairIn& in, const PairGeom& g, int32_t* counts, int blocks,
                    hipStream_t s)
{
    hipLaunchKernelGGL((count_kernel<DIM, EXCL>), dim3(blocks), dim3(kBlock), 0, s, in, g, counts);
}

template <int DIM, int EXCL>
void launch_fill_t(const PairIn& in, const PairGeom& g, const FillOut& o, bool nl, bool hist,
                   int blocks, hipStream_t s)
{
    const size_t lds = (hist && o.bins <= kMaxLdsBins) ? sizeof(unsigned) * (size_t)o.bins : 0;
    if (nl && hist)
        hipLaunchKernelGGL((fill_kernel<DIM, EXCL, true, true>), dim3(blocks), dim3(kBlock), lds, s,
                           in, g, o);
    else if (nl)
        hipLaunchKernelGGL((fill_kernel<DIM, EXCL, true, false>), dim3(blocks), dim3(kBlock), lds,
                           s, in, g, o);
    else
        hipLaunchKernelGGL((fill_kernel<DIM, EXCL, false, true>), dim3(blocks), dim3(kBlock), lds,
                           s, in, g, o);
}

PairIn make_in(const PairArgs& a)
{
    PairIn in;
    in.cand = a.cand;
    in.cand_start = a.cand_start;
    in.qs = a.qsorted;
    in.q_start = a.q_start;
    return in;
}

}  // namespace

void launch_count(const PairArgs& a, int dim, int excl, int blocks, hipStream_t s)
{
    const PairIn in = make_in(a);
#define PPA_COUNT(D, E) launch_count_t<D, E>(in, a.geom, a.counts, blocks, s)
    if (dim == 3) {
        if (excl == 1) PPA_COUNT(3, 1); else if (excl == 2) PPA_COUNT(3, 2); else PPA_COUNT(3, 0);
    } else {
        if (excl == 1) PPA_COUNT(2, 1); else if (excl == 2) PPA_COUNT(2, 2); else PPA_COUNT(2, 0);
    }
#undef PPA_COUNT
}

void launch_fill(const PairArgs& a, int dim, int excl, bool nl, bool hist, int blocks,
                 hipStream_t s)
{
    const PairIn in = make_in(a);
    FillOut o;
    o.offsets = a.offsets;
    o.point_idx = a.point_idx;
    o.dist = a.dist;
    o.capacity = a.capacity;
    o.status = a.status;
    o.hist = a.hist;
    o.bins = hist ? a.bins : 0;
    o.r_min = a.r_min;
    o.inv_dr = a.inv_dr;
#define PPA_FILL(D, E) launch_fill_t<D, E>(in, a.geom, o, nl, hist, blocks, s)
    if (dim == 3) {
        if (excl == 1) PPA_FILL(3, 1); else if (excl == 2) PPA_FILL(3, 2); else PPA_FILL(3, 0);
    } else {
        if (excl == 1) PPA_FILL(2, 1); else if (excl == 2) PPA_FILL(2, 2); else PPA_FILL(2, 0);
    }
#undef PPA_FILL
}

int pair_grid_blocks(int ncells)
{
    static int cached = 0;
    if (cached == 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        }
        cached = cus * 4;  // four 256-thread workgroups per CU
    }
    // at least one home cell per wavefront, and a multiple of 8 (XCD renumbering)
    long long want = (ncells + kWavesPerBlock - 1) / kWavesPerBlock;
    if (want > cached) want = cached;
    if (want < 1) want = 1;
    return (int)((want + 7) / 8 * 8);
}

void launch_hist_from_dist(const float* dist, const int64_t* n_pairs, int64_t capacity, int bins,
                           float r_min, float inv_dr, unsigned long long* hist, hipStream_t s)
{
    const size_t lds = bins <= kMaxLdsBins ? sizeof(unsigned) * (size_t)bins : 0;
    hipLaunchKernelGGL(hist_from_dist_kernel, dim3(1024), dim3(256), lds, s, dist, n_pairs,
                       capacity, bins, r_min, inv_dr, hist);
}

}  // namespace ppa
