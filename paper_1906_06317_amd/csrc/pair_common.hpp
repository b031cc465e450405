// Device helpers shared by the pair kernels (ball query, RDF, k-NN, PMFT,
// smoothed RDF): stencil of a home cell, candidates in register slots,
// query points prefetched 64 at a time.
#pragma once

#include "internal.hpp"

namespace ppa {
namespace pair {

constexpr float kFar = 1.0e18f;
constexpr int kChunkSlots = 8;  // slots per chunk of an oversized stencil

__device__ __forceinline__ unsigned lane_prefix(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// base + the number of set bits of mask below this lane (the running count
// rides in the mbcnt addend, so no separate add is needed).
__device__ __forceinline__ int lane_slot(unsigned long long mask, int base)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, (unsigned)base));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float uniformf(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ int lane_of(int v, int t) { return __builtin_amdgcn_readlane(v, t); }

__device__ __forceinline__ float lane_off(float v, int t)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t));
}

// The writelane intrinsic, called directly rather than written as inline
// assembly, so the compiler sees the instruction and inserts the wait
// states it needs (a v_writelane reading an SGPR that a vector instruction
// has just written can otherwise see the old value).
__device__ int amdgcn_writelane(int x, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// v with lane t replaced by the uniform value x (one v_writelane).
__device__ __forceinline__ int with_lane(int v, int t, int x) { return amdgcn_writelane(x, t, v); }

__device__ __forceinline__ unsigned long long uniform64(unsigned long long v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Inclusive prefix sum over the wavefront by DPP: shifts by 1, 2, 4 and 8
// lanes within each 16-lane row, then lane 15 of each even row added to the
// row above and lane 31 to the upper half (vector instructions only).
__device__ __forceinline__ int wave_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// x + x of lane l ^ 16 (one permlane16 swap), and of lane l ^ 32.
__device__ __forceinline__ int pair_sum16(int x)
{
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (int)r[0] + (int)r[1];
}
__device__ __forceinline__ int pair_sum32(int x)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (int)r[0] + (int)r[1];
}

__device__ __forceinline__ long long lane_of64(long long v, int t)
{
    const unsigned lo = (unsigned)lane_of((int)(unsigned)v, t);
    const unsigned hi = (unsigned)lane_of((int)(v >> 32), t);
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Square root by the hardware instruction (within 1 ulp).
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

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
    int pre[32];   // candidates in the cells before stencil slot j
    int base[32];  // first sorted position of slot j's cell, less pre[j]
    // candidate k's stencil cell without a search: bit p of mask[p / 64]
    // marks a non-empty cell whose candidates start at p (for p below
    // kMaxSlots * 64), and jrank[r] is the r-th non-empty cell, so k lies in
    // cell jrank[(set bits at or below k) - 1]
    unsigned long long mask[kMaxSlots];
    unsigned char jrank[32];
};

// Home cells of this wavefront: [t0, t1).  Workgroups are renumbered so the
// workgroups of one XCD (dispatched round-robin over the 8 XCDs) own a
// contiguous range of cells; the grid is a multiple of 8.
template <int WPB>
__device__ __forceinline__ void wave_tiles_n(int ncells, int wv, int& t0, int& t1)
{
    const int G = gridDim.x;
    const int lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    const long long gw = (long long)lb * WPB + wv;
    const long long nw = (long long)G * WPB;
    t0 = uniform((int)(gw * ncells / nw));
    t1 = uniform((int)((gw + 1) * ncells / nw));
}

__device__ __forceinline__ void wave_tiles(int ncells, int wv, int& t0, int& t1)
{
    wave_tiles_n<kWavesPerBlock>(ncells, wv, t0, t1);
}

// Home cells of this wavefront, interleaved: the cells of XCD x (workgroups
// dispatched round-robin over the 8 XCDs) are [x C / 8, (x + 1) C / 8), and
// its wavefronts take them in turn, t0, t0 + stride, ... below t1, so the
// cells in flight on an XCD at any time are neighbours and share their
// stencil cells in that XCD's L2.
template <int WPB>
__device__ __forceinline__ void wave_tiles_interleaved(int ncells, int wv, int& t0, int& t1,
                                                       int& stride)
{
    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7;
    const int per = G >> 3;  // workgroups per XCD
    const int c0 = (int)((long long)xcd * ncells / 8);
    const int c1 = (int)((long long)(xcd + 1) * ncells / 8);
    t0 = uniform(c0 + (blockIdx.x >> 3) * WPB + wv);
    t1 = uniform(c1);
    stride = per * WPB;
    if ((int)(blockIdx.x >> 3) >= per) t1 = t0;  // launches are whole multiples of 8
}

// Work item v of a pass whose home cells are shared by `split` wavefronts
// each: its cell, and its part of the cell's queries [q0, q1) (contiguous
// parts of equal length; the last ones may be empty).  split <= 1: item v is
// cell v with all its queries.
struct CellPart {
    int tile, qc, q0, q1;  // cell, its first query, this part's queries
};

__device__ __forceinline__ CellPart cell_part(const PairIn& in, int v, int split)
{
    CellPart p;
    if (split <= 1) {
        p.tile = v;
        p.qc = p.q0 = in.q_start[v];
        p.q1 = in.q_start[v + 1];
        return p;
    }
    p.tile = uniform(v / split);
    const int part = v - p.tile * split;
    p.qc = in.q_start[p.tile];
    const int end = in.q_start[p.tile + 1];
    const int per = (end - p.qc + split - 1) / split;
    p.q0 = min(end, p.qc + part * per);
    p.q1 = min(end, p.q0 + per);
    return p;
}

// Stencil slot -> offset code d = (dx+1) + 3 (dy+1) + 9 (dz+1): the home
// cell (centre code) is slot 0 and takes the place of code 0.
__device__ __forceinline__ int stencil_code(int s, int nsten)
{
    const int centre = nsten / 2;
    return s == 0 ? centre : (s == centre ? 0 : s);
}

// Stencil of home cell `tile` (a global cell id; its frame's cells start at
// cell_base and form an n0 x n1 x n2 grid): per-offset starts and prefix
// counts in LDS; returns the candidate count C (uniform).
template <int DIM>
__device__ __forceinline__ int stencil(const PairIn& in, int n0, int n1, int n2, int nsten,
                                       int cell_base, int tile, int lane, StencilLds& S)
{
    const int local = tile - cell_base;
    const int cx = local % n0;
    const int rest = local / n0;
    const int cy = rest % n1;
    const int cz = rest / n1;
    int cnt = 0, st = 0;
    if (lane < nsten) {
        // slot 0 is the home cell itself (offset code 13 in 3D, 4 in 2D)
        const int code = stencil_code(lane, nsten);
        const int dx = code % 3 - 1, dy = (code / 3) % 3 - 1, dz = DIM == 3 ? code / 9 - 1 : 0;
        int x = cx + dx, y = cy + dy, z = cz + dz;
        x += x < 0 ? n0 : 0;
        x -= x >= n0 ? n0 : 0;
        y += y < 0 ? n1 : 0;
        y -= y >= n1 ? n1 : 0;
        z += z < 0 ? n2 : 0;
        z -= z >= n2 ? n2 : 0;
        const int nc = cell_base + (z * n1 + y) * n0 + x;
        st = in.cand_start[nc];
        cnt = in.cand_start[nc + 1] - st;
    }
    const int incl = wave_incl_scan(cnt);
    if (lane < nsten) {
        S.pre[lane + 1] = incl;
        S.base[lane] = st - (incl - cnt);
    }
    if (lane == 0) S.pre[0] = 0;
    if (lane < kMaxSlots) S.mask[lane] = 0ull;
    wave_sync();
    const bool nonempty = lane < nsten && cnt > 0;
    const unsigned long long ne = __ballot(nonempty);
    if (nonempty) {
        const int p = incl - cnt;
        S.jrank[lane_prefix(ne)] = (unsigned char)lane;
        if (p < kMaxSlots * kWave) atomicOr(&S.mask[p >> 6], 1ull << (p & 63));
    }
    wave_sync();
    return lane_of(incl, nsten - 1);
}

template <int DIM>
__device__ __forceinline__ int stencil(const PairIn& in, const PairGeom& G, int tile, int lane,
                                       StencilLds& S)
{
    return stencil<DIM>(in, G.n[0], G.n[1], G.n[2], G.nsten, 0, tile, lane, S);
}

// Stencil cell of candidate k = k0 + 64 s + lane of a stencil walk (for
// k < C; 0 otherwise).  A walk from the stencil's first candidate reads slot
// s's start mask: k lies in the non-empty cell whose start is the last set
// bit at or below k, counted with `before`, the non-empty cells starting in
// earlier slots (which the call advances).  Other walks (a chunk that starts
// further in, or slots past the masks) search the prefix counts.
__device__ __forceinline__ int cell_of(const StencilLds& S, int nsten, int k0, int s, int k,
                                       int C, int& before)
{
    int j = 0;
    if (k0 == 0 && s < kMaxSlots) {
        const unsigned long long m = uniform64(S.mask[s]);
        // set bits of m at or below this lane: bit 0, then the mbcnt of m >> 1
        if (k < C) j = S.jrank[lane_slot(m >> 1, before + (int)(m & 1ull) - 1)];
        before += __popcll(m);
    } else if (k < C) {
#pragma unroll
        for (int step = 16; step > 0; step >>= 1)
            if (j + step < nsten && S.pre[j + step] <= k) j += step;
    }
    return j;
}

// Fills slot s (candidates k0 + 64 s + lane) of a register-slot load with
// the candidate relative to the home cell's centre; entries past C are left
// as they are.
template <int DIM>
__device__ __forceinline__ void fetch_slot(const PairIn& in, int nsten, const StencilLds& S,
                                           const float4* off, int k0, int s, int C, int lane,
                                           int& before, float& x, float& y, float& z, int& id)
{
    const int k = k0 + s * kWave + lane;
    const int j = cell_of(S, nsten, k0, s, k, C, before);
    if (k < C) {
        const float4 v = in.cand[S.base[j] + k];
        const float4 o = off[j];
        x = v.x + o.x;
        y = v.y + o.y;
        z = DIM == 3 ? v.z + o.z : 0.f;
        id = __float_as_int(v.w);
    }
}

// What the pair loops need of a frame's geometry (one frame, or the frame of
// the current home cell in a batch).
struct GeomView {
    int n0, n1, n2, nsten;
    int cell_base;  // first global cell id of the frame
    float r2max;
    int dot;        // expanded in/out test allowed
};

__device__ __forceinline__ GeomView view_of(const PairGeom& G)
{
    GeomView v;
    v.n0 = G.n[0];
    v.n1 = G.n[1];
    v.n2 = G.n[2];
    v.nsten = G.nsten;
    v.cell_base = 0;
    v.r2max = G.r2max;
    v.dot = G.dot;
    return v;
}

template <int DIM>
__device__ __forceinline__ int stencil(const PairIn& in, const GeomView& V, int tile, int lane,
                                       StencilLds& S)
{
    return stencil<DIM>(in, V.n0, V.n1, V.n2, V.nsten, V.cell_base, tile, lane, S);
}

// One query point in scalar registers, with the constants of both tests.
struct Query {
    float x, y, z;
    float m2x, m2y, m2z;  // -2 q
    float thr;            // r_max^2 - |q|^2
    int id;
};

template <int DIM>
__device__ __forceinline__ Query make_query(float x, float y, float z, int id, float r2max)
{
    Query q;
    q.x = x;
    q.y = y;
    q.z = DIM == 3 ? z : 0.f;
    q.m2x = -2.f * x;
    q.m2y = -2.f * y;
    q.m2z = -2.f * q.z;
    q.thr = uniformf(r2max - dist2<DIM>(x, y, q.z));
    q.id = id;
    return q;
}

// The candidates of one home cell in NS register slots (entries past the
// end are far away, so they never hit).
template <int DIM, int NS>
struct Slots {
    float x[NS > 0 ? NS : 1], y[NS > 0 ? NS : 1], z[NS > 0 ? NS : 1];
    float cc[NS > 0 ? NS : 1];  // |c|^2
    int id[NS > 0 ? NS : 1];

    __device__ __forceinline__ void load(const PairIn& in, int nsten, const StencilLds& S,
                                         const float4* off, int k0, int C, int lane)
    {
        int before = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            x[s] = y[s] = z[s] = kFar;
            id[s] = -1;
            fetch_slot<DIM>(in, nsten, S, off, k0, s, C, lane, before, x[s], y[s], z[s], id[s]);
            cc[s] = dist2<DIM>(x[s], y[s], z[s]);
        }
    }
    __device__ __forceinline__ void load(const PairIn& in, const PairGeom& G, const StencilLds& S,
                                         const float4* off, int k0, int C, int lane)
    {
        load(in, G.nsten, S, off, k0, C, lane);
    }
    // the in/out test of slot s against q; identical in both passes
    template <bool DOT>
    __device__ __forceinline__ bool hit(int s, const Query& q, float r2max) const
    {
        if (DOT) {
            float t = fmaf(x[s], q.m2x, cc[s]);
            t = fmaf(y[s], q.m2y, t);
            if (DIM == 3) t = fmaf(z[s], q.m2z, t);
            return t < q.thr;
        }
        return dist2<DIM>(x[s] - q.x, y[s] - q.y, z[s] - q.z) < r2max;
    }
};

// The candidates of one home cell in NS register slots, held for the
// expanded in/out test: -2c and |c|^2 per candidate, so a test against a
// query in scalar registers is three FMAs and a compare,
//     t = |c|^2 + (-2c).q < r_max^2 - |q|^2.
// (-2c).q is the same exact product as c.(-2q), so t equals the value the
// test of Slots computes, bit for bit; c = -0.5 (-2c) is recovered exactly.
// Entries past the end are far away, so they never hit.
template <int DIM, int NS>
struct DotSlots {
    float mx[NS > 0 ? NS : 1], my[NS > 0 ? NS : 1], mz[NS > 0 ? NS : 1];
    float cc[NS > 0 ? NS : 1];
    int id[NS > 0 ? NS : 1];

    __device__ __forceinline__ void load(const PairIn& in, int nsten, const StencilLds& S,
                                         const float4* off, int k0, int C, int lane)
    {
        int before = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            float x = kFar, y = kFar, z = kFar;
            id[s] = -1;
            fetch_slot<DIM>(in, nsten, S, off, k0, s, C, lane, before, x, y, z, id[s]);
            cc[s] = dist2<DIM>(x, y, z);
            mx[s] = -2.f * x;
            my[s] = -2.f * y;
            mz[s] = -2.f * z;
        }
    }
    __device__ __forceinline__ bool hit(int s, float qx, float qy, float qz, float thr) const
    {
        float t = fmaf(mx[s], qx, cc[s]);
        t = fmaf(my[s], qy, t);
        if (DIM == 3) t = fmaf(mz[s], qz, t);
        return t < thr;
    }
};

// One query of a DotChunk.
struct DQuery {
    float x, y, z;
    float thr;  // r_max^2 - |q|^2
    int id;
};

// Query points of a tile, 64 at a time: each lane loads one and writes
// (x, y, z, r_max^2 - |q|^2) to its wavefront's row of 64 float4 in LDS
// (the expression the Query of QueryChunk holds).  A query is then read by
// every lane with one broadcast LDS load, so its values arrive in vector
// registers, the operands the tests read fastest, with no cross-lane VALU
// work per query.
struct DotChunk {
    float4 q;  // this lane's query point (index bits in w)
    int n;
    float4* row;

    template <int DIM>
    __device__ __forceinline__ void load(const PairIn& in, int first, int count, int lane,
                                         float r2max, float4* lds_row)
    {
        n = uniform(min(kWave, count));
        q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < n) q = in.qs[first + lane];
        const float z = DIM == 3 ? q.z : 0.f;
        row = lds_row;
        wave_sync();  // the previous chunk's reads are done
        row[lane] = make_float4(q.x, q.y, z, r2max - dist2<DIM>(q.x, q.y, z));
        wave_sync();
    }
    __device__ __forceinline__ DQuery get(int t) const
    {
        const float4 v = row[t];
        DQuery r;
        r.x = v.x;
        r.y = v.y;
        r.z = v.z;
        r.thr = v.w;
        r.id = lane_of(__float_as_int(q.w), t);
        return r;
    }
    __device__ __forceinline__ int my_id() const { return __float_as_int(q.w); }
};

// Query points of a tile, 64 at a time, one per lane.
struct QueryChunk {
    float4 q;
    int n;

    __device__ __forceinline__ void load(const PairIn& in, int first, int count, int lane)
    {
        n = uniform(min(kWave, count));
        q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < n) q = in.qs[first + lane];
    }
    template <int DIM>
    __device__ __forceinline__ Query get(int t, float r2max) const
    {
        return make_query<DIM>(lane_off(q.x, t), lane_off(q.y, t), lane_off(q.z, t),
                               lane_of(__float_as_int(q.w), t), r2max);
    }
    __device__ __forceinline__ int my_id() const { return __float_as_int(q.w); }
};


// Sum of per-workgroup partial arrays, first stage: partial[g][w] for
// g < G, w < W; workgroup (x, y) sums rows [y per, (y + 1) per) for 64
// consecutive w into level2[y][w].  Fixed order, so the result does not
// depend on timing.  Launch: grid (ceil(W / 64), ceil(G / per)), 256 threads.
template <typename T>
__global__ void __launch_bounds__(256) partial_sum_stage1(const T* __restrict__ partial, int G,
                                                          int W, int per, T* __restrict__ level2)
{
    __shared__ T s[4][64];
    const int lane = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int w = blockIdx.x * 64 + lane;
    const int g0 = blockIdx.y * per;
    const int g1 = min(G, g0 + per);
    T acc = 0;
    if (w < W)
        for (int g = g0 + sub; g < g1; g += 4) acc += partial[(size_t)g * W + w];
    s[sub][lane] = acc;
    __syncthreads();
    if (sub == 0 && w < W)
        level2[(size_t)blockIdx.y * W + w] = (s[0][lane] + s[1][lane]) + (s[2][lane] + s[3][lane]);
}

// Workgroups for a persistent launch of `kernel`: as many as fit on the
// device at once, at least one home cell per wavefront, a multiple of 8.
template <typename K>
inline int resident_blocks(K kernel, size_t lds, long long ncells)
{
    const int cus = device_cus();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    long long want = (ncells + kWavesPerBlock - 1) / kWavesPerBlock;
    const long long cap = (long long)cus * per_cu;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    return (int)((want + 7) / 8 * 8);
}

}  // namespace pair
}  // namespace ppa
