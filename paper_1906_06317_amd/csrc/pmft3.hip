// PMFT histograms over three pair coordinates (the paper's PMFT section: in
// 2D the full PMFT also resolves the orientation of the second particle
// relative to the first; in 3D the translational part alone has three
// coordinates).  For every ball pair (i, j) the bond d = p_j - q_i (minimum
// image) is taken into the query particle's frame and counted in a uniform
// histogram:
//   XYT (2D): (x', y') = R(-theta_i) d and t = (theta_j - theta_i) mod 2 pi,
//             counts[(ix * nby + iy) * nbt + it], t in nbt bins of [0, 2 pi);
//   XYZ (3D): d' = R(q_i)^T d with R the rotation of the unit quaternion
//             q_i = (w, x, y, z), counts[(ix * nby + iy) * nbz + iz].
//
// The pairs come from the ball query's cell list (one wavefront per home
// cell, candidates in register slots, each query in scalar registers).  The
// histograms are larger than a workgroup's LDS at useful resolutions (e.g.
// 100 x 100 x 36 or 50^3 bins), so bonds are counted with global atomics;
// the few million bonds of a frame spread over 10^5 - 10^6 bins, so the
// atomics rarely collide.
#include "pair_common.hpp"

namespace ppa {

namespace {

using namespace pair;

constexpr int kP3Chunk = 4;  // slots per chunk of a stencil beyond 4 slots
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.15915494309189533577f;

// Per-lane frame of a query: XYT keeps (cos, sin, theta) in f[0..2]; XYZ the
// rotation matrix R of the normalised quaternion, row-major in f[0..8].
struct P3Frame {
    float f[9];
};

template <int MODE>
__device__ __forceinline__ P3Frame query_frame(const Pmft3Args& a, int qid, bool valid)
{
    P3Frame F;
#pragma unroll
    for (int k = 0; k < 9; ++k) F.f[k] = 0.f;
    if (!valid) return F;
    if (MODE == kPmftXyt) {
        const float th = a.q_orient[qid];
        if (!isfinite(th)) atomicOr(a.status, kStatusNonFinite);
        sincosf(th, &F.f[1], &F.f[0]);
        F.f[2] = th;
    } else {
        const float4 q = reinterpret_cast<const float4*>(a.q_orient)[qid];
        const float n2 = q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w;
        if (!(n2 > 0.f && isfinite(n2))) atomicOr(a.status, kStatusNonFinite);
        const float s = 1.f / sqrtf(n2);
        const float w = q.x * s, x = q.y * s, y = q.z * s, z = q.w * s;
        F.f[0] = 1.f - 2.f * (y * y + z * z);
        F.f[1] = 2.f * (x * y - w * z);
        F.f[2] = 2.f * (x * z + w * y);
        F.f[3] = 2.f * (x * y + w * z);
        F.f[4] = 1.f - 2.f * (x * x + z * z);
        F.f[5] = 2.f * (y * z - w * x);
        F.f[6] = 2.f * (x * z - w * y);
        F.f[7] = 2.f * (y * z + w * x);
        F.f[8] = 1.f - 2.f * (x * x + y * y);
    }
    return F;
}

__device__ __forceinline__ bool bin_of(float v, float lo, float inv_w, int nb, int& i)
{
    const float t = (v - lo) * inv_w;
    if (!(t >= 0.f && t < (float)nb)) return false;
    i = min((int)t, nb - 1);
    return true;
}

// Counts one bond of the lanes with `hit` (F: the query's frame in scalars).
template <int MODE>
__device__ __forceinline__ void bin_bond(const Pmft3Args& a, const P3Frame& F, float dx, float dy,
                                         float dz, float tj)
{
    float u, v, w;
    if (MODE == kPmftXyt) {
        u = fmaf(F.f[0], dx, F.f[1] * dy);
        v = fmaf(F.f[0], dy, -(F.f[1] * dx));
        float t = tj - F.f[2];
        t = fmaf(-kTwoPi, floorf(t * kInvTwoPi), t);
        w = t;
    } else {
        // R^T d: component k is column k of R against d
        u = fmaf(F.f[0], dx, fmaf(F.f[3], dy, F.f[6] * dz));
        v = fmaf(F.f[1], dx, fmaf(F.f[4], dy, F.f[7] * dz));
        w = fmaf(F.f[2], dx, fmaf(F.f[5], dy, F.f[8] * dz));
    }
    int ix, iy, iw;
    if (!bin_of(u, -a.max[0], a.inv_w[0], a.nb[0], ix)) return;
    if (!bin_of(v, -a.max[1], a.inv_w[1], a.nb[1], iy)) return;
    if (MODE == kPmftXyt) {
        // t lies in [0, 2 pi) up to rounding: clamp rather than drop
        iw = min(max((int)(w * a.inv_w[2]), 0), a.nb[2] - 1);
    } else if (!bin_of(w, -a.max[2], a.inv_w[2], a.nb[2], iw)) {
        return;
    }
    atomicAdd(&a.counts[((size_t)ix * a.nb[1] + iy) * a.nb[2] + iw], 1u);
}

// The queries of one home cell against candidates [k0, k0 + 64 NS) of its
// stencil.
template <int MODE, int NS>
__device__ __forceinline__ void p3_tile(const Pmft3Args& a, const PairIn& in,
                                        const StencilLds& S, const float4* off, int C, int k0,
                                        int q0, int q1, int lane)
{
    constexpr int DIM = MODE == kPmftXyt ? 2 : 3;
    const PairGeom& G = a.geom;
    Slots<DIM, NS> c;
    c.load(in, G, S, off, k0, C, lane);
    float tj[NS > 0 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        tj[s] = 0.f;
        if (MODE == kPmftXyt && c.id[s] >= 0) {
            tj[s] = a.p_orient[c.id[s]];
            if (!isfinite(tj[s])) atomicOr(a.status, kStatusNonFinite);
        }
    }
    const float r2max = G.r2max;
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        QueryChunk Q;
        Q.load(in, c0, q1 - c0, lane);
        const P3Frame Fl = query_frame<MODE>(a, Q.my_id(), lane < Q.n);
        for (int t = 0; t < Q.n; ++t) {
            const float qx = lane_off(Q.q.x, t), qy = lane_off(Q.q.y, t);
            const float qz = DIM == 3 ? lane_off(Q.q.z, t) : 0.f;
            const int qid = lane_of(Q.my_id(), t);
            P3Frame F;
#pragma unroll
            for (int k = 0; k < (MODE == kPmftXyt ? 3 : 9); ++k) F.f[k] = lane_off(Fl.f[k], t);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float dx = c.x[s] - qx, dy = c.y[s] - qy;
                const float dz = DIM == 3 ? c.z[s] - qz : 0.f;
                bool h = dist2<DIM>(dx, dy, dz) < r2max;
                if (a.excl) h = h && c.id[s] != qid;
                if (h) bin_bond<MODE>(a, F, dx, dy, dz, tj[s]);
            }
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) pmft3_kernel(const Pmft3Args a)
{
    constexpr int DIM = MODE == kPmftXyt ? 2 : 3;
    __shared__ float4 s_off[27];
    __shared__ StencilLds s_st[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    const PairGeom& G = a.geom;
    if (threadIdx.x < 27)
        s_off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1],
                                         G.off[threadIdx.x][2], 0.f);
    __syncthreads();
    const PairIn in{a.cand, a.cand_start, a.qsorted, a.q_start};
    StencilLds& S = s_st[wv];
    int t0, t1, stride;
    wave_tiles_interleaved<kWavesPerBlock>(G.ncells, wv, t0, t1, stride);
    for (int tile = t0; tile < t1; tile += stride) {
        const int q0 = in.q_start[tile];
        const int q1 = in.q_start[tile + 1];
        if (q0 == q1) continue;
        const int C = stencil<DIM>(in, G, tile, lane, S);
        const int ns = (C + kWave - 1) / kWave;
        switch (ns) {
#define PPA_CASE(N) \
    case N: p3_tile<MODE, N>(a, in, S, s_off, C, 0, q0, q1, lane); break;
            PPA_CASE(0) PPA_CASE(1) PPA_CASE(2) PPA_CASE(3) PPA_CASE(4)
#undef PPA_CASE
        default:
            for (int k0 = 0; k0 < C; k0 += kP3Chunk * kWave)
                p3_tile<MODE, kP3Chunk>(a, in, S, s_off, C, k0, q0, q1, lane);
        }
    }
}

}  // namespace

void launch_pmft3(const Pmft3Args& a, hipStream_t s)
{
    if (a.mode == kPmftXyt) {
        const int blocks = resident_blocks(pmft3_kernel<kPmftXyt>, 0, a.geom.ncells);
        hipLaunchKernelGGL(pmft3_kernel<kPmftXyt>, dim3(blocks), dim3(kBlock), 0, s, a);
    } else {
        const int blocks = resident_blocks(pmft3_kernel<kPmftXyz>, 0, a.geom.ncells);
        hipLaunchKernelGGL(pmft3_kernel<kPmftXyz>, dim3(blocks), dim3(kBlock), 0, s, a);
    }
}

}  // namespace ppa
