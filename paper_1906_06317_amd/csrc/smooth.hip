// Gaussian-smoothed RDF and its adjoint (an extension beyond the paper: a
// differentiable form of the density module's RDF).
//
//   phi(u) = exp(-u^2 / (2 s^2)) / (s sqrt(2 pi)),   c_b = (b + 1/2) dr,
//   h_b    = dr * sum over ordered pairs (i, j), i != j, r_ij < r_max + 8 s,
//            of phi(c_b - r_ij) for the bins with |c_b - r_ij| <= 8 s;
//   given G_b = dL/dh_b:
//   dL/dp_k = sum over j != k of 2 A(r_kj) (p_k - p_j) / r_kj,
//   A(r)    = sum_b G_b dr (c_b - r) / s^2 phi(c_b - r)   (same window),
// the factor 2 collecting the pairs (k, j) and (j, k); a pair at r = 0
// contributes nothing to the gradient.
//
// Both passes find their pairs over the cell list (cells of width >= r_max
// + 8 s, one wavefront per home cell, candidates in register slots tested
// in float32) and compact the hits into a per-wavefront LDS buffer as
// (candidate position in the sorted array, stencil slot, query lane).  At
// the flush every lane takes one hit and recomputes its pair vector in
// float64 from the stored cell-local coordinates and a float64 stencil
// offset, so the distance entering the Gaussian is exact to the rounding of
// the stored coordinates; the window terms are then evaluated in float32
// with the hardware exp2.  The forward adds each term into a float64 LDS
// histogram per workgroup (partials summed by a second kernel); the adjoint
// gathers each query's row in float64, so every particle's gradient is
// written once, by the wavefront that owns it, with no atomics.  The
// adjoint recomputes the pairs instead of reading anything stored by the
// forward.
#include "pair_common.hpp"

namespace ppa {

namespace {

using namespace pair;

constexpr int kSmSlots = 8;   // candidate slots per chunk
constexpr int kSmBuf = 768;   // hits buffered per wavefront
constexpr int kSmFlushAt = kSmBuf - kSmSlots * kWave;

struct SmoothLds {
    int2 hit[kSmBuf];  // (sorted candidate index, stencil slot | query lane << 5)
    float4 q[kWave];   // the query chunk: cell-local xyz, index bits
    StencilLds st;
};

struct SmoothShared {
    float4 off[27];
    double offd[27][3];
    SmoothLds w[kWavesPerBlock];
};

// Candidates [k0, k0 + 64 NS) of a stencil: coordinates relative to the
// home cell's centre in float32 (for the cut), sorted index and slot.
template <int DIM, int NS>
struct SmSlots {
    float x[NS], y[NS], z[NS];
    int idx[NS];  // sorted position; -1 past the end
    int j[NS];    // stencil slot

    __device__ __forceinline__ void load(const PairIn& in, const PairGeom& G, const StencilLds& S,
                                         const float4* off, int k0, int C, int lane)
    {
        int before = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            x[s] = y[s] = z[s] = kFar;
            idx[s] = -1;
            j[s] = 0;
            const int k = k0 + s * kWave + lane;
            const int jj = cell_of(S, G.nsten, k0, s, k, C, before);
            if (k < C) {
                const int p = S.base[jj] + k;
                const float4 v = in.cand[p];
                const float4 o = off[jj];
                x[s] = v.x + o.x;
                y[s] = v.y + o.y;
                z[s] = DIM == 3 ? v.z + o.z : 0.f;
                idx[s] = p;
                j[s] = jj;
            }
        }
    }
};

// Pair vector of a buffered hit in float64, candidate minus query.
template <int DIM>
__device__ __forceinline__ void hit_vector(const SmoothArgs& a, const SmoothShared& L,
                                           const SmoothLds& W, int2 h, double& dx, double& dy,
                                           double& dz)
{
    const int j = h.y & 31;
    const float4 v = a.cand[h.x];
    const float4 q = W.q[h.y >> 5];
    dx = ((double)v.x - (double)q.x) + L.offd[j][0];
    dy = ((double)v.y - (double)q.y) + L.offd[j][1];
    dz = DIM == 3 ? ((double)v.z - (double)q.z) + L.offd[j][2] : 0.0;
}

// Bins of the window around r: |c_b - r| <= 8 s, inside [0, bins).  The
// bounds are found in float32 (a bin at the edge carries weight e^-32, so
// where rounding puts the edge does not matter); the offset of the first
// bin centre from r is exact to float64 before rounding.
__device__ __forceinline__ void window(const SmoothArgs& a, double r, int& b0, int& b1, float& u0)
{
    const float rf = (float)r, w8 = (float)a.w8;
    b0 = max(0, (int)ceilf(fmaf(rf - w8, a.inv_dr, -0.5f)));
    b1 = min(a.bins - 1, (int)floorf(fmaf(rf + w8, a.inv_dr, -0.5f)));
    u0 = (float)fma((double)b0 + 0.5, a.dr, -r);
}

// Hits of query t (scalar) against NS slots, appended to the buffer.
template <int DIM, int NS>
__device__ __forceinline__ int buffer_query(const SmSlots<DIM, NS>& c, SmoothLds& W, int nh,
                                            float qx, float qy, float qz, int qpos, int t,
                                            float r2s)
{
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool h = dist2<DIM>(c.x[s] - qx, c.y[s] - qy, c.z[s] - qz) < r2s && c.idx[s] != qpos;
        const unsigned long long m = __ballot(h);
        if (h) W.hit[nh + (int)lane_prefix(m)] = make_int2(c.idx[s], c.j[s] | (t << 5));
        nh += __popcll(m);
    }
    return nh;
}

// Forward flush: every buffered pair's window terms into the LDS histogram.
template <int DIM>
__device__ __forceinline__ void flush_fwd(const SmoothArgs& a, const SmoothShared& L,
                                          SmoothLds& W, double* hist, int nh, int lane)
{
    wave_sync();
    const float drf = (float)a.dr;
    for (int e = lane; e < nh; e += kWave) {
        double dx, dy, dz;
        hit_vector<DIM>(a, L, W, W.hit[e], dx, dy, dz);
        const double r = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
        int b0, b1;
        float u0;
        window(a, r, b0, b1, u0);
        // each lane starts its walk at a different bin of its window, so the
        // lanes of one instruction rarely add to the same bin
        const int nb = b1 - b0 + 1;
        int m = nb > 0 ? lane % nb : 0;
#pragma unroll 4
        for (int j = 0; j < nb; ++j) {
            const float u = fmaf((float)m, drf, u0);
            const float v = a.hscale * __builtin_amdgcn_exp2f(-(u * u) * a.k2);
            atomicAdd(&hist[b0 + m], (double)v);
            m = m + 1 == nb ? 0 : m + 1;
        }
    }
    wave_sync();
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// Adjoint flush for the hits of one query: the sum of -2 A(r) d / r.
template <int DIM>
__device__ __forceinline__ void flush_bwd(const SmoothArgs& a, const SmoothShared& L,
                                          SmoothLds& W, const float* G, int nh, int lane,
                                          double& gx, double& gy, double& gz)
{
    wave_sync();
    const float drf = (float)a.dr;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int e = lane; e < nh; e += kWave) {
        double dx, dy, dz;
        hit_vector<DIM>(a, L, W, W.hit[e], dx, dy, dz);
        const double r = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
        if (r > 0.0) {
            int b0, b1;
            float u0;
            window(a, r, b0, b1, u0);
            // the window's terms change sign with u: sum them in float64.
            // Consecutive bins' Gaussians by recurrence: with u' = u + dr,
            // e(u') = e(u) p(u) and p(u') = p(u) c, where p(u) =
            // 2^(-k2 (2 u dr + dr^2)) and c = 2^(-2 k2 dr^2); two exp2 per
            // pair instead of one per bin (relative error of a term after
            // the window's ~20 steps: a few 1e-6)
            double A = 0.0;
            const int nb = b1 - b0 + 1;
            float u = u0;
            float e = __builtin_amdgcn_exp2f(-(u * u) * a.k2);
            float p = __builtin_amdgcn_exp2f(-a.k2 * drf * fmaf(2.f, u, drf));
            const float c = a.step2;
            const float* g = G + b0;
#pragma unroll 4
            for (int j = 0; j < nb; ++j) {
                A += (double)(g[j] * u * e);
                e *= p;
                p *= c;
                u += drf;
            }
            const double f = -2.0 * A / r;
            ax = fma(f, dx, ax);
            ay = fma(f, dy, ay);
            az = fma(f, dz, az);
        }
    }
    gx += wave_sum(ax);
    gy += wave_sum(ay);
    gz += wave_sum(az);
    wave_sync();
}

template <int DIM, bool BWD>
__global__ void __launch_bounds__(kBlock) smooth_kernel(const SmoothArgs a)
{
    extern __shared__ double s_dyn[];  // forward: histogram (float64); adjoint: G (float32)
    __shared__ SmoothShared L;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    SmoothLds& W = L.w[wv];
    const PairGeom& G = a.geom;
    if (threadIdx.x < 27) {
        L.off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1],
                                         G.off[threadIdx.x][2], 0.f);
        for (int c = 0; c < 3; ++c) L.offd[threadIdx.x][c] = a.offd[threadIdx.x][c];
    }
    double* hist = s_dyn;
    float* Gs = reinterpret_cast<float*>(s_dyn);
    for (int b = threadIdx.x; b < a.bins; b += kBlock) {
        if (BWD)
            Gs[b] = (float)a.grad_h[b] * a.gscale;
        else
            hist[b] = 0.0;
    }
    __syncthreads();
    const PairIn in{a.cand, a.cand_start, a.cand, a.cand_start};
    const float r2s = G.r2max;
    // work units: each home cell's queries in a.split parts (more units than
    // cells keep enough wavefronts busy when cells are few and full)
    int t0, t1, stride;
    wave_tiles_interleaved<kWavesPerBlock>(G.ncells * a.split, wv, t0, t1, stride);
    int nh = 0;
    for (int unit = t0; unit < t1; unit += stride) {
        const int tile = unit / a.split, part = unit - tile * a.split;
        const int qa = in.q_start[tile], qb = in.q_start[tile + 1];
        const int q0 = qa + (int)((long long)(qb - qa) * part / a.split);
        const int q1 = qa + (int)((long long)(qb - qa) * (part + 1) / a.split);
        if (q0 == q1) continue;
        const int C = stencil<DIM>(in, G, tile, lane, W.st);
        for (int c0 = q0; c0 < q1; c0 += kWave) {
            QueryChunk Q;
            Q.load(in, c0, q1 - c0, lane);
            W.q[lane] = Q.q;
            double gx = 0.0, gy = 0.0, gz = 0.0;  // adjoint: lane t holds query t's row
            for (int k0 = 0; k0 < C; k0 += kSmSlots * kWave) {
                SmSlots<DIM, kSmSlots> c;
                c.load(in, G, W.st, L.off, k0, C, lane);
                for (int t = 0; t < Q.n; ++t) {
                    const float qx = lane_off(Q.q.x, t), qy = lane_off(Q.q.y, t);
                    const float qz = DIM == 3 ? lane_off(Q.q.z, t) : 0.f;
                    nh = buffer_query<DIM, kSmSlots>(c, W, nh, qx, qy, qz, c0 + t, t, r2s);
                    if (BWD && nh > 0) {
                        double sx = 0.0, sy = 0.0, sz = 0.0;
                        flush_bwd<DIM>(a, L, W, Gs, nh, lane, sx, sy, sz);
                        nh = 0;
                        if (lane == t) {
                            gx += sx;
                            gy += sy;
                            gz += sz;
                        }
                    } else if (nh >= kSmFlushAt) {
                        flush_fwd<DIM>(a, L, W, hist, nh, lane);
                        nh = 0;
                    }
                }
            }
            if (BWD) {
                if (lane < Q.n) {
                    const int id = Q.my_id();
                    a.grad[3 * (size_t)id] = (float)gx;
                    a.grad[3 * (size_t)id + 1] = (float)gy;
                    a.grad[3 * (size_t)id + 2] = DIM == 3 ? (float)gz : 0.f;
                }
            } else if (nh > 0) {
                flush_fwd<DIM>(a, L, W, hist, nh, lane);  // the query chunk is about to change
                nh = 0;
            }
            wave_sync();
        }
    }
    if (!BWD) {
        __syncthreads();
        double* out = a.partial + (size_t)blockIdx.x * a.bins;
        for (int b = threadIdx.x; b < a.bins; b += kBlock) out[b] = hist[b];
    }
}

// h[b] += the first stage's sums (level2[row][b]) of the partial histograms.
__global__ void __launch_bounds__(256) smooth_reduce_kernel(const double* __restrict__ level2,
                                                            int rows, int bins,
                                                            double* __restrict__ h)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= bins) return;
    double sum = 0.0;
    for (int g = 0; g < rows; ++g) sum += level2[(size_t)g * bins + b];
    h[b] += sum;
}

template <int DIM, bool BWD>
int occupancy_blocks(size_t dyn)
{
    const int cus = device_cus();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, smooth_kernel<DIM, BWD>, kBlock,
                                                     dyn) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return (cus * per_cu + 7) / 8 * 8;
}

}  // namespace

// Workgroups of a smoothed-RDF launch (the forward's partial histograms are
// sized by it): every workgroup the device holds at once, a multiple of 8.
int smooth_workgroups(bool adjoint, int dim, int bins)
{
    const size_t dyn = (adjoint ? sizeof(float) : sizeof(double)) * (size_t)bins;
    if (dim == 3)
        return adjoint ? occupancy_blocks<3, true>(dyn) : occupancy_blocks<3, false>(dyn);
    return adjoint ? occupancy_blocks<2, true>(dyn) : occupancy_blocks<2, false>(dyn);
}

void launch_smooth_fwd(const SmoothArgs& a, int dim, int blocks, hipStream_t s)
{
    const size_t dyn = sizeof(double) * (size_t)a.bins;
    if (dim == 3)
        hipLaunchKernelGGL((smooth_kernel<3, false>), dim3(blocks), dim3(kBlock), dyn, s, a);
    else
        hipLaunchKernelGGL((smooth_kernel<2, false>), dim3(blocks), dim3(kBlock), dyn, s, a);
    const int rows = partial_rows(blocks);
    hipLaunchKernelGGL(partial_sum_stage1<double>, dim3((a.bins + 63) / 64, rows), dim3(256), 0, s,
                       a.partial, blocks, a.bins, kPartialRowsPer, a.level2);
    hipLaunchKernelGGL(smooth_reduce_kernel, dim3((a.bins + 255) / 256), dim3(256), 0, s,
                       a.level2, rows, a.bins, a.h);
}

void launch_smooth_bwd(const SmoothArgs& a, int dim, int blocks, hipStream_t s)
{
    const size_t dyn = sizeof(float) * (size_t)a.bins;
    if (dim == 3)
        hipLaunchKernelGGL((smooth_kernel<3, true>), dim3(blocks), dim3(kBlock), dyn, s, a);
    else
        hipLaunchKernelGGL((smooth_kernel<2, true>), dim3(blocks), dim3(kBlock), dyn, s, a);
}

}  // namespace ppa
