// Spatial correlation function of per-particle values (the density module's
// correlation functions of arbitrary quantities in the paper's analysis
// modules; its overview figure correlates the hexatic order parameter).
// For every ball pair (i, j), r_min <= r < r_max, with query value f_i and
// point value g_j (complex), bin b of r receives the term conj(f_i) g_j and
// one count:  S_b += conj(f_i) g_j,  N_b += 1;  the correlation is S_b / N_b.
//
// Terms are formed in float64 from the float32 values: the products of two
// floats are exact in double and the sum of two such products rounds once,
// so every term is the correctly rounded value.  The pairs come from the
// ball query's cell list (one wavefront per home cell, candidates and their
// values in register slots, each query in scalar registers); each workgroup
// accumulates its pairs in LDS (float64 sums, 64-bit counts), writes them to
// its own partial row, and a fixed-order two-stage sum adds the rows to the
// caller's arrays.
#include "pair_common.hpp"

namespace ppa {

namespace {

using namespace pair;

constexpr int kCorrChunk = 4;  // slots per chunk of a stencil beyond 4 slots

template <int DIM, int NS>
__device__ __forceinline__ void corr_tile(const CorrArgs& a, const PairIn& in,
                                          const StencilLds& S, const float4* off, double* hs,
                                          unsigned long long* hc, int C, int k0, int q0, int q1,
                                          int lane)
{
    const PairGeom& G = a.geom;
    Slots<DIM, NS> c;
    c.load(in, G, S, off, k0, C, lane);
    float gr[NS > 0 ? NS : 1], gi[NS > 0 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        gr[s] = gi[s] = 0.f;
        if (c.id[s] >= 0) {
            const float2 g = a.pval[c.id[s]];
            gr[s] = g.x;
            gi[s] = g.y;
            if (!(isfinite(g.x) && isfinite(g.y))) atomicOr(a.status, kStatusNonFinite);
        }
    }
    const float r2max = G.r2max;
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        QueryChunk Q;
        Q.load(in, c0, q1 - c0, lane);
        float2 f = make_float2(0.f, 0.f);
        if (lane < Q.n) {
            f = a.qval[Q.my_id()];
            if (!(isfinite(f.x) && isfinite(f.y))) atomicOr(a.status, kStatusNonFinite);
        }
        for (int t = 0; t < Q.n; ++t) {
            const float qx = lane_off(Q.q.x, t), qy = lane_off(Q.q.y, t);
            const float qz = DIM == 3 ? lane_off(Q.q.z, t) : 0.f;
            const int qid = lane_of(Q.my_id(), t);
            const double fr = (double)lane_off(f.x, t), fi = (double)lane_off(f.y, t);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float d2 = dist2<DIM>(c.x[s] - qx, c.y[s] - qy, c.z[s] - qz);
                bool h = d2 < r2max;
                if (a.excl) h = h && c.id[s] != qid;
                if (!h) continue;
                const float u = (fast_sqrt(d2) - a.r_min) * a.inv_dr;
                if (!(u >= 0.f && u < (float)a.bins)) continue;
                const int b = min((int)u, a.bins - 1);
                // conj(f) g = (fr gr + fi gi) + i (fr gi - fi gr)
                const double re = fma(fr, (double)gr[s], fi * (double)gi[s]);
                const double im = fma(fr, (double)gi[s], -(fi * (double)gr[s]));
                atomicAdd(&hs[2 * b], re);
                atomicAdd(&hs[2 * b + 1], im);
                atomicAdd(&hc[b], 1ull);
            }
        }
    }
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) corr_kernel(const CorrArgs a)
{
    extern __shared__ double s_corr[];
    __shared__ float4 s_off[27];
    __shared__ StencilLds s_st[kWavesPerBlock];
    double* hs = s_corr;                                                       // [2 bins]
    unsigned long long* hc = reinterpret_cast<unsigned long long*>(s_corr + 2 * a.bins);  // [bins]
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    const PairGeom& G = a.geom;
    if (threadIdx.x < 27)
        s_off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1],
                                         G.off[threadIdx.x][2], 0.f);
    for (int k = threadIdx.x; k < 2 * a.bins; k += kBlock) hs[k] = 0.0;
    for (int k = threadIdx.x; k < a.bins; k += kBlock) hc[k] = 0ull;
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
    case N: corr_tile<DIM, N>(a, in, S, s_off, hs, hc, C, 0, q0, q1, lane); break;
            PPA_CASE(0) PPA_CASE(1) PPA_CASE(2) PPA_CASE(3) PPA_CASE(4)
#undef PPA_CASE
        default:
            for (int k0 = 0; k0 < C; k0 += kCorrChunk * kWave)
                corr_tile<DIM, kCorrChunk>(a, in, S, s_off, hs, hc, C, k0, q0, q1, lane);
        }
    }
    __syncthreads();
    double* ps = a.psum + (size_t)blockIdx.x * 2 * a.bins;
    unsigned long long* pc = a.pcnt + (size_t)blockIdx.x * a.bins;
    for (int k = threadIdx.x; k < 2 * a.bins; k += kBlock) ps[k] = hs[k];
    for (int k = threadIdx.x; k < a.bins; k += kBlock) pc[k] = hc[k];
}

// sums[k] += sum over rows of ls[row][k]; counts likewise.
__global__ void __launch_bounds__(256) corr_reduce_kernel(const double* __restrict__ ls,
                                                          const unsigned long long* __restrict__ lc,
                                                          int rows, int bins,
                                                          double* __restrict__ sums,
                                                          unsigned long long* __restrict__ counts)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < 2 * bins) {
        double acc = 0.0;
        for (int g = 0; g < rows; ++g) acc += ls[(size_t)g * 2 * bins + k];
        sums[k] += acc;
    }
    if (k < bins) {
        unsigned long long acc = 0;
        for (int g = 0; g < rows; ++g) acc += lc[(size_t)g * bins + k];
        counts[k] += acc;
    }
}

}  // namespace

size_t corr_lds_bytes(int bins)
{
    return (size_t)bins * (2 * sizeof(double) + sizeof(unsigned long long));
}

int corr_workgroups(int dim, int bins, long long ncells)
{
    const size_t lds = corr_lds_bytes(bins);
    return dim == 3 ? resident_blocks(corr_kernel<3>, lds, ncells)
                    : resident_blocks(corr_kernel<2>, lds, ncells);
}

void launch_corr(const CorrArgs& a, int dim, int blocks, hipStream_t s)
{
    const size_t lds = corr_lds_bytes(a.bins);
    if (dim == 3) {
        (void)hipFuncSetAttribute((const void*)corr_kernel<3>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(corr_kernel<3>, dim3(blocks), dim3(kBlock), lds, s, a);
    } else {
        (void)hipFuncSetAttribute((const void*)corr_kernel<2>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(corr_kernel<2>, dim3(blocks), dim3(kBlock), lds, s, a);
    }
    const int rows = partial_rows(blocks);
    hipLaunchKernelGGL(partial_sum_stage1<double>, dim3((2 * a.bins + 63) / 64, rows), dim3(256), 0,
                       s, a.psum, blocks, 2 * a.bins, kPartialRowsPer, a.lsum);
    hipLaunchKernelGGL(partial_sum_stage1<unsigned long long>, dim3((a.bins + 63) / 64, rows),
                       dim3(256), 0, s, a.pcnt, blocks, a.bins, kPartialRowsPer, a.lcnt);
    hipLaunchKernelGGL(corr_reduce_kernel, dim3((2 * a.bins + 255) / 256), dim3(256), 0, s, a.lsum,
                       a.lcnt, rows, a.bins, a.sums, a.counts);
}

}  // namespace ppa
