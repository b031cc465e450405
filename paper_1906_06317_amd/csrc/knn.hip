// k nearest neighbours over the cell list (the paper's neighbor query with a
// neighbour-count argument, "Implementation"; a row lists its neighbours by
// increasing distance, ties broken by point index).
//
// The cells of this query are sized from the mean spacing: their width is a
// little above the expected distance of the k-th neighbour at the points'
// density, so the 27-cell (2D: 9) block around a query usually holds its k
// nearest.  The block guarantees every query a radius R, the distance from
// the query to the nearest face of the block: a point closer than R lies in
// the block, so the k smallest distances of the block, when below R, are the
// k nearest overall.
//
// Common path, one wavefront per home cell (candidates in 64-wide register
// slots, each query in scalar registers):
//   1. squared distance of every candidate (difference of cell-local
//      coordinates);
//   2. a threshold T <= R^2 with k <= #{d^2 < T} <= 64, found by counting
//      ballots: first a guess carried over from the previous query of the
//      cell (neighbouring queries have similar k-th distances), then
//      widening or bisection;
//   3. the candidates under T are compacted into LDS as 64-bit keys
//      (d^2 bits, index): the keys order exactly as (r^2, j);
//   4. each lane ranks its key among them; lanes of rank < k write the row,
//      already sorted.
// Queries this path cannot settle (fewer than k candidates closer than R,
// more than 64 candidates tied under every useful threshold, or a home cell
// with more candidates than the register slots hold) go to a list handled by
// a second kernel: one wavefront per query, shells of cells grown until the
// k-th distance is below the shell's guaranteed radius, the best k kept
// sorted in LDS and merged with each new batch of candidates by rank.
#include "pair_common.hpp"

namespace ppa {

namespace {

using namespace pair;

constexpr int kKnnSlots = 4;    // register slots of the common path (256 candidates)
constexpr int kKnnIter = 16;    // threshold refinements before a query is deferred
constexpr float kKnnGrow = 1.1f;  // next guess: this times the previous k-th r^2
constexpr unsigned long long kNoKey = ~0ull;

__device__ __forceinline__ unsigned long long knn_key(float d2, int id)
{
    return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)id;
}

__device__ __forceinline__ float key_d2(unsigned long long key)
{
    return __uint_as_float((unsigned)(key >> 32));
}

// Squared radius the 27-cell (9-cell) block around a query's home cell
// guarantees, for a query at cell-local position (x, y, z): the distance to
// the block's nearest face, (s + 1/2 - |t_k|) cell widths for the shell of
// half-width s, with t_k the query's offset from the cell centre in cell
// units.  Shrunk slightly so rounding of the stored coordinates never
// matters.
template <int DIM>
__device__ __forceinline__ float guaranteed_r2(const KnnGeom& K, float x, float y, float z,
                                               float s)
{
    const float fx = fmaf(K.minv[0][2], z, fmaf(K.minv[0][1], y, K.minv[0][0] * x));
    const float fy = fmaf(K.minv[1][2], z, K.minv[1][1] * y);
    const float fz = K.minv[2][2] * z;
    float r = (s + 0.5f - fabsf(fx * K.nf[0])) * K.cellw[0];
    r = fminf(r, (s + 0.5f - fabsf(fy * K.nf[1])) * K.cellw[1]);
    if (DIM == 3) r = fminf(r, (s + 0.5f - fabsf(fz * K.nf[2])) * K.cellw[2]);
    r = fmaxf(r, 0.f) * 0.99999f;
    return r * r;
}

// Row length a query must reach when no r_guard limits it: k, or every
// other point when there are fewer.
__device__ __forceinline__ int expected_len(const KnnGeom& K, int qid)
{
    const int elig = K.n_points - ((K.excl && qid < K.n_points) ? 1 : 0);
    return min(K.k, elig);
}

struct KnnLds {
    alignas(16) unsigned long long key[kWave];
    StencilLds st;
};

// Candidates of one home cell in NS register slots (entries past the end
// are far away and never selected).
template <int DIM, int NS>
struct KnnSlots {
    float x[NS], y[NS], z[NS];
    int id[NS];

    __device__ __forceinline__ void load(const PairIn& in, const PairGeom& G, const StencilLds& S,
                                         const float4* off, int C, int lane)
    {
        int before = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            x[s] = y[s] = z[s] = kFar;
            id[s] = -1;
            fetch_slot<DIM>(in, G.nsten, S, off, 0, s, C, lane, before, x[s], y[s], z[s], id[s]);
        }
    }
};

template <int DIM, int NS>
__device__ __forceinline__ int count_below(const float (&d2)[NS], float T)
{
    int c = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) c += __popcll(__ballot(d2[s] < T));
    return c;
}

// Outcome of the common path for one query.
enum { kRowFull = 0, kRowShort = 1, kRowDefer = 2 };

template <int DIM, int NS>
__device__ __forceinline__ void knn_tile(const KnnArgs& a, const PairIn& in, const StencilLds& S,
                                         const float4* off, KnnLds& W, int C, int q0, int q1,
                                         int lane)
{
    const KnnGeom& K = a.knn;
    const int k = K.k;
    KnnSlots<DIM, NS> c;
    c.load(in, a.geom, S, off, C, lane);
    float tg = K.t0;  // threshold guess, r^2
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        QueryChunk Q;
        Q.load(in, c0, q1 - c0, lane);
        // per lane: the squared search bound of its own query and whether the
        // block (not r_guard or half the box) sets it
        const float rb2 = guaranteed_r2<DIM>(K, Q.q.x, Q.q.y, Q.q.z, 1.f);
        const float thi_l = fminf(rb2, K.lim2);
        const int blk_l = rb2 < K.lim2 ? 1 : 0;
        unsigned long long defer = 0ull;
        int len_v = 0;
        for (int t = 0; t < Q.n; ++t) {
            const float qx = lane_off(Q.q.x, t), qy = lane_off(Q.q.y, t);
            const float qz = DIM == 3 ? lane_off(Q.q.z, t) : 0.f;
            const int qid = lane_of(Q.my_id(), t);
            const float thi = lane_off(thi_l, t);
            const int blk = lane_of(blk_l, t);
            float d2[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                d2[s] = dist2<DIM>(c.x[s] - qx, c.y[s] - qy, c.z[s] - qz);
                if (K.excl && c.id[s] == qid) d2[s] = kFar;
            }
            // threshold with k <= count <= 64 (or every candidate under thi)
            float T = fminf(tg, thi);
            float lo = 0.f, hi = thi;
            bool hi_set = false;
            int state = kRowDefer, cnt = 0;
            for (int it = 0; it < kKnnIter; ++it) {
                cnt = count_below<DIM, NS>(d2, T);
                if (cnt >= k && cnt <= kWave) {
                    state = kRowFull;
                    break;
                }
                if (cnt < k) {
                    if (T >= thi) {
                        state = blk ? kRowDefer : kRowShort;
                        break;
                    }
                    lo = T;
                    T = hi_set ? 0.5f * (T + hi) : fminf(fmaxf(T * 1.5f, 1e-3f * K.t0), thi);
                } else {
                    hi = T;
                    hi_set = true;
                    T = 0.5f * (lo + T);
                }
            }
            if (state == kRowDefer) {
                defer |= 1ull << t;
                continue;
            }
            // compact the candidates under T (the rest of the buffer holds
            // keys that sort last) and rank them
            W.key[lane] = kNoKey;
            int nb = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const bool h = d2[s] < T;
                const unsigned long long m = __ballot(h);
                if (h) W.key[nb + (int)lane_prefix(m)] = knn_key(d2[s], c.id[s]);
                nb += __popcll(m);
            }
            wave_sync();
            // Each key is ranked by one lane of every group of gsz >= cnt
            // lanes; the groups split the buffer between them (four keys per
            // step, independent LDS reads) and their partial ranks are summed
            // across groups.  Past cnt the buffer holds keys that sort last.
            const int gsz = cnt <= 16 ? 16 : (cnt <= 32 ? 32 : kWave);
            const int ng = kWave / gsz;
            const int share = ((cnt + ng - 1) / ng + 3) & ~3;
            const unsigned long long mine = W.key[lane & (gsz - 1)];
            const unsigned long long* part = &W.key[(lane / gsz) * share];
            int r = 0;
            for (int u = 0; u < share; u += 4) {
                const ulonglong2 a2 = *reinterpret_cast<const ulonglong2*>(&part[u]);
                const ulonglong2 b2 = *reinterpret_cast<const ulonglong2*>(&part[u + 2]);
                r += (a2.x < mine ? 1 : 0) + (a2.y < mine ? 1 : 0) + (b2.x < mine ? 1 : 0) +
                     (b2.y < mine ? 1 : 0);
            }
            if (gsz <= 32) r = pair_sum32(r);
            if (gsz <= 16) r = pair_sum16(r);
            const int len = state == kRowFull ? k : cnt;
            if (lane < cnt && r < len) {
                const long long o = (long long)k * qid + r;
                a.out_idx[o] = (int)(unsigned)mine;
                if (a.out_dist) a.out_dist[o] = fast_sqrt(key_d2(mine));
            }
            if (state == kRowFull) {
                const unsigned long long km = __ballot(lane < cnt && r == k - 1);
                const float kd2 = key_d2(lane_of64((long long)mine, __ffsll((long long)km) - 1));
                tg = fmaxf(kKnnGrow * kd2, 1e-3f * K.t0);
            } else if (!K.guard && len < expected_len(K, qid) && lane == 0) {
                atomicOr(a.status, kStatusRange);  // a neighbour lies beyond half the box
            }
            len_v = lane == t ? len : len_v;
            wave_sync();
        }
        if (a.row_len && lane < Q.n && !((defer >> lane) & 1ull)) a.row_len[Q.my_id()] = len_v;
        if (defer) {
            const int nd = __popcll(defer);
            int base = 0;
            if (lane == 0) base = (int)atomicAdd(a.n_deferred, (unsigned long long)nd);
            base = uniform(base);
            if ((defer >> lane) & 1ull) a.deferred[base + (int)lane_prefix(defer)] = c0 + lane;
        }
    }
}

// Every query of a home cell to the deferred list (stencil too large for the
// register slots).
__device__ __forceinline__ void defer_all(const KnnArgs& a, int q0, int q1, int lane)
{
    const int nd = q1 - q0;
    int base = 0;
    if (lane == 0) base = (int)atomicAdd(a.n_deferred, (unsigned long long)nd);
    base = uniform(base);
    for (int i = lane; i < nd; i += kWave) a.deferred[base + i] = q0 + i;
}

// Six wavefronts per SIMD (80 VGPRs, a few spilled in set-up code): the
// 2^20-point FCC query at k = 12 took 0.355 ms at five, 0.340 at six and
// 0.347 at eight.
template <int DIM>
__global__ void __launch_bounds__(kBlock, 6) knn_kernel(const KnnArgs a)
{
    __shared__ float4 s_off[27];
    __shared__ KnnLds s_w[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    KnnLds& W = s_w[wv];
    const PairGeom& G = a.geom;
    if (threadIdx.x < 27)
        s_off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1],
                                         G.off[threadIdx.x][2], 0.f);
    __syncthreads();
    const PairIn in{a.cand, a.cand_start, a.qsorted, a.q_start};
    int t0, t1, stride;
    wave_tiles_interleaved<kWavesPerBlock>(G.ncells, wv, t0, t1, stride);
    for (int tile = t0; tile < t1; tile += stride) {
        const int q0 = in.q_start[tile];
        const int q1 = in.q_start[tile + 1];
        if (q0 == q1) continue;
        const int C = stencil<DIM>(in, G, tile, lane, W.st);
        const int ns = (C + kWave - 1) / kWave;
        switch (ns) {
        case 0:
        case 1: knn_tile<DIM, 1>(a, in, W.st, s_off, W, C, q0, q1, lane); break;
        case 2: knn_tile<DIM, 2>(a, in, W.st, s_off, W, C, q0, q1, lane); break;
        case 3: knn_tile<DIM, 3>(a, in, W.st, s_off, W, C, q0, q1, lane); break;
        case 4: knn_tile<DIM, 4>(a, in, W.st, s_off, W, C, q0, q1, lane); break;
        default: defer_all(a, q0, q1, lane);
        }
        static_assert(kKnnSlots == 4, "switch above covers kKnnSlots slots");
    }
}

// ---------------------------------------------------------------------------
// Deferred queries: one wavefront per query, growing shells of cells.
// ---------------------------------------------------------------------------
struct FarLds {
    unsigned long long best[kWave];  // the best keys so far, sorted
    unsigned long long fresh[kWave]; // keys of one batch that beat the k-th
};

__device__ __forceinline__ int wrap(int c, int n)
{
    c %= n;
    return c < 0 ? c + n : c;
}

// Merges the batch of lanes in `m` (their keys in `key`) into the sorted best
// list of `cnt` keys, keeping the first k.  Keys are distinct.
__device__ __forceinline__ void merge_batch(FarLds& W, unsigned long long m,
                                            unsigned long long key, int lane, int k, int& cnt)
{
    const int mn = __popcll(m);
    if ((m >> lane) & 1ull) W.fresh[lane_prefix(m)] = key;
    wave_sync();
    const unsigned long long e = lane < cnt ? W.best[lane] : kNoKey;
    const unsigned long long f = lane < mn ? W.fresh[lane] : kNoKey;
    int shift = 0, rf = 0;
    for (int u = 0; u < mn; ++u) {
        const unsigned long long ku = W.fresh[u];
        shift += ku < e ? 1 : 0;
        rf += ku < f ? 1 : 0;
    }
    for (int u = 0; u < cnt; ++u) rf += W.best[u] < f ? 1 : 0;
    wave_sync();
    if (lane < cnt && lane + shift < k) W.best[lane + shift] = e;
    if (lane < mn && rf < k) W.best[rf] = f;
    cnt = min(k, cnt + mn);
    wave_sync();
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) knn_far_kernel(const KnnArgs a)
{
    __shared__ FarLds s_w[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    FarLds& W = s_w[wv];
    const KnnGeom& K = a.knn;
    const PairGeom& G = a.geom;
    const int k = K.k;
    const int ndef = (int)*a.n_deferred;
    const int nwaves = gridDim.x * kWavesPerBlock;
    for (int d = blockIdx.x * kWavesPerBlock + wv; d < ndef; d += nwaves) {
        const int p = uniform(a.deferred[d]);
        const float4 qv = a.qsorted[p];
        const float qx = uniformf(qv.x), qy = uniformf(qv.y);
        const float qz = DIM == 3 ? uniformf(qv.z) : 0.f;
        const int qid = uniform(__float_as_int(qv.w));
        const int home = uniform(a.q_cell_of[qid]);
        const int hx = home % G.n[0];
        const int hy = (home / G.n[0]) % G.n[1];
        const int hz = home / (G.n[0] * G.n[1]);
        int cnt = 0;
        unsigned long long kth = kNoKey;
        for (int s = 1; s <= K.smax; ++s) {
            const int sz = DIM == 3 ? s : 0;
            for (int dz = -sz; dz <= sz; ++dz)
                for (int dy = -s; dy <= s; ++dy) {
                    // the shell's cells: whole rows on its faces, the two end
                    // cells elsewhere (the first shell is the whole block)
                    const bool face = s == 1 || dy == -s || dy == s || (DIM == 3 && (dz == -s || dz == s));
                    const int step = face ? 1 : 2 * s;
                    for (int dx = -s; dx <= s; dx += step) {
                        const int cell =
                            (wrap(hz + dz, G.n[2]) * G.n[1] + wrap(hy + dy, G.n[1])) * G.n[0] +
                            wrap(hx + dx, G.n[0]);
                        const double fx = (double)dx / G.n[0], fy = (double)dy / G.n[1],
                                     fz = (double)dz / G.n[2];
                        const float ox = (float)(K.M[0][0] * fx + K.M[0][1] * fy + K.M[0][2] * fz);
                        const float oy = (float)(K.M[1][1] * fy + K.M[1][2] * fz);
                        const float oz = (float)(K.M[2][2] * fz);
                        const int b = a.cand_start[cell], e = a.cand_start[cell + 1];
                        for (int j0 = b; j0 < e; j0 += kWave) {
                            const int j = j0 + lane;
                            unsigned long long key = kNoKey;
                            if (j < e) {
                                const float4 v = a.cand[j];
                                const int id = __float_as_int(v.w);
                                const float d2 =
                                    dist2<DIM>(v.x + ox - qx, v.y + oy - qy, v.z + oz - qz);
                                if (d2 < K.lim2 && !(K.excl && id == qid)) key = knn_key(d2, id);
                            }
                            const unsigned long long m =
                                __ballot(key != kNoKey && (cnt < k || key < kth));
                            if (m) {
                                merge_batch(W, m, key, lane, k, cnt);
                                if (cnt == k) kth = W.best[k - 1];
                            }
                        }
                    }
                }
            const float rs2 = guaranteed_r2<DIM>(K, qx, qy, qz, (float)s);
            if (cnt == k && key_d2(kth) < rs2) break;  // nothing outside can beat the k-th
            if (rs2 >= K.lim2) break;                  // every point within the limit seen
        }
        if (lane < cnt) {
            const unsigned long long key = W.best[lane];
            const long long o = (long long)k * qid + lane;
            a.out_idx[o] = (int)(unsigned)key;
            if (a.out_dist) a.out_dist[o] = fast_sqrt(key_d2(key));
        }
        if (lane == 0) {
            if (a.row_len) a.row_len[qid] = cnt;
            if (!K.guard && cnt < expected_len(K, qid)) atomicOr(a.status, kStatusRange);
        }
        wave_sync();
    }
}

// Full rows: offsets[i] = k i, and the pair count.
__global__ void knn_offsets_kernel(int64_t* __restrict__ offsets, int64_t nq, int k,
                                   int64_t* __restrict__ n_pairs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= nq) offsets[i] = (int64_t)k * i;
    if (i == 0) *n_pairs = (int64_t)k * nq;
}

// Rows that may be short: rows staged at stride k are packed at their CSR
// offsets.  One thread per staged entry.
__global__ void knn_pack_kernel(int64_t nq, int k, const int32_t* __restrict__ row_len,
                                const int64_t* __restrict__ offsets,
                                const int32_t* __restrict__ st_idx,
                                const float* __restrict__ st_dist, int32_t* __restrict__ point_idx,
                                float* __restrict__ dist)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq * k) return;
    const int64_t i = t / k;
    const int e = (int)(t - i * k);
    if (e >= row_len[i]) return;
    point_idx[offsets[i] + e] = st_idx[t];
    if (dist) dist[offsets[i] + e] = st_dist[t];
}

}  // namespace

void launch_knn(const KnnArgs& a, int dim, hipStream_t s)
{
    if (dim == 3) {
        const int blocks = resident_blocks(knn_kernel<3>, 0, a.geom.ncells);
        hipLaunchKernelGGL(knn_kernel<3>, dim3(blocks), dim3(kBlock), 0, s, a);
        const int far = resident_blocks(knn_far_kernel<3>, 0, 1LL << 40);
        hipLaunchKernelGGL(knn_far_kernel<3>, dim3(far), dim3(kBlock), 0, s, a);
    } else {
        const int blocks = resident_blocks(knn_kernel<2>, 0, a.geom.ncells);
        hipLaunchKernelGGL(knn_kernel<2>, dim3(blocks), dim3(kBlock), 0, s, a);
        const int far = resident_blocks(knn_far_kernel<2>, 0, 1LL << 40);
        hipLaunchKernelGGL(knn_far_kernel<2>, dim3(far), dim3(kBlock), 0, s, a);
    }
}

void launch_knn_offsets(int64_t* offsets, int64_t nq, int k, int64_t* n_pairs, hipStream_t s)
{
    const unsigned blocks = (unsigned)((nq + 1 + 255) / 256);
    hipLaunchKernelGGL(knn_offsets_kernel, dim3(blocks), dim3(256), 0, s, offsets, nq, k, n_pairs);
}

void launch_knn_pack(int64_t nq, int k, const int32_t* row_len, const int64_t* offsets,
                     const int32_t* st_idx, const float* st_dist, int32_t* point_idx, float* dist,
                     hipStream_t s)
{
    const int64_t total = nq * k;
    if (total == 0) return;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(knn_pack_kernel, dim3(blocks), dim3(256), 0, s, nq, k, row_len, offsets,
                       st_idx, st_dist, point_idx, dist);
}

}  // namespace ppa
