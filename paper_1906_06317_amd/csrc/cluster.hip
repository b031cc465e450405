// Clusters of the cluster module (the paper's analysis modules: cluster
// membership is defined by neighbour bonds): the connected components of
// the undirected graph on n points whose edges are the pairs of a
// NeighborList.  labels[i] is the smallest point index of i's component;
// optional outputs number the components in order of that index
// (cluster_idx), count their points (sizes) and count them (n_clusters).
//
// Union-find over the labels array as the parent forest.  A seed pass
// points every point at its smallest listed neighbour; hooking rounds over
// all bonds (the larger label pointed at the smaller by atomic minimum, a
// step of the Shiloach-Vishkin kind) alternate with passes that point every
// node at its root, until a round changes nothing, so the large components
// form flat; a last lock-free union pass over every bond makes the result
// exact, most of its unions ending after two one-step finds.  Finds in the union passes halve paths with plain stores; the
// compress passes only read the forest and write their own entries.  A union finds
// both roots and links the larger under the smaller with a compare-and-swap
// on the larger root's parent; a failed swap means that root was linked
// meanwhile, and the union continues from its new parent.  Parents only
// ever point to smaller indices, so the root of a component is its smallest
// index, every find ends, and the larger of the two roots a union works on
// shrinks on every retry, so every union ends.  A compress pass sets every
// label to its root, each lane writing only its own entry (by atomic
// minimum, which keeps a root a concurrent union may have written); the
// compact numbering is a scan over the roots.  For a list the caller declares
// symmetric, the rounds sample two bonds per row and the union pass skips the
// points of the largest sampled component (their bonds to other points are
// in those points' rows).
#include "internal.hpp"

namespace ppa {

namespace {

constexpr int kClBlock = 256;
constexpr int kClRounds = kClusterRounds;  // hooking rounds at most
constexpr int kClSampled = 2;              // bonds per row the rounds hook (symmetric lists)

__device__ __forceinline__ int parent_of(int* p, int x)
{
    return __hip_atomic_load(&p[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, without writes: the lanes of a large component all walk
// through the few nodes near its root, and writes there would serialise.
__device__ __forceinline__ int root_of(int* p, int x)
{
    int px;
    while ((px = parent_of(p, x)) != x) x = px;
    return x;
}

// Root of x, halving the path on the way (the union passes): each visited
// node is pointed at its grandparent by a plain store.  Only non-roots are
// written, every value is an ancestor, and no other kind of write to a
// non-root happens during a union pass, so the forest stays valid.
__device__ __forceinline__ int root_halving(int* p, int x)
{
    while (true) {
        const int px = parent_of(p, x);
        if (px == x) return x;
        const int gp = parent_of(p, px);
        if (gp == px) return px;
        __hip_atomic_store(&p[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

__device__ void unite(int* p, int a, int b)
{
    while (true) {
        a = root_halving(p, a);
        b = root_halving(p, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        // a > b: hang root a under b unless a stopped being a root
        const int old = atomicCAS(&p[a], a, b);
        if (old == a) return;
        a = old;
    }
}

// Zeroes `words` 32-bit words at z (status, scan state) and words2 at z2
// (sizes); with n > 0 also sets labels[i] = i.
__global__ void __launch_bounds__(kClBlock) cl_init_kernel(int n, int* labels, unsigned* z,
                                                           long long words, unsigned* z2,
                                                           long long words2)
{
    const long long stride = (long long)gridDim.x * kClBlock;
    const long long t = (long long)blockIdx.x * kClBlock + threadIdx.x;
    for (long long i = t; i < n; i += stride) labels[i] = (int)i;
    for (long long i = t; i < words; i += stride) z[i] = 0u;
    for (long long i = t; i < words2; i += stride) z2[i] = 0u;
}

// Checked bounds of row i of the list (empty when the row is invalid).
__device__ __forceinline__ bool row_bounds(const int64_t* offsets, int i, long long capacity,
                                           unsigned* status, long long& e0, long long& e1)
{
    e0 = offsets[i];
    e1 = offsets[i + 1];
    if (e0 < 0 || e1 < e0 || e1 > capacity) {
        atomicOr(status, kStatusBadList);
        e0 = e1 = 0;
        return false;
    }
    return true;
}

// First links: every point to the smallest of itself and its listed
// neighbours (each lane writes only its own parent, a smaller index, so the
// result is a valid forest of unions without any atomics).
__global__ void __launch_bounds__(kClBlock) cl_seed_kernel(const int64_t* __restrict__ offsets,
                                                           const int32_t* __restrict__ idx, int n,
                                                           long long capacity, int* labels,
                                                           unsigned* status)
{
    const int i = blockIdx.x * kClBlock + threadIdx.x;
    if (i >= n) return;
    long long e0, e1;
    row_bounds(offsets, i, capacity, status, e0, e1);
    int m = i;
    for (long long e = e0; e < e1; ++e) {
        const int j = idx[e];
        if (j < 0 || j >= n) {
            atomicOr(status, kStatusBadList);
            continue;
        }
        m = j < m ? j : m;
    }
    labels[i] = m;
}

// One hooking round over every bond: the larger of the two current labels
// is pointed (atomic minimum) at the smaller.  A hook may replace an earlier
// parent, dropping that link, but it only ever joins bonded points and keeps
// every parent below its node, so the forest stays a valid subset of the
// components; the closing union pass restores anything dropped.
__global__ void __launch_bounds__(kClBlock) cl_sv_kernel(const int64_t* __restrict__ offsets,
                                                         const int32_t* __restrict__ idx, int n,
                                                         long long capacity, int first,
                                                         int* labels, const int* prev_changed,
                                                         int* changed)
{
    // nothing moved in the previous round: the forest has converged
    if (prev_changed && __hip_atomic_load(prev_changed, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) == 0)
        return;
    const int i = blockIdx.x * kClBlock + threadIdx.x;
    if (i >= n) return;
    long long e0 = offsets[i], e1 = offsets[i + 1];
    if (e0 < 0 || e1 < e0 || e1 > capacity) return;
    if (first > 0 && e1 > e0 + first) e1 = e0 + first;  // a sample of the bonds
    // cached loads: a stale label is an older ancestor, which only makes a
    // hook weaker; the closing union pass is exact either way
    const int li = labels[i];
    bool moved = false;
    for (long long e = e0; e < e1; ++e) {
        const int j = idx[e];
        if (j < 0 || j >= n || j == i) continue;
        const int lj = labels[j];
        if (lj == li) continue;
        const int hi = lj < li ? li : lj, lo = lj < li ? lj : li;
        // read first: in a large component the target is one shared root
        if (labels[hi] > lo) {
            atomicMin(&labels[hi], lo);
            moved = true;
        }
    }
    if (__ballot(moved) && (threadIdx.x & (warpSize - 1)) == __ffsll((long long)__ballot(moved)) - 1)
        atomicOr(changed, 1);
}

// Unites point i with the neighbour at position `pos` of its row (pos >= 0:
// one sampling round), or with every neighbour (pos < 0).
__global__ void __launch_bounds__(kClBlock) cl_hook_kernel(const int64_t* __restrict__ offsets,
                                                           const int32_t* __restrict__ idx, int n,
                                                           long long capacity, int pos,
                                                           const int* giant, int* labels)
{
    const int i = blockIdx.x * kClBlock + threadIdx.x;
    if (i >= n) return;
    // a symmetric list: a point already in the sampled largest component
    // leaves its bonds to the other ends (a bond to a point outside is in
    // that point's row; a bond inside joins nothing new)
    if (giant && labels[i] == *giant) return;
    // bounds were checked (and reported) by the seed pass
    long long e0 = offsets[i], e1 = offsets[i + 1];
    if (e0 < 0 || e1 < e0 || e1 > capacity) return;
    if (pos >= 0) {
        if (e0 + pos >= e1) return;
        e0 += pos;
        e1 = e0 + 1;
    }
    for (long long e = e0; e < e1; ++e) {
        const int j = idx[e];
        if (j < 0 || j >= n || j == i) continue;
        unite(labels, i, j);
    }
}

// The root most of kClSamples evenly spaced points share (ties: the smaller
// root), after a compress pass: one workgroup, the samples in LDS, each
// thread counting the samples equal to its own.
constexpr int kClSamples = 1024;

__global__ void __launch_bounds__(kClSamples) cl_giant_kernel(int n, const int* labels, int* giant)
{
    __shared__ int s_lab[kClSamples];
    __shared__ unsigned long long s_best[kClSamples / 64];
    const int t = threadIdx.x;
    const int lab = labels[(int)(((long long)t * n) / kClSamples)];
    s_lab[t] = lab;
    __syncthreads();
    int c = 0;
    for (int u = 0; u < kClSamples; ++u) c += s_lab[u] == lab ? 1 : 0;
    // largest count first, then smallest root: one 64-bit key per thread
    unsigned long long key = ((unsigned long long)(unsigned)c << 32) | (unsigned)(0x7fffffff - lab);
    for (int sh = 32; sh > 0; sh >>= 1) {
        const unsigned long long o = __shfl_xor(key, sh);
        key = o > key ? o : key;
    }
    if ((t & 63) == 0) s_best[t >> 6] = key;
    __syncthreads();
    if (t == 0) {
        unsigned long long b = s_best[0];
        for (int w = 1; w < kClSamples / 64; ++w) b = s_best[w] > b ? s_best[w] : b;
        *giant = 0x7fffffff - (int)(unsigned)(b & 0xffffffffull);
    }
}

__global__ void __launch_bounds__(kClBlock) cl_compress_kernel(int n, int* labels, int* is_root,
                                                               const int* changed)
{
    if (changed && __hip_atomic_load(changed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        return;  // the hooking round before changed nothing
    const int i = blockIdx.x * kClBlock + threadIdx.x;
    if (i >= n) return;
    // each lane writes only its own entry; the minimum keeps a root that a
    // union may have written since (no other lane writes this entry here).
    // Between hooking rounds a cached walk is enough (a stale root is still
    // an ancestor); the last pass reads coherently.
    int r;
    if (changed) {
        int x = i, px;
        while ((px = labels[x]) != x) x = px;
        r = x;
    } else {
        r = root_of(labels, i);
    }
    atomicMin(&labels[i], r);
    if (is_root) is_root[i] = r == i ? 1 : 0;
}

constexpr int kClIndexBlock = 1024;

__global__ void __launch_bounds__(kClIndexBlock) cl_index_kernel(int n,
                                                                 const int* __restrict__ labels,
                                                                 const int64_t* __restrict__ rank,
                                                                 int32_t* cluster_idx,
                                                                 int32_t* sizes)
{
    __shared__ int s_c[kClIndexBlock / 64], s_n[kClIndexBlock / 64];
    const int i = blockIdx.x * kClIndexBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool live = i < n;
    const int c = live ? (int)rank[labels[i]] : -1;
    if (live && cluster_idx) cluster_idx[i] = c;
    if (!sizes) return;
    // the cluster of each wavefront's first point is counted for the whole
    // workgroup: the wavefronts that share it (all of them inside a large
    // cluster) add one total with one atomic
    const int c0 = __builtin_amdgcn_readfirstlane(c);
    const unsigned long long m0 = __ballot(live && c == c0);
    if (lane == 0) {
        s_c[wv] = c0;
        s_n[wv] = __popcll(m0);
    }
    __syncthreads();
    if (threadIdx.x < kClIndexBlock / 64) {
        const int w = threadIdx.x;
        // the first wavefront holding this cluster adds for all that hold it
        int first = w, total = 0;
        for (int u = 0; u < kClIndexBlock / 64; ++u)
            if (s_c[u] == s_c[w]) {
                if (u < first) first = u;
                total += s_n[u];
            }
        if (first == w && s_c[w] >= 0 && total > 0) atomicAdd(&sizes[s_c[w]], total);
    }
    // the other points: one atomic per distinct cluster of the wavefront for
    // three more rounds, then one by one
    bool done = !live || c == c0;
    for (int round = 0; round < 3; ++round) {
        const unsigned long long pend = __ballot(!done);
        if (!pend) break;
        const int cr = __builtin_amdgcn_readlane(c, __ffsll((unsigned long long)pend) - 1);
        const unsigned long long m = __ballot(!done && c == cr);
        if (!done && c == cr) {
            const unsigned below = __builtin_amdgcn_mbcnt_hi(
                (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            if (below == 0) atomicAdd(&sizes[cr], __popcll(m));
            done = true;
        }
    }
    if (!done) atomicAdd(&sizes[c], 1);
}

inline int blocks_for(long long n) { return (int)((n + kClBlock - 1) / kClBlock); }

}  // namespace

void launch_cluster(const ClusterArgs& a, hipStream_t s)
{
    const int n = (int)a.n;
    const bool ranks = a.cluster_idx || a.sizes || a.n_clusters;
    const long long zwords = (long long)(a.zero_bytes / 4);
    const long long swords = a.sizes ? (long long)n : 0;
    long long most = n > zwords ? n : zwords;
    if (swords > most) most = swords;
    const int ib = (int)(most < 1 ? 1 : (blocks_for(most) < 4096 ? blocks_for(most) : 4096));
    hipLaunchKernelGGL(cl_init_kernel, dim3(ib), dim3(kClBlock), 0, s, 0, a.labels, a.zero,
                       zwords, (unsigned*)a.sizes, swords);
    if (n == 0) return;
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(cl_seed_kernel, dim3(nb), dim3(kClBlock), 0, s, a.offsets, a.idx, n,
                       a.capacity, a.labels, a.status);
    hipLaunchKernelGGL(cl_compress_kernel, dim3(nb), dim3(kClBlock), 0, s, n, a.labels, nullptr,
                       nullptr);
    // hooking rounds, each flattened, until one changes nothing (later
    // rounds then return at once: no host synchronisation); then the union
    // pass over every bond makes the result exact whatever the rounds left
    // sparse lists (below about 3 bonds per point, under the percolation
    // threshold of random geometric graphs) form no large component: the
    // union pass alone is faster there
    // With a symmetric list (every bond in both rows) the rounds hook only
    // the first kClSampled bonds of each row; the root most sampled points
    // share then marks the largest component, whose points the union pass
    // skips (the sampling of the Afforest method).  On the 2^20-point
    // uniform system: r = 1.2 1.73 -> 1.32 ms, r = 1.6 2.49 -> 1.28 ms.
    const int rounds = a.capacity < 3 * (long long)n ? 0 : kClRounds;
    const int first = a.symmetric ? kClSampled : 0;
    for (int r = 0; r < rounds; ++r) {
        const int* prev = r > 0 ? a.round_flags + (r - 1) : nullptr;
        hipLaunchKernelGGL(cl_sv_kernel, dim3(nb), dim3(kClBlock), 0, s, a.offsets, a.idx, n,
                           a.capacity, first, a.labels, prev, a.round_flags + r);
        hipLaunchKernelGGL(cl_compress_kernel, dim3(nb), dim3(kClBlock), 0, s, n, a.labels,
                           nullptr, a.round_flags + r);
    }
    const bool skip_giant = a.symmetric && rounds > 0;  // no large component without rounds
    if (skip_giant) {
        // the last round's compress read a cached walk: one exact pass first
        hipLaunchKernelGGL(cl_compress_kernel, dim3(nb), dim3(kClBlock), 0, s, n, a.labels,
                           nullptr, nullptr);
        hipLaunchKernelGGL(cl_giant_kernel, dim3(1), dim3(kClSamples), 0, s, n, a.labels,
                           a.giant);
    }
    hipLaunchKernelGGL(cl_hook_kernel, dim3(nb), dim3(kClBlock), 0, s, a.offsets, a.idx, n,
                       a.capacity, -1, skip_giant ? a.giant : nullptr, a.labels);
    hipLaunchKernelGGL(cl_compress_kernel, dim3(nb), dim3(kClBlock), 0, s, n, a.labels,
                       ranks ? a.is_root : nullptr, nullptr);
    if (!ranks) return;
    launch_scan_i64_total(a.is_root, a.rank, n, a.scan_flags, a.ticket,
                          (unsigned long long*)a.n_clusters, s);
    if (a.cluster_idx || a.sizes)
        hipLaunchKernelGGL(cl_index_kernel, dim3((n + kClIndexBlock - 1) / kClIndexBlock),
                           dim3(kClIndexBlock), 0, s, n, a.labels,
                           a.rank, a.cluster_idx, a.sizes);
}

}  // namespace ppa
