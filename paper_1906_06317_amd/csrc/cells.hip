// Cell-list build on the GPU: cell index, counting sort by cell, prefix scan.
//
// The paper's LinkCell finds neighbours with linked cell lists ("General
// Utilities").  Here the list is rebuilt as flat arrays suited to a GPU:
// every point gets a cell of a uniform grid in fractional coordinates, the
// points are counting-sorted by cell (counts by atomics, an exclusive
// decoupled look-back scan gives the cell starts, a scatter places them) and
// each cell's run is then ordered by point index so the layout does not
// depend on atomic arrival order.  Each point is stored relative to the
// centre of its cell, so a pair vector later is a small difference plus a
// per-stencil offset computed once in float64.
#include "internal.hpp"

namespace ppa {

namespace {

struct ZeroRanges {
    unsigned* ptr[8];
    long long words[8];
    int count;
};

__global__ void zero_kernel(ZeroRanges z)
{
    for (int r = 0; r < z.count; ++r) {
        unsigned* p = z.ptr[r];
        const long long nw = z.words[r];
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
             i += (long long)gridDim.x * blockDim.x)
            p[i] = 0u;
    }
}

constexpr int kAssignRounds = 16;  // grouping rounds; lanes left over take an atomic each

// Cell index and cell-centred local coordinates of point i, in float64;
// cells of this box are numbered from cell_base.  Writes cell_of[i] and
// local[i]; returns the cell.
__device__ __forceinline__ int locate_point(const float* __restrict__ pts, int64_t i,
                                            const AssignBox& B, int cell_base,
                                            int* __restrict__ cell_of,
                                            float4* __restrict__ local,
                                            unsigned* __restrict__ status)
{
    double p0 = (double)pts[3 * i];
    double p1 = (double)pts[3 * i + 1];
    double p2 = B.dim == 3 ? (double)pts[3 * i + 2] : 0.0;
    if (!(isfinite(p0) && isfinite(p1) && isfinite(p2))) {
        atomicOr(status, kStatusNonFinite);
        p0 = p1 = p2 = 0.0;
    }
    // fractional coordinates s = M^-1 p, shifted to u = s + 1/2 and folded into [0, 1)
    double u[3];
    u[2] = B.dim == 3 ? B.Minv[2][2] * p2 + 0.5 : 0.5;
    u[1] = B.Minv[1][1] * p1 + B.Minv[1][2] * p2 + 0.5;
    u[0] = B.Minv[0][0] * p0 + B.Minv[0][1] * p1 + B.Minv[0][2] * p2 + 0.5;
    int c[3];
    double f[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        u[k] -= floor(u[k]);
        int ck = (int)(u[k] * B.n[k]);
        ck = ck < 0 ? 0 : (ck >= B.ni[k] ? B.ni[k] - 1 : ck);
        c[k] = ck;
        f[k] = u[k] - ((double)ck + 0.5) * B.inv_n[k];
    }
    if (B.dim != 3) f[2] = 0.0;
    const double x = B.M[0][0] * f[0] + B.M[0][1] * f[1] + B.M[0][2] * f[2];
    const double y = B.M[1][1] * f[1] + B.M[1][2] * f[2];
    const double z = B.M[2][2] * f[2];
    const int cell = cell_base + (c[2] * B.ni[1] + c[1]) * B.ni[0] + c[0];
    cell_of[i] = cell;
    local[i] = make_float4((float)x, (float)y, (float)z, __int_as_float((int)i));
    return cell;
}

// locate_point, then a slot in the cell's run from the global counters.
__device__ __forceinline__ void assign_point(const float* __restrict__ pts, int64_t i,
                                             const AssignBox& B, int cell_base,
                                             int* __restrict__ cell_of, int* __restrict__ slot,
                                             float4* __restrict__ local,
                                             int* __restrict__ cell_count,
                                             unsigned* __restrict__ status)
{
    const int cell = locate_point(pts, i, B, cell_base, cell_of, local, status);
    // A slot in the cell's run.  Lanes of the wavefront (those active here)
    // that share a cell share one atomic: inputs ordered in space put few
    // distinct cells in a wavefront, and same-address atomics serialise.
    // The groups are found by ballots first, for a few rounds (lanes still
    // ungrouped, as in scattered input, stay alone); then every group's
    // first lane adds the group's size in one atomic instruction, and the
    // members take consecutive slots from its result.  Measured on the
    // 2^20-point FCC: 60 -> 19 us in lattice order, unchanged when shuffled.
    const int lane = (int)(threadIdx.x & (kWave - 1));
    unsigned long long pending = __ballot(1);
    int leader_of = lane, size = 1, rank = 0;
    for (int round = 0; round < kAssignRounds && pending; ++round) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int lc = __builtin_amdgcn_readlane(cell, leader);
        const unsigned long long grp = __ballot(cell == lc) & pending;
        if ((grp >> lane) & 1ull) {
            leader_of = leader;
            rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(grp >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((unsigned)grp, 0u));
        }
        if (lane == leader) size = __popcll(grp);
        pending &= ~grp;
    }
    int base = 0;
    if (leader_of == lane) base = atomicAdd(&cell_count[cell], size);
    const int my_slot = __shfl(base, leader_of) + rank;
    slot[i] = my_slot;
}

__global__ void __launch_bounds__(256) assign_kernel(const float* pts, int64_t n, AssignBox B,
                                                     int* cell_of, int* slot, float4* local,
                                                     int* cell_count, unsigned* status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    assign_point(pts, i, B, 0, cell_of, slot, local, cell_count, status);
}

// A batch: every point finds its frame (point_base[f] <= i < point_base[f+1])
// and is assigned in that frame's box; the cells of frame f are numbered
// from its cell_base, so all frames share one list.
__global__ void __launch_bounds__(256) assign_batch_kernel(const float* pts, int64_t n,
                                                           const FrameInfo* __restrict__ frames,
                                                           const int* __restrict__ point_base,
                                                           int nframes, int* cell_of, int* slot,
                                                           float4* local, int* cell_count,
                                                           unsigned* status)
{
    __shared__ int s_f;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x;
    if (threadIdx.x == 0) {
        int lo = 0, hi = nframes - 1;  // last frame starting at or before `first`
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (point_base[mid] <= first)
                lo = mid;
            else
                hi = mid - 1;
        }
        s_f = lo;
    }
    __syncthreads();
    const int64_t i = first + threadIdx.x;
    if (i >= n) return;
    int f = s_f;
    while (f + 1 < nframes && point_base[f + 1] <= i) ++f;
    // one pass per distinct frame of the wave, so each box is read uniformly;
    // the points of chunked frames are counted by assign_chunks_kernel
    for (;;) {
        const int fu = __builtin_amdgcn_readfirstlane(f);
        if (f == fu) {
            if (frames[fu].nchunks == 0)
                assign_point(pts, i, frames[fu].box, frames[fu].cell_base, cell_of, slot, local,
                             cell_count, status);
            break;
        }
    }
}

// One chunk of one frame per workgroup: every point located, its slot inside
// the chunk taken from the chunk's per-cell counters in LDS (two 16-bit
// counters per word: a chunk holds at most kChunkPoints < 2^16 points, so a
// half never carries into the other), then the counters written to the
// chunk's row of `part`.
__global__ void __launch_bounds__(1024) assign_chunks_kernel(const float* pts,
                                                             const FrameInfo* __restrict__ frames,
                                                             const ChunkInfo* __restrict__ chunks,
                                                             int* cell_of, int* slot,
                                                             float4* local, int* part,
                                                             unsigned* status)
{
    extern __shared__ unsigned s_cnt[];
    const ChunkInfo C = chunks[blockIdx.x];
    const int words = (C.ncells + 1) >> 1;
    for (int w = threadIdx.x; w < words; w += blockDim.x) s_cnt[w] = 0u;
    __syncthreads();
    const AssignBox& B = frames[C.frame].box;
    for (int k = threadIdx.x; k < C.n; k += blockDim.x) {
        const int64_t i = (int64_t)C.first + k;
        const int j = locate_point(pts, i, B, C.cell_base, cell_of, local, status) - C.cell_base;
        const unsigned sh = (unsigned)(j & 1) << 4;
        const unsigned old = atomicAdd(&s_cnt[j >> 1], 1u << sh);
        slot[i] = (int)((old >> sh) & 0xffffu);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < C.ncells; j += blockDim.x)
        part[C.part + j] = (int)((s_cnt[j >> 1] >> ((unsigned)(j & 1) << 4)) & 0xffffu);
}

// Per chunk, after every chunk of the batch has counted: the chunk's first
// slot in each cell of its frame (the sum of the earlier chunks' counts
// there, in LDS), the frame's cell counts (by its last chunk), and each of
// its points' slot made final (first slot + slot inside the chunk).
__global__ void __launch_bounds__(1024) chunk_finish_kernel(const FrameInfo* __restrict__ frames,
                                                            const ChunkInfo* __restrict__ chunks,
                                                            const int* __restrict__ part,
                                                            const int* __restrict__ cell_of,
                                                            int* slot, int* cell_count)
{
    extern __shared__ int s_first[];
    const int k = blockIdx.x;
    const ChunkInfo C = chunks[k];
    const int k0 = frames[C.frame].chunk0;
    const bool last = k == k0 + frames[C.frame].nchunks - 1;
    // the earlier chunks' rows follow each other in `part` (ncells apart)
    const int* rows = part + chunks[k0].part;
    const int nrows = k - k0;
    for (int j = threadIdx.x; j < C.ncells; j += blockDim.x) {
        int b = 0;
        int q = 0;
        for (; q + 4 <= nrows; q += 4)  // four independent loads in flight
            b += rows[(size_t)q * C.ncells + j] + rows[(size_t)(q + 1) * C.ncells + j] +
                 rows[(size_t)(q + 2) * C.ncells + j] + rows[(size_t)(q + 3) * C.ncells + j];
        for (; q < nrows; ++q) b += rows[(size_t)q * C.ncells + j];
        s_first[j] = b;
        if (last) cell_count[C.cell_base + j] = b + part[C.part + j];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < C.n; t += blockDim.x) {
        const int64_t i = (int64_t)C.first + t;
        slot[i] += s_first[cell_of[i] - C.cell_base];
    }
}

// Place every point in its cell's run at the slot its atomic returned (the
// order inside a run is arrival order, not yet deterministic).
__global__ void __launch_bounds__(256) scatter_kernel(int64_t n, const int* __restrict__ cell_of,
                                                      const int* __restrict__ slot,
                                                      const float4* __restrict__ local,
                                                      const int* __restrict__ cell_start,
                                                      float4* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[cell_start[cell_of[i]] + slot[i]] = local[i];
}

// Order each cell's run by point index: every entry counts the entries of its
// run with a smaller index (its rank) and moves there.  The runs a
// workgroup's entries belong to are contiguous (the entries are sorted by
// cell), so their indices are staged in LDS once and every count reads LDS;
// runs spanning more than kRankSpan entries read global memory instead.  An
// entry's cell is found by binary search in the workgroup's slice of the
// cell starts, also staged in LDS, rather than read through the point's
// index (a read at a random place when the points are in random order:
// the 256-frame batch 175 -> 130 us); slices of more than kRankCells cells
// (long runs of empty cells) read it through the index.
constexpr int kRankSpan = 2048;
constexpr int kRankCells = 512;

__global__ void __launch_bounds__(256) rank_kernel(int64_t n, const int* __restrict__ cell_of,
                                                   const int* __restrict__ cell_start,
                                                   const float4* __restrict__ in,
                                                   float4* __restrict__ out)
{
    __shared__ int s_id[kRankSpan];
    __shared__ int s_cs[kRankCells + 1];
    __shared__ int s_c0, s_c1;
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t p = p0 + threadIdx.x;
    if (threadIdx.x == 0) {
        const int64_t last = p0 + blockDim.x - 1 < n ? p0 + blockDim.x - 1 : n - 1;
        s_c0 = cell_of[__float_as_int(in[p0].w)];
        s_c1 = cell_of[__float_as_int(in[last].w)];
    }
    __syncthreads();
    const int c0 = s_c0, c1 = s_c1;
    const bool cells_staged = c1 - c0 < kRankCells;
    if (cells_staged)
        for (int k = threadIdx.x; k <= c1 - c0 + 1; k += blockDim.x) s_cs[k] = cell_start[c0 + k];
    __syncthreads();
    const int lo = cells_staged ? s_cs[0] : cell_start[c0];
    const int hi = cells_staged ? s_cs[c1 - c0 + 1] : cell_start[c1 + 1];
    const bool staged = hi - lo <= kRankSpan;
    if (staged)
        for (int j = lo + (int)threadIdx.x; j < hi; j += blockDim.x)
            s_id[j - lo] = __float_as_int(in[j].w);
    __syncthreads();
    if (p >= n) return;
    const float4 v = in[p];
    const int id = __float_as_int(v.w);
    int b, e;
    if (cells_staged) {
        // the last cell of the slice starting at or before p holds it (empty
        // cells before it start at the same place)
        int k = 0;
        for (int step = kRankCells; step > 0; step >>= 1)
            if (k + step <= c1 - c0 && s_cs[k + step] <= p) k += step;
        b = s_cs[k];
        e = s_cs[k + 1];
    } else {
        const int c = cell_of[id];
        b = cell_start[c];
        e = cell_start[c + 1];
    }
    int r = 0;
    if (staged) {
        for (int j = b; j < e; ++j) r += s_id[j - lo] < id;
    } else {
        for (int j = b; j < e; ++j) r += __float_as_int(in[j].w) < id;
    }
    out[b + r] = v;
}

// ---------------------------------------------------------------------------
// Exclusive prefix scan, single pass with decoupled look-back.  Tiles take
// ids from a ticket counter in launch order, so a tile only ever waits on
// tiles that are already running or finished.  Each tile publishes its
// aggregate, then walks back over predecessors until it meets an inclusive
// prefix.  A status word packs the state in its top two bits (1 aggregate,
// 2 inclusive prefix) and the value in the low 62.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
// items per thread: 2 for short arrays (many tiles in flight), 4 from
// 131,072 items and 16 from 2^20 (tiles of 4096 and 16384 items per
// workgroup, read and written as 16-byte vectors; 2^20 items make 64 tiles
// of 16384, a look-back of one window).  Against 4 items per thread, 16
// took 2^20 row counts 15.0 -> 11.0 us and 1.1e7 (a 256-frame batch)
// 146 -> 87 us, but 2.4e5 cell counts (the k-NN grid) 5.5 -> 7.4 us: too
// few tiles to fill the CUs.
constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagInc = 2ull << 62;
constexpr unsigned long long kValueMask = (1ull << 62) - 1;

// Four consecutive outputs (16-byte aligned) in 16-byte stores.
__device__ __forceinline__ void store4(int* p, int a, int b, int c, int d)
{
    *reinterpret_cast<int4*>(p) = make_int4(a, b, c, d);
}
__device__ __forceinline__ void store4(int64_t* p, int64_t a, int64_t b, int64_t c, int64_t d)
{
    *reinterpret_cast<longlong2*>(p) = make_longlong2(a, b);
    *reinterpret_cast<longlong2*>(p + 2) = make_longlong2(c, d);
}

template <typename Out, int kScanItems>
__global__ void __launch_bounds__(kScanThreads) scan_kernel(const int* __restrict__ in,
                                                            Out* __restrict__ out, int64_t n,
                                                            unsigned long long* flags,
                                                            int* ticket,
                                                            unsigned long long* total_out)
{
    __shared__ long long s_warp[kScanThreads / kWave];
    __shared__ long long s_prefix;
    __shared__ int s_tile;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1);
    __syncthreads();
    const int64_t tile = s_tile;
    constexpr int kTile = kScanThreads * kScanItems;
    const int64_t base = tile * kTile + (int64_t)threadIdx.x * kScanItems;
    long long v[kScanItems];
    long long sum = 0;
    // whole, aligned groups of four items move as 16-byte vectors (the
    // lanes of a wavefront then read one contiguous run)
    constexpr bool kVec = kScanItems % 4 == 0;
    const bool vec = kVec && base + kScanItems <= n &&
                     ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if (vec) {
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) {
            const int4 q = *reinterpret_cast<const int4*>(&in[base + k]);
            v[k] = q.x;
            v[k + 1] = q.y;
            v[k + 2] = q.z;
            v[k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t i = base + k;
            v[k] = i < n ? (long long)in[i] : 0;
        }
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) sum += v[k];
    // block-wide exclusive scan of per-thread sums
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    long long incl = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        long long t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
    }
    if (lane == kWave - 1) s_warp[wv] = incl;
    __syncthreads();
    long long warp_before = 0, block_total = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wv) warp_before += s_warp[w];
        block_total += s_warp[w];
    }
    if (wv == 0) {
        // publish the aggregate, then look back 64 predecessors at a time
        if (lane == 0)
            __hip_atomic_store(&flags[tile],
                               (tile == 0 ? kFlagInc : kFlagAgg) | (unsigned long long)block_total,
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        long long prefix = 0;
        int64_t win = tile - 1;  // predecessor examined by lane 0
        while (win >= 0) {
            const int64_t j = win - lane;
            unsigned long long f = kFlagInc;  // before tile 0: an empty inclusive prefix
            if (j >= 0) {
                do {
                    f = __hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } while ((f >> 62) == 0);
            }
            const unsigned long long inc = __ballot((f >> 62) == 2);
            const int stop = __ffsll((long long)inc) - 1;  // nearest inclusive prefix, if any
            long long v = (long long)(f & kValueMask);
            if (stop >= 0 && lane > stop) v = 0;
            for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
            prefix += v;
            if (stop >= 0) break;
            win -= kWave;
        }
        if (lane == 0) {
            if (tile != 0)
                __hip_atomic_store(&flags[tile],
                                   kFlagInc | (unsigned long long)(prefix + block_total),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = prefix;
            const int64_t ntiles = n > 0 ? (n + kTile - 1) / kTile : 1;
            if (tile == ntiles - 1) {
                out[n] = (Out)(prefix + block_total);
                if (total_out) *total_out = (unsigned long long)(prefix + block_total);
            }
        }
    }
    __syncthreads();
    long long run = s_prefix + warp_before + (incl - sum);
    Out r[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        r[k] = (Out)run;
        run += v[k];
    }
    if (vec) {
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) store4(&out[base + k], r[k], r[k + 1], r[k + 2], r[k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < n) out[base + k] = r[k];
    }
}

}  // namespace

constexpr int kSmallItems = 2;
constexpr int kMidItems = 4;
constexpr int kLargeItems = 16;
constexpr int64_t kLargeFrom = 64LL * kScanThreads * kSmallItems;
constexpr int64_t kHugeFrom = 64LL * kScanThreads * kLargeItems;  // 2^20: 64 tiles of 16384

// Status words the scan of n items needs (one per tile of the small size).
size_t scan_flag_count(int64_t n)
{
    const int64_t tile = (int64_t)kScanThreads * kSmallItems;
    int64_t t = (n + tile - 1) / tile;
    return (size_t)(t < 1 ? 1 : t);
}

template <typename Out>
static void launch_scan(const int* in, Out* out, int64_t n, unsigned long long* flags, int* ticket,
                        unsigned long long* total, hipStream_t s)
{
    if (n < kLargeFrom) {
        const int64_t tile = (int64_t)kScanThreads * kSmallItems;
        const int64_t tiles = n > 0 ? (n + tile - 1) / tile : 1;
        hipLaunchKernelGGL((scan_kernel<Out, kSmallItems>), dim3((unsigned)tiles),
                           dim3(kScanThreads), 0, s, in, out, n, flags, ticket, total);
    } else if (n < kHugeFrom) {
        const int64_t tile = (int64_t)kScanThreads * kMidItems;
        const int64_t tiles = (n + tile - 1) / tile;
        hipLaunchKernelGGL((scan_kernel<Out, kMidItems>), dim3((unsigned)tiles),
                           dim3(kScanThreads), 0, s, in, out, n, flags, ticket, total);
    } else {
        const int64_t tile = (int64_t)kScanThreads * kLargeItems;
        const int64_t tiles = (n + tile - 1) / tile;
        hipLaunchKernelGGL((scan_kernel<Out, kLargeItems>), dim3((unsigned)tiles),
                           dim3(kScanThreads), 0, s, in, out, n, flags, ticket, total);
    }
}

void launch_scan_i64(const int* in, int64_t* out, int64_t n, unsigned long long* flags, int* ticket,
                     hipStream_t s)
{
    launch_scan<int64_t>(in, out, n, flags, ticket, nullptr, s);
}

void launch_scan_i64_total(const int* in, int64_t* out, int64_t n, unsigned long long* flags,
                           int* ticket, unsigned long long* total, hipStream_t s)
{
    launch_scan<int64_t>(in, out, n, flags, ticket, total, s);
}

void launch_zero(Workspace& ws, const Grid& g, bool separate_queries, void* extra,
                 size_t extra_bytes, hipStream_t s)
{
    ZeroRanges z{};
    auto add = [&](void* p, size_t bytes) {
        z.ptr[z.count] = (unsigned*)p;
        z.words[z.count] = (long long)((bytes + 3) / 4);
        ++z.count;
    };
    add(ws.status, 256);  // status word and counters share the header
    const size_t nf = scan_flag_count(g.ncells);
    add(ws.pts.cell_count, sizeof(int) * (size_t)g.ncells);
    add(ws.pts.scan_flags, sizeof(unsigned long long) * nf + 256);
    if (separate_queries) {
        add(ws.qry.cell_count, sizeof(int) * (size_t)g.ncells);
        add(ws.qry.scan_flags, sizeof(unsigned long long) * nf + 256);
    }
    if (ws.row_scan_flags)
        add(ws.row_scan_flags, sizeof(unsigned long long) * scan_flag_count(ws.qry.n) + 256);
    if (extra) add(extra, extra_bytes);
    hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(256), 0, s, z);
}

// Counting sort of the assigned points into their cells: scan of the cell
// counts, scatter in arrival order, then ranks by index within each cell.
static void finish_cells(CellList& cl, int ncells, hipStream_t s)
{
    const int64_t n = cl.n;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    launch_scan<int>(cl.cell_count, cl.cell_start, ncells, cl.scan_flags, cl.scan_ticket, nullptr,
                     s);
    if (n > 0) {
        // arrival order into `sorted`, then ranked by index back into `local`,
        // which from here on holds the final cell-sorted points
        hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(256), 0, s, n, cl.cell_of, cl.slot,
                           cl.local, cl.cell_start, cl.sorted);
        hipLaunchKernelGGL(rank_kernel, dim3(blocks), dim3(256), 0, s, n, cl.cell_of,
                           cl.cell_start, cl.sorted, cl.local);
    }
}

void launch_build_cells(const float* pts, CellList& cl, const BoxPrep& b, const Grid& g,
                        unsigned* status, hipStream_t s)
{
    AssignBox ab;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            ab.M[r][c] = b.M[r][c];
            ab.Minv[r][c] = b.Minv[r][c];
        }
    for (int k = 0; k < 3; ++k) {
        ab.n[k] = (double)g.n[k];
        ab.inv_n[k] = 1.0 / (double)g.n[k];
        ab.ni[k] = g.n[k];
    }
    ab.dim = b.dim;
    const int64_t n = cl.n;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (n > 0)
        hipLaunchKernelGGL(assign_kernel, dim3(blocks), dim3(256), 0, s, pts, n, ab, cl.cell_of,
                           cl.slot, cl.local, cl.cell_count, status);
    finish_cells(cl, g.ncells, s);
}

void launch_build_cells_batch(const float* pts, CellList& cl, const FrameInfo* frames,
                              const int* point_base, int nframes,
                              int ncells, const ChunkInfo* chunks, int nchunks, int max_chunk_cells,
                              int* part, bool global_frames, unsigned* status, hipStream_t s)
{
    const int64_t n = cl.n;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (n > 0 && global_frames)
        hipLaunchKernelGGL(assign_batch_kernel, dim3(blocks), dim3(256), 0, s, pts, n, frames,
                           point_base, nframes, cl.cell_of, cl.slot, cl.local, cl.cell_count,
                           status);
    if (nchunks > 0) {
        const size_t lds = sizeof(unsigned) * (size_t)((max_chunk_cells + 1) / 2);
        (void)hipFuncSetAttribute((const void*)assign_chunks_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(assign_chunks_kernel, dim3((unsigned)nchunks), dim3(1024), lds, s, pts,
                           frames, chunks, cl.cell_of, cl.slot, cl.local, part, status);
        const size_t lds2 = sizeof(int) * (size_t)max_chunk_cells;
        (void)hipFuncSetAttribute((const void*)chunk_finish_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
        hipLaunchKernelGGL(chunk_finish_kernel, dim3((unsigned)nchunks), dim3(1024), lds2, s,
                           frames, chunks, part, cl.cell_of, cl.slot, cl.cell_count);
    }
    launch_scan<int>(cl.cell_count, cl.cell_start, ncells, cl.scan_flags, cl.scan_ticket, nullptr,
                     s);
    if (n > 0) {
        hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(256), 0, s, n, cl.cell_of, cl.slot,
                           cl.local, cl.cell_start, cl.sorted);
        hipLaunchKernelGGL(rank_kernel, dim3(blocks), dim3(256), 0, s, n, cl.cell_of,
                           cl.cell_start, cl.sorted, cl.local);
    }
}

}  // namespace ppa
