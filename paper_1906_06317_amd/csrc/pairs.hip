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
//   * for a home cell, the 27 (2D: 9) stencil cells are gathered into NS
//     64-wide slots held in registers, each candidate shifted by its stencil
//     offset so it is relative to the home cell's centre; the code for each
//     slot count NS is unrolled separately, so the slot loop has no branches;
//   * the home cell's query points are prefetched 64 at a time into lanes
//     and read into scalar registers one by one; each is tested against
//     every slot with one ballot per slot.
// The in/out test of a candidate c against query q is either the plain
// |c - q|^2 < r_max^2 or, when the host has bounded its rounding error well
// inside the parity band, the expanded |c|^2 - 2 c.q < r_max^2 - |q|^2 (three
// FMAs).  The count pass keeps -2c and |c|^2 in its slots and reads each
// query, with its r_max^2 - |q|^2, from a per-wavefront LDS row by one
// broadcast load, so the tests take all operands from vector registers; two
// queries go at a time.  The fill pass keeps c and forms -2q per query; the
// products (-2c).q and c.(-2q) are equal and exact inside the FMA, so both
// passes evaluate the same value and agree pair by pair.  Every reported
// distance and bin is recomputed from the difference c - q.
// The NeighborList takes two passes so rows land in query order without
// atomics: count_kernel writes row lengths, a scan turns them into CSR
// offsets, and fill_kernel compacts hits with ballot + mbcnt into a small
// per-wavefront LDS list of whole rows, flushed densely: the distance, the
// histogram bin and coalesced stores for 64 hits per instruction.  Since the
// count pass fixed every row's length, the fill pass tests two queries
// against the same candidate registers at once and places the second row
// right after the first before either is found; the two independent chains
// interleave.  The RDF alone (no list) needs only the fill pass.  Stencils with more candidates
// than the register slots hold are processed in chunks, writing directly.
#include "pair_common.hpp"

namespace ppa {

namespace {

using namespace pair;

constexpr int kHitCap = 320;  // hits buffered per wavefront between flushes
constexpr int kRows = 64;     // rows buffered per wavefront
constexpr int kFillSlots = 10;  // register slots of the fill pass (it needs more registers)
static_assert(kFillSlots * kWave <= kCandCap, "a whole stencil fits the r^2 buffer");
constexpr int kMaxBatchLdsBins = 1024;  // per-wavefront histograms of a batch up to this size

// ---------------------------------------------------------------------------
// Pass 1: row lengths.
// ---------------------------------------------------------------------------
// Row lengths of the tile's queries, expanded test: candidates as -2c and
// |c|^2, each query's coordinates and r_max^2 - |q|^2 read from its lane
// (four readlanes), then three FMAs and a compare per slot.
template <int DIM, int EXCL, int NS>
__device__ __forceinline__ void count_tile_dot(const PairIn& in, const GeomView& G,
                                               const StencilLds& S, const float4* off, int C,
                                               int q0, int q1, int lane, float4* qrow,
                                               int32_t* __restrict__ counts)
{
    DotSlots<DIM, NS> c;
    c.load(in, G.nsten, S, off, 0, C, lane);
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        DotChunk Q;
        Q.template load<DIM>(in, c0, q1 - c0, lane, G.r2max, qrow);
        int cnt_v = 0;
        // two queries at a time: two independent test chains interleave
        int t = 0;
        for (; t + 1 < Q.n; t += 2) {
            const DQuery qa = Q.get(t);
            const DQuery qb = Q.get(t + 1);
            int na = 0, nb = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                bool ha = c.hit(s, qa.x, qa.y, qa.z, qa.thr);
                bool hb = c.hit(s, qb.x, qb.y, qb.z, qb.thr);
                if (EXCL == 2) {
                    ha = ha && c.id[s] != qa.id;
                    hb = hb && c.id[s] != qb.id;
                }
                na += __popcll(__ballot(ha));
                nb += __popcll(__ballot(hb));
            }
            // a point querying itself always finds its own entry, at r = 0
            if (EXCL == 1) {
                na -= 1;
                nb -= 1;
            }
            cnt_v = with_lane(cnt_v, t, na);
            cnt_v = with_lane(cnt_v, t + 1, nb);
        }
        if (t < Q.n) {
            const DQuery q = Q.get(t);
            int n = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                bool h = c.hit(s, q.x, q.y, q.z, q.thr);
                if (EXCL == 2) h = h && c.id[s] != q.id;
                n += __popcll(__ballot(h));
            }
            if (EXCL == 1) n -= 1;
            cnt_v = with_lane(cnt_v, t, n);
        }
        if (lane < Q.n) counts[Q.my_id()] = cnt_v;
    }
}

// The same with the plain test |c - q|^2 < r_max^2 (when the host could not
// bound the expanded test's rounding inside the parity band).
template <int DIM, int EXCL, int NS>
__device__ __forceinline__ void count_tile_plain(const PairIn& in, const GeomView& G,
                                                 const StencilLds& S, const float4* off, int C,
                                                 int q0, int q1, int lane,
                                                 int32_t* __restrict__ counts)
{
    Slots<DIM, NS> c;
    c.load(in, G.nsten, S, off, 0, C, lane);
    const float r2max = G.r2max;
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        QueryChunk Q;
        Q.load(in, c0, q1 - c0, lane);
        int cnt_v = 0;
        for (int t = 0; t < Q.n; ++t) {
            const Query q = Q.get<DIM>(t, r2max);
            int n = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                bool h = c.template hit<false>(s, q, r2max);
                if (EXCL == 2) h = h && c.id[s] != q.id;
                n += __popcll(__ballot(h));
            }
            if (EXCL == 1) n -= 1;
            cnt_v = with_lane(cnt_v, t, n);
        }
        if (lane < Q.n) counts[Q.my_id()] = cnt_v;
    }
}

// Stencils too large for the register slots: candidate chunks of
// kChunkSlots slots, each loaded once per 64 queries.
template <int DIM, int EXCL>
__device__ __forceinline__ void count_chunked(const PairIn& in, const GeomView& G,
                                              const StencilLds& S, const float4* off, int C,
                                              int q0, int q1, int lane,
                                              int32_t* __restrict__ counts)
{
    const float r2max = G.r2max;
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        QueryChunk Q;
        Q.load(in, c0, q1 - c0, lane);
        int cnt_v = EXCL == 1 ? -1 : 0;
        for (int k0 = 0; k0 < C; k0 += kChunkSlots * kWave) {
            Slots<DIM, kChunkSlots> c;
            c.load(in, G.nsten, S, off, k0, C, lane);
            for (int t = 0; t < Q.n; ++t) {
                const Query q = Q.get<DIM>(t, r2max);
                int n = 0;
#pragma unroll
                for (int s = 0; s < kChunkSlots; ++s) {
                    bool h = G.dot ? c.template hit<true>(s, q, r2max)
                                   : c.template hit<false>(s, q, r2max);
                    if (EXCL == 2) h = h && c.id[s] != q.id;
                    n += __popcll(__ballot(h));
                }
                cnt_v += lane == t ? n : 0;
            }
        }
        if (lane < Q.n) counts[Q.my_id()] = cnt_v;
    }
}

// Row lengths of one home cell: the slot count picks the unrolled code.
template <int DIM, int EXCL>
__device__ __forceinline__ void count_cell(const PairIn& in, const GeomView& V,
                                           const StencilLds& S, const float4* off, int C, int q0,
                                           int q1, int lane, float4* qrow,
                                           int32_t* __restrict__ counts)
{
    const int ns = (C + kWave - 1) / kWave;
    if (V.dot) {
        switch (ns) {
#define PPA_CASE(N) \
    case N: count_tile_dot<DIM, EXCL, N>(in, V, S, off, C, q0, q1, lane, qrow, counts); return;
            PPA_CASE(0) PPA_CASE(1) PPA_CASE(2) PPA_CASE(3) PPA_CASE(4) PPA_CASE(5) PPA_CASE(6)
            PPA_CASE(7) PPA_CASE(8) PPA_CASE(9) PPA_CASE(10) PPA_CASE(11) PPA_CASE(12)
#undef PPA_CASE
        default: break;
        }
    } else {
        switch (ns) {
#define PPA_CASE(N) \
    case N: count_tile_plain<DIM, EXCL, N>(in, V, S, off, C, q0, q1, lane, counts); return;
            PPA_CASE(0) PPA_CASE(1) PPA_CASE(2) PPA_CASE(3) PPA_CASE(4) PPA_CASE(5) PPA_CASE(6)
            PPA_CASE(7) PPA_CASE(8) PPA_CASE(9) PPA_CASE(10) PPA_CASE(11) PPA_CASE(12)
#undef PPA_CASE
        default: break;
        }
    }
    count_chunked<DIM, EXCL>(in, V, S, off, C, q0, q1, lane, counts);
}

template <int DIM, int EXCL>
__global__ void __launch_bounds__(kBlock, 6) count_kernel(const PairIn in, const PairGeom G,
                                                       int32_t* __restrict__ counts)
{
    __shared__ float4 s_off[27];
    __shared__ StencilLds s_st[kWavesPerBlock];
    __shared__ float4 s_q[kWavesPerBlock][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    StencilLds& S = s_st[wv];
    if (threadIdx.x < 27)
        s_off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1],
                                         G.off[threadIdx.x][2], 0.f);
    __syncthreads();
    const GeomView V = view_of(G);
    const int split = G.split > 1 ? G.split : 1;
    int t0, t1, stride;
    wave_tiles_interleaved<kWavesPerBlock>(G.ncells * split, wv, t0, t1, stride);
    for (int v = t0; v < t1; v += stride) {
        const CellPart P = cell_part(in, v, split);
        if (P.q0 == P.q1) continue;
        const int C = stencil<DIM>(in, V, P.tile, lane, S);
        count_cell<DIM, EXCL>(in, V, S, s_off, C, P.q0, P.q1, lane, s_q[wv], counts);
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

// Per-wavefront LDS of the fill pass.  With a list, a hit keeps the
// candidate's coordinates (its exact distance is recomputed at the flush)
// and rows are whole; for the histogram alone, a hit keeps only its exact
// r^2 from the difference form.
template <bool NL>
struct FillLds;

template <>
struct FillLds<true> {
    float4 hit[kHitCap];               // candidate xyz relative to the home centre, index bits
    float4 rq[kRows];                  // each non-empty row's query xyz, index bits
    long long base[kRows];             // offsets[q] - first buffered hit of the row
    unsigned long long starts[kHitCap / 64];  // bit e: a non-empty row starts at hit e
    StencilLds st;
};

template <>
struct FillLds<false> {
    float r2[kCandCap];
    StencilLds st;
};

// Per-wavefront state of the fill pass.
template <int DIM, int EXCL, bool NL, bool HIST>
struct Filler {
    FillLds<NL>& W;
    const FillOut O;
    unsigned* hist_lds;  // NULL: bin straight into ghist
    unsigned long long* ghist;  // the histogram in global memory (the frame's, in a batch)
    int id_base;  // subtracted from point indices written to the list (frame-local indices)
    int lane;
    int nh;     // hits buffered
    int nrows;  // rows buffered
    int selfs;  // own entries binned by the histogram-only path (all at r = 0)
    bool over;

    __device__ Filler(FillLds<NL>& w, const FillOut& o, unsigned* h, int l)
        : W(w), O(o), hist_lds(h), ghist(o.hist), id_base(0), lane(l), nh(0), nrows(0), selfs(0),
          over(false)
    {
    }

    __device__ __forceinline__ void bin_at(float t)
    {
        const int b = min((int)t, O.bins - 1);
        if (hist_lds)
            atomicAdd(&hist_lds[b], 1u);
        else
            atomicAdd(&ghist[b], 1ull);
    }
    __device__ __forceinline__ void bin(float r)
    {
        if (O.r_min == 0.f) {
            // r >= 0, and r - 0 is r: the same t without the subtraction or
            // the lower test
            const float t = r * O.inv_dr;
            if (t < (float)O.bins) bin_at(t);
        } else {
            const float t = (r - O.r_min) * O.inv_dr;
            if (t >= 0.f && t < (float)O.bins) bin_at(t);
        }
    }
    __device__ __forceinline__ void emit(long long dst, int id, float r)
    {
        if (dst < O.capacity) {
            // the list is written once and read by a later kernel: stream it
            // past the caches, which keep the stencil cells
            __builtin_nontemporal_store(id - id_base, &O.point_idx[dst]);
            if (O.dist) __builtin_nontemporal_store(r, &O.dist[dst]);
        } else {
            over = true;
        }
    }
    // Records a buffered row starting at position rs: query t of the chunk
    // (its lane holds the point and its row offset rb_v) writes the record
    // and the row's start bit.
    __device__ __forceinline__ void add_row(const QueryChunk& Q, long long rb_v, int t, int rs)
    {
        if constexpr (NL) {
            if (lane == t) {
                W.rq[nrows] = Q.q;
                W.base[nrows] = rb_v - rs;
                // the two rows of a pair may share a word: different lanes
                atomicOr(&W.starts[rs >> 6], 1ull << (rs & 63));
            }
            ++nrows;
        }
    }
    // Emits every buffered hit: exact distance, list store and histogram bin.
    // The row of hit e is the number of row starts at or before e, minus one.
    __device__ __forceinline__ void flush()
    {
        wave_sync();
        if constexpr (NL) {
            int before = 0;  // row starts in earlier 64-hit blocks
            for (int e0 = 0; e0 < nh; e0 += kWave) {
                const unsigned long long bm = uniform64(W.starts[e0 >> 6]);
                const int e = e0 + lane;
                // starts at hits e0 .. e: those at bits 1 .. lane counted by
                // the mbcnt of bm >> 1, plus bit 0
                const int r = lane_slot(bm >> 1, before + (int)(bm & 1ull) - 1);
                before += __popcll(bm);
                if (e < nh) {
                    // the three reads depend only on e and r: issue them together
                    const float4 h = W.hit[e];
                    const float4 q = W.rq[r];
                    const long long b = W.base[r];
                    // keep the index with the rest of the record's read (one
                    // 16-byte read, not a second one in the store branch)
                    int id = __float_as_int(h.w);
                    asm volatile("" : "+v"(id));
                    const float d = fast_sqrt(dist2<DIM>(h.x - q.x, h.y - q.y, h.z - q.z));
                    emit(b + e, id, d);
                    if (HIST) bin(d);
                }
            }
            if (lane < kHitCap / 64) W.starts[lane] = 0ull;
        } else {
            for (int e = lane; e < nh; e += kWave) bin(fast_sqrt(W.r2[e]));
        }
        nh = 0;
        nrows = 0;
        wave_sync();
    }

    // Buffers the hits of query q against NS slots.  For a point querying
    // itself, its own entry is lane `self` of slot 0 (the home cell comes
    // first in the stencil and lists its points in query order); BY_ID drops
    // the entry with the query's index instead (separate query points, or a
    // home cell too full for the lane rule).
    template <int NS, bool DOT, bool BY_ID>
    __device__ __forceinline__ void buffer_hits(const Slots<DIM, NS>& c, const Query& q,
                                                float r2max, int self)
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if constexpr (NL) {
                bool h = c.template hit<DOT>(s, q, r2max);
                if (BY_ID) h = h && c.id[s] != q.id;
                if (!BY_ID && EXCL == 1 && s == 0) h = h && lane != self;
                const unsigned long long m = __ballot(h);
                if (h) {
                    float4* dst = &W.hit[nh];
                    dst[lane_prefix(m)] =
                        make_float4(c.x[s], c.y[s], c.z[s], __int_as_float(c.id[s]));
                }
                nh += __popcll(m);
            } else {
                const float r2 = dist2<DIM>(c.x[s] - q.x, c.y[s] - q.y, c.z[s] - q.z);
                bool h = r2 < r2max;
                if (EXCL == 2) h = h && c.id[s] != q.id;
                const unsigned long long m = __ballot(h);
                if (h) W.r2[nh + (int)lane_prefix(m)] = r2;
                nh += __popcll(m);
            }
        }
        // the histogram-only path keeps a point's own entry (r = 0) and
        // removes it from bin 0 at the end
        if (!NL && EXCL == 1) ++selfs;
    }
    // Buffers the hits of two queries at once: a's row (its length known
    // from the count pass) at wa, b's at wb, right after it.  The two in/out
    // chains share the candidate registers and are independent, so their
    // instructions interleave.
    template <int NS, bool DOT, bool BY_ID>
    __device__ __forceinline__ void buffer_pair(const Slots<DIM, NS>& c, const Query& qa,
                                                const Query& qb, float r2max, int self_a,
                                                int self_b, int wa, int wb)
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            bool ha = c.template hit<DOT>(s, qa, r2max);
            bool hb = c.template hit<DOT>(s, qb, r2max);
            if (BY_ID) {
                ha = ha && c.id[s] != qa.id;
                hb = hb && c.id[s] != qb.id;
            }
            if (!BY_ID && EXCL == 1 && s == 0) {
                ha = ha && lane != self_a;
                hb = hb && lane != self_b;
            }
            const unsigned long long ma = __ballot(ha);
            const unsigned long long mb = __ballot(hb);
            const float4 v = make_float4(c.x[s], c.y[s], c.z[s], __int_as_float(c.id[s]));
            if (ha) W.hit[wa + (int)lane_prefix(ma)] = v;
            if (hb) W.hit[wb + (int)lane_prefix(mb)] = v;
            wa += __popcll(ma);
            wb += __popcll(mb);
        }
    }
    // Writes the hits of query q against NS slots straight to the outputs,
    // at rbase + w onwards.
    template <int NS, bool DOT>
    __device__ __forceinline__ void direct_hits(const Slots<DIM, NS>& c, const Query& q,
                                                float r2max, long long rbase, int& w)
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            bool h = c.template hit<DOT>(s, q, r2max);
            if (EXCL != 0) h = h && c.id[s] != q.id;
            const unsigned long long m = __ballot(h);
            if (h) {
                const float d = fast_sqrt(dist2<DIM>(c.x[s] - q.x, c.y[s] - q.y, c.z[s] - q.z));
                if (NL) emit(rbase + w + (int)lane_prefix(m), c.id[s], d);
                if (HIST) bin(d);
            }
            w += __popcll(m);
        }
    }
};

// Queries [q0, q1) of the home cell whose first query is qc.
template <int DIM, int EXCL, bool NL, bool HIST, int NS>
__device__ __forceinline__ void fill_tile(const PairIn& in, const GeomView& G, const StencilLds& S,
                                          const float4* off, int C, int qc, int q0, int q1,
                                          Filler<DIM, EXCL, NL, HIST>& F)
{
    const int lane = F.lane;
    Slots<DIM, NS> c;
    c.load(in, G.nsten, S, off, 0, C, lane);
    const float r2max = G.r2max;
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        QueryChunk Q;
        Q.load(in, c0, q1 - c0, lane);
        long long rb_v = 0;
        int rl_v = 0;
        if (NL && lane < Q.n) {
            rb_v = F.O.offsets[Q.my_id()];
            rl_v = (int)(F.O.offsets[Q.my_id() + 1] - rb_v);
        }
        for (int t = 0; t < Q.n; ++t) {
            // position of the query's own entry in slot 0 (home cell first)
            const int self = (c0 - qc) + t < kWave ? (c0 - qc) + t : -1;
            if constexpr (NL) {
                const int need = lane_of(rl_v, t);  // the row, from the count pass
                if (need > kHitCap) {
                    int w = 0;
                    const long long rbase = lane_of64(rb_v, t);
                    if (G.dot)
                        F.template direct_hits<NS, true>(c, Q.get<DIM>(t, r2max), r2max, rbase, w);
                    else
                        F.template direct_hits<NS, false>(c, Q.get<DIM>(t, r2max), r2max, rbase, w);
                    continue;
                }
                // two rows at once when both fit the buffer
                const int need_b = t + 1 < Q.n ? lane_of(rl_v, t + 1) : kHitCap + 1;
                if (need + need_b <= kHitCap) {
                    if (F.nh + need + need_b > kHitCap || F.nrows + 2 > kRows) F.flush();
                    const int rsa = F.nh;
                    const int rsb = rsa + need;
                    const int self_b = (c0 - qc) + t + 1 < kWave ? (c0 - qc) + t + 1 : -1;
                    const bool by_id = EXCL == 2 || (EXCL == 1 && self_b < 0);
                    const Query qa = Q.get<DIM>(t, r2max);
                    const Query qb = Q.get<DIM>(t + 1, r2max);
                    if (G.dot) {
                        if (by_id)
                            F.template buffer_pair<NS, true, true>(c, qa, qb, r2max, self, self_b,
                                                                   rsa, rsb);
                        else
                            F.template buffer_pair<NS, true, false>(c, qa, qb, r2max, self, self_b,
                                                                    rsa, rsb);
                    } else {
                        if (by_id)
                            F.template buffer_pair<NS, false, true>(c, qa, qb, r2max, self,
                                                                    self_b, rsa, rsb);
                        else
                            F.template buffer_pair<NS, false, false>(c, qa, qb, r2max, self,
                                                                     self_b, rsa, rsb);
                    }
                    if (need > 0) F.add_row(Q, rb_v, t, rsa);
                    if (need_b > 0) F.add_row(Q, rb_v, t + 1, rsb);
                    F.nh = rsb + need_b;
                    ++t;
                    continue;
                }
                if (F.nh + need > kHitCap || F.nrows == kRows) F.flush();
            } else {
                // the histogram alone: at most every candidate
                if (F.nh + C > kCandCap) F.flush();
            }
            const int rs = F.nh;
            const bool by_id = EXCL == 2 || (EXCL == 1 && self < 0);
            const Query q = Q.get<DIM>(t, r2max);
            if (NL && G.dot) {
                if (by_id)
                    F.template buffer_hits<NS, true, true>(c, q, r2max, self);
                else
                    F.template buffer_hits<NS, true, false>(c, q, r2max, self);
            } else {
                if (by_id)
                    F.template buffer_hits<NS, false, true>(c, q, r2max, self);
                else
                    F.template buffer_hits<NS, false, false>(c, q, r2max, self);
            }
            if (NL && F.nh > rs) F.add_row(Q, rb_v, t, rs);
        }
    }
}

template <int DIM, int EXCL, bool NL, bool HIST>
__device__ __forceinline__ void fill_chunked(const PairIn& in, const GeomView& G,
                                             const StencilLds& S, const float4* off, int C,
                                             int q0, int q1, Filler<DIM, EXCL, NL, HIST>& F)
{
    const int lane = F.lane;
    const float r2max = G.r2max;
    for (int c0 = q0; c0 < q1; c0 += kWave) {
        QueryChunk Q;
        Q.load(in, c0, q1 - c0, lane);
        long long rb_v = 0;
        if (NL && lane < Q.n) rb_v = F.O.offsets[Q.my_id()];
        int w_v = 0;  // entries written so far, per query
        for (int k0 = 0; k0 < C; k0 += kChunkSlots * kWave) {
            Slots<DIM, kChunkSlots> c;
            c.load(in, G.nsten, S, off, k0, C, lane);
            for (int t = 0; t < Q.n; ++t) {
                const Query q = Q.get<DIM>(t, r2max);
                const long long rbase = NL ? lane_of64(rb_v, t) : 0;
                int w = lane_of(w_v, t);
                if (G.dot)
                    F.template direct_hits<kChunkSlots, true>(c, q, r2max, rbase, w);
                else
                    F.template direct_hits<kChunkSlots, false>(c, q, r2max, rbase, w);
                w_v = lane == t ? w : w_v;
            }
        }
    }
}

template <int DIM, int EXCL, bool NL, bool HIST>
__global__ void __launch_bounds__(kBlock, 5) fill_kernel(const PairIn in, const PairGeom G,
                                                      const FillOut O)
{
    extern __shared__ unsigned s_hist[];
    __shared__ float4 s_off[27];
    __shared__ FillLds<NL> s_w[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    StencilLds& S = s_w[wv].st;
    const bool lds_hist = HIST && O.bins <= kMaxLdsBins;
    if (threadIdx.x < 27)
        s_off[threadIdx.x] = make_float4(G.off[threadIdx.x][0], G.off[threadIdx.x][1],
                                         G.off[threadIdx.x][2], 0.f);
    if (lds_hist)
        for (int b = threadIdx.x; b < O.bins; b += kBlock) s_hist[b] = 0u;
    __syncthreads();

    if constexpr (NL) {
        if (lane < kHitCap / 64) s_w[wv].starts[lane] = 0ull;
        wave_sync();
    }
    Filler<DIM, EXCL, NL, HIST> F(s_w[wv], O, lds_hist ? s_hist : nullptr, lane);
    const GeomView V = view_of(G);
    const int split = G.split > 1 ? G.split : 1;
    int t0, t1, stride;
    wave_tiles_interleaved<kWavesPerBlock>(G.ncells * split, wv, t0, t1, stride);
    for (int v = t0; v < t1; v += stride) {
        const CellPart P = cell_part(in, v, split);
        if (P.q0 == P.q1) continue;
        const int C = stencil<DIM>(in, V, P.tile, lane, S);
        const int ns = (C + kWave - 1) / kWave;
        switch (ns) {
#define PPA_CASE(N)                                                                        \
    case N: fill_tile<DIM, EXCL, NL, HIST, N>(in, V, S, s_off, C, P.qc, P.q0, P.q1, F); \
        break;
            PPA_CASE(0) PPA_CASE(1) PPA_CASE(2) PPA_CASE(3) PPA_CASE(4) PPA_CASE(5) PPA_CASE(6)
            PPA_CASE(7) PPA_CASE(8) PPA_CASE(9) PPA_CASE(10)
#undef PPA_CASE
            static_assert(kFillSlots == 10, "the cases above cover 0..kFillSlots");
        default: fill_chunked<DIM, EXCL, NL, HIST>(in, V, S, s_off, C, P.q0, P.q1, F);
        }
    }
    if (F.nh > 0) F.flush();
    if (NL && __ballot(F.over) && lane == 0) atomicOr(O.status, kStatusCapacity);
    if (!NL && EXCL == 1 && F.selfs > 0 && O.r_min <= 0.f && lane == 0) {
        if (lds_hist)
            atomicSub(&s_hist[0], (unsigned)F.selfs);
        else
            atomicAdd(&O.hist[0], (unsigned long long)(-(long long)F.selfs));
    }

    __syncthreads();
    if (lds_hist)
        for (int b = threadIdx.x; b < O.bins; b += kBlock) {
            const unsigned v = s_hist[b];
            if (v) atomicAdd(&O.hist[b], (unsigned long long)v);
        }
}

// ---------------------------------------------------------------------------
// Batch: the same passes over the cells of many frames at once.  The home
// cells of all frames form one global range, cut into runs of B.run
// consecutive cells; a wavefront switches geometry (grid, stencil offsets,
// frame-local point indices, the frame's histogram) when a run takes it into
// another frame.
// ---------------------------------------------------------------------------
// Work queues of a batch pass.  The cells of XCD x (workgroups are
// dispatched round-robin over the 8 XCDs) are [x C / 8, (x + 1) C / 8); its
// runs are handed out in order by an atomic counter (queue[x]), so the runs
// in flight on an XCD are neighbours sharing stencil cells in its L2, and a
// wavefront that finds its own XCD's queue empty takes runs from the other
// XCDs' queues in turn, so uneven frames (cheap and dear cells) finish
// together.  Every wavefront ends when all eight queues are empty.
struct RunQueue {
    int x;       // XCD whose queue is being drained
    int visited; // queues tried so far
    int c0, c1;  // that XCD's cells
    int nruns;

    __device__ __forceinline__ void set(const BatchGeom& B, int xcd)
    {
        x = xcd;
        c0 = (int)((long long)x * B.ncells / 8);
        c1 = (int)((long long)(x + 1) * B.ncells / 8);
        nruns = (c1 - c0 + B.run - 1) / B.run;
    }
    // The next run [t, te) for this wavefront; false when every queue is empty.
    __device__ __forceinline__ bool next(const BatchGeom& B, unsigned long long* queue, int lane,
                                         int& t, int& te)
    {
        for (;;) {
            unsigned long long k = 0;
            if (lane == 0) k = atomicAdd(&queue[x], 1ull);
            const int kk = uniform((int)(k < (unsigned long long)nruns ? k : nruns));
            if (kk < nruns) {
                t = c0 + kk * B.run;
                te = min(t + B.run, c1);
                return true;
            }
            if (++visited == 8) return false;
            set(B, (x + 1) & 7);
        }
    }
};

// Frame of global cell `tile`: the last f with cell_base[f] <= tile.
__device__ __forceinline__ int frame_of(const BatchGeom& B, int tile)
{
    int lo = 0, hi = B.nframes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.cell_base[mid] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return uniform(lo);
}

// Loads frame f's geometry: the view in scalar registers, the stencil
// offsets into this wavefront's LDS.
__device__ __forceinline__ GeomView load_frame(const BatchGeom& B, int f, float4* off, int lane)
{
    const FrameInfo& F = B.frames[f];
    GeomView v;
    v.n0 = uniform(F.box.ni[0]);
    v.n1 = uniform(F.box.ni[1]);
    v.n2 = uniform(F.box.ni[2]);
    v.nsten = uniform(F.nsten);
    v.cell_base = uniform(F.cell_base);
    v.r2max = B.r2max;
    v.dot = uniform(F.dot);
    if (lane < 27) off[lane] = make_float4(F.off[lane][0], F.off[lane][1], F.off[lane][2], 0.f);
    wave_sync();
    return v;
}

// Row lengths of a batch; WPB wavefronts per workgroup.
template <int DIM, int EXCL, int WPB>
__global__ void __launch_bounds__(WPB * kWave, 5) count_batch_kernel(
    const PairIn in, const BatchGeom B, int32_t* __restrict__ counts)
{
    __shared__ float4 s_off[WPB][27];
    __shared__ StencilLds s_st[WPB];
    __shared__ float4 s_q[WPB][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    StencilLds& S = s_st[wv];
    float4* off = s_off[wv];
    RunQueue R;
    R.visited = 0;
    R.set(B, blockIdx.x & 7);
    int f = -1, cur = 0, next = -1;
    GeomView V;
    int t, te;
    while (R.next(B, B.queue, lane, t, te)) {
        for (int tile = t; tile < te; ++tile) {
            if (tile < cur || tile >= next) {
                f = frame_of(B, tile);
                V = load_frame(B, f, off, lane);
                cur = B.cell_base[f];
                next = B.cell_base[f + 1];
            }
            const int q0 = in.q_start[tile];
            const int q1 = in.q_start[tile + 1];
            if (q0 == q1) continue;
            const int C = stencil<DIM>(in, V, tile, lane, S);
            count_cell<DIM, EXCL>(in, V, S, off, C, q0, q1, lane, s_q[wv], counts);
        }
    }
}

// Adds this wavefront's LDS histogram into the global one and clears it.
__device__ __forceinline__ void merge_wave_hist(unsigned* h, unsigned long long* g, int bins,
                                                int lane)
{
    wave_sync();
    for (int b = lane; b < bins; b += kWave) {
        const unsigned v = h[b];
        if (v) {
            atomicAdd(&g[b], (unsigned long long)v);
            h[b] = 0u;
        }
    }
    wave_sync();
}

// NeighborList and per-frame RDF (histograms [nframes][bins]) of a batch;
// WPB wavefronts per workgroup.
template <int DIM, int EXCL, int WPB>
__global__ void __launch_bounds__(WPB * kWave, 5) fill_batch_kernel(
    const PairIn in, const BatchGeom B, const FillOut O)
{
    extern __shared__ unsigned s_dyn[];  // one histogram per wavefront when bins are few
    __shared__ float4 s_off[WPB][27];
    __shared__ FillLds<true> s_w[WPB];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = uniform(threadIdx.x / kWave);
    StencilLds& S = s_w[wv].st;
    float4* off = s_off[wv];
    const bool lds_hist = O.bins <= kMaxBatchLdsBins;
    unsigned* h = lds_hist ? s_dyn + (size_t)wv * O.bins : nullptr;
    if (lds_hist)
        for (int b = lane; b < O.bins; b += kWave) h[b] = 0u;
    if (lane < kHitCap / 64) s_w[wv].starts[lane] = 0ull;
    wave_sync();
    Filler<DIM, EXCL, true, true> F(s_w[wv], O, h, lane);
    RunQueue R;
    R.visited = 0;
    R.set(B, blockIdx.x & 7);
    int f = -1, cur = 0, next = -1;
    GeomView V;
    int t, te;
    while (R.next(B, B.queue + 8, lane, t, te)) {
        for (int tile = t; tile < te; ++tile) {
            if (tile < cur || tile >= next) {
                // buffered hits belong to the old frame: write them and its bins first
                if (F.nh > 0) F.flush();
                if (lds_hist && f >= 0) merge_wave_hist(h, F.ghist, O.bins, lane);
                f = frame_of(B, tile);
                V = load_frame(B, f, off, lane);
                F.ghist = O.hist + (size_t)f * O.bins;
                F.id_base = uniform(B.frames[f].point_base);
                cur = B.cell_base[f];
                next = B.cell_base[f + 1];
            }
            const int q0 = in.q_start[tile];
            const int q1 = in.q_start[tile + 1];
            if (q0 == q1) continue;
            const int C = stencil<DIM>(in, V, tile, lane, S);
            const int ns = (C + kWave - 1) / kWave;
            switch (ns) {
#define PPA_CASE(N) \
    case N: fill_tile<DIM, EXCL, true, true, N>(in, V, S, off, C, q0, q0, q1, F); break;
                PPA_CASE(0) PPA_CASE(1) PPA_CASE(2) PPA_CASE(3) PPA_CASE(4) PPA_CASE(5)
                PPA_CASE(6) PPA_CASE(7) PPA_CASE(8) PPA_CASE(9) PPA_CASE(10)
#undef PPA_CASE
            default: fill_chunked<DIM, EXCL, true, true>(in, V, S, off, C, q0, q1, F);
            }
        }
    }
    if (F.nh > 0) F.flush();
    if (lds_hist && f >= 0) merge_wave_hist(h, F.ghist, O.bins, lane);
    if (__ballot(F.over) && lane == 0) atomicOr(O.status, kStatusCapacity);
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
        if (t >= 0.f && t < (float)bins) {
            const int b = min((int)t, bins - 1);
            if (lds_hist)
                atomicAdd(&s_hist[b], 1u);
            else
                atomicAdd(&hist[b], 1ull);
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
void launch_count_t(const PairIn& in, const PairGeom& g, int32_t* counts, hipStream_t s)
{
    auto k = count_kernel<DIM, EXCL>;
    const int blocks = resident_blocks(k, 0, (long long)g.ncells * (g.split > 1 ? g.split : 1));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(kBlock), 0, s, in, g, counts);
}

template <int DIM, int EXCL>
void launch_fill_t(const PairIn& in, const PairGeom& g, const FillOut& o, bool nl, bool hist,
                   hipStream_t s)
{
    const size_t lds = (hist && o.bins <= kMaxLdsBins) ? sizeof(unsigned) * (size_t)o.bins : 0;
    auto k = nl ? (hist ? fill_kernel<DIM, EXCL, true, true> : fill_kernel<DIM, EXCL, true, false>)
                : fill_kernel<DIM, EXCL, false, true>;
    const int blocks = resident_blocks(k, lds, (long long)g.ncells * (g.split > 1 ? g.split : 1));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(kBlock), lds, s, in, g, o);
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

void launch_count(const PairArgs& a, int dim, int excl, hipStream_t s)
{
    const PairIn in = make_in(a);
#define PPA_COUNT(D, E) launch_count_t<D, E>(in, a.geom, a.counts, s)
    if (dim == 3) {
        if (excl == 1) PPA_COUNT(3, 1); else if (excl == 2) PPA_COUNT(3, 2); else PPA_COUNT(3, 0);
    } else {
        if (excl == 1) PPA_COUNT(2, 1); else if (excl == 2) PPA_COUNT(2, 2); else PPA_COUNT(2, 0);
    }
#undef PPA_COUNT
}

// Workgroups for a batch pass: as many as fit at once (times the cap per CU
// when one is set), a multiple of 8; the queues hand out the work.
template <typename K>
static int batch_blocks(K kernel, int threads, size_t lds, int blocks_cap)
{
    const int cus = device_cus();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (blocks_cap > 0 && per_cu > blocks_cap) per_cu = blocks_cap;
    return (cus * per_cu + 7) / 8 * 8;
}

template <int DIM, int EXCL, int WPB>
static void count_batch_t(const PairIn& in, const BatchGeom& b, int32_t* counts, int blocks_cap,
                          hipStream_t s)
{
    auto k = count_batch_kernel<DIM, EXCL, WPB>;
    const int blocks = batch_blocks(k, WPB * kWave, 0, blocks_cap);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(WPB * kWave), 0, s, in, b, counts);
}

template <int DIM, int EXCL, int WPB>
static void fill_batch_t(const PairIn& in, const BatchGeom& b, const FillOut& o, int blocks_cap,
                         hipStream_t s)
{
    const size_t lds =
        o.bins <= kMaxBatchLdsBins ? sizeof(unsigned) * (size_t)o.bins * WPB : 0;
    auto k = fill_batch_kernel<DIM, EXCL, WPB>;
    const int blocks = batch_blocks(k, WPB * kWave, lds, blocks_cap);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(WPB * kWave), lds, s, in, b, o);
}

void launch_count_batch(const PairArgs& a, const BatchGeom& b, int dim, int excl, int blocks_cap,
                        int waves, hipStream_t s)
{
    const PairIn in = make_in(a);
#define PPA_CB(D, E)                                                         \
    do {                                                                     \
        if (waves == 2) count_batch_t<D, E, 2>(in, b, a.counts, blocks_cap, s); \
        else count_batch_t<D, E, 4>(in, b, a.counts, blocks_cap, s);        \
    } while (0)
    if (dim == 3) {
        if (excl) PPA_CB(3, 1); else PPA_CB(3, 0);
    } else {
        if (excl) PPA_CB(2, 1); else PPA_CB(2, 0);
    }
#undef PPA_CB
}

void launch_fill_batch(const PairArgs& a, const BatchGeom& b, int dim, int excl, int blocks_cap,
                       int waves, hipStream_t s)
{
    const PairIn in = make_in(a);
    FillOut o;
    o.offsets = a.offsets;
    o.point_idx = a.point_idx;
    o.dist = a.dist;
    o.capacity = a.capacity;
    o.status = a.status;
    o.hist = a.hist;
    o.bins = a.bins;
    o.r_min = a.r_min;
    o.inv_dr = a.inv_dr;
#define PPA_FB(D, E)                                                 \
    do {                                                             \
        if (waves == 2) fill_batch_t<D, E, 2>(in, b, o, blocks_cap, s); \
        else fill_batch_t<D, E, 4>(in, b, o, blocks_cap, s);        \
    } while (0)
    if (dim == 3) {
        if (excl) PPA_FB(3, 1); else PPA_FB(3, 0);
    } else {
        if (excl) PPA_FB(2, 1); else PPA_FB(2, 0);
    }
#undef PPA_FB
}

void launch_fill(const PairArgs& a, int dim, int excl, bool nl, bool hist, hipStream_t s)
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
#define PPA_FILL(D, E) launch_fill_t<D, E>(in, a.geom, o, nl, hist, s)
    if (dim == 3) {
        if (excl == 1) PPA_FILL(3, 1); else if (excl == 2) PPA_FILL(3, 2); else PPA_FILL(3, 0);
    } else {
        if (excl == 1) PPA_FILL(2, 1); else if (excl == 2) PPA_FILL(2, 2); else PPA_FILL(2, 0);
    }
#undef PPA_FILL
}

void launch_hist_from_dist(const float* dist, const int64_t* n_pairs, int64_t capacity, int bins,
                           float r_min, float inv_dr, unsigned long long* hist, hipStream_t s)
{
    const size_t lds = bins <= kMaxLdsBins ? sizeof(unsigned) * (size_t)bins : 0;
    hipLaunchKernelGGL(hist_from_dist_kernel, dim3(1024), dim3(256), lds, s, dist, n_pairs,
                       capacity, bins, r_min, inv_dr, hist);
}

}  // namespace ppa
