// Batched analysis of many frames (a trajectory, or many systems of uneven
// size each with its own box): the ball query NeighborList and a per-frame
// RDF for every frame in one sequence of launches over one global cell list.
// A plan fixes the frames and, per launch configuration, their cell grids;
// the frame tables are uploaded into the caller's workspace once, after
// which a run is a fixed sequence of kernels that can be captured in a HIP
// graph and replayed with one launch.  The pair kernels take their home
// cells from per-XCD work queues (runs of consecutive cells, handed out by
// atomic counters, with stealing across XCDs), so one launch of each pass
// covers every frame however uneven they are.  The autotuner times the
// configurations on the caller's data and keeps the fastest; they vary the
// cell width relative to r_max (at least r_max: the 27-cell stencil needs
// it), the block shape (wavefronts per workgroup and the home cells per
// queue item) and the resident workgroups per CU.  Configurations differ
// only in float32 rounding of the cell-local coordinates, so their lists and
// histograms agree except for pairs in the rounding band at r_max or at a
// bin edge.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "internal.hpp"

using namespace ppa;

namespace {

struct BatchConfig {
    double cell_scale;  // cell width >= cell_scale * r_max
    int blocks_cap;     // resident workgroups per CU of the pair kernels (0: all that fit)
    int run;            // home cells per work-queue item
    int waves;          // wavefronts per workgroup of the pair kernels (2 or 4)
};

const BatchConfig kConfigs[] = {
    {1.0, 0, 16, 4}, {1.0, 0, 4, 4},  {1.0, 0, 64, 4}, {1.0, 0, 16, 2},
    {1.0, 2, 16, 4}, {1.2, 0, 16, 4}, {1.2, 0, 16, 2}, {1.45, 0, 16, 4},
};
constexpr int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

struct ConfigTables {
    std::vector<FrameInfo> frames;
    std::vector<int> cell_base;  // [nframes + 1]
    std::vector<ChunkInfo> chunks;  // frames whose cells are counted in LDS, by chunks
    int ncells;
    int max_chunk_cells;   // cells of the largest chunked frame
    int64_t part_entries;  // entries of the partial-count array the chunks use
    bool global_frames;    // some frame counts with global atomics
    size_t frames_off, cell_base_off, chunks_off;  // workspace offsets of the device copies
};

// Splits the frames into chunks for the cell build: each frame with at most
// kChunkMaxCells cells gets ceil(points / kChunkPoints) chunks, each with a
// row of the frame's cells in the partial-count array.
// Upper bound on the partial-count array of the chunked cell build (entries,
// 4 bytes each); frames that would pass it count with global atomics instead.
constexpr int64_t kMaxPartEntries = int64_t(1) << 27;

void make_chunks(ConfigTables& T, const std::vector<int>& point_base, int nframes)
{
    T.chunks.clear();
    T.max_chunk_cells = 0;
    T.part_entries = 0;
    T.global_frames = false;
    for (int f = 0; f < nframes; ++f) {
        FrameInfo& F = T.frames[f];
        const int np = point_base[f + 1] - point_base[f];
        const int nc = T.cell_base[f + 1] - T.cell_base[f];
        const int k = (np + kChunkPoints - 1) / kChunkPoints;
        F.chunk0 = (int)T.chunks.size();
        F.nchunks = 0;
        if (np == 0) continue;
        if (nc > kChunkMaxCells || T.part_entries + (int64_t)k * nc > kMaxPartEntries) {
            T.global_frames = true;
            continue;
        }
        F.nchunks = k;
        for (int c = 0; c < k; ++c) {
            ChunkInfo C;
            C.frame = f;
            C.first = point_base[f] + c * kChunkPoints;
            C.n = np - c * kChunkPoints < kChunkPoints ? np - c * kChunkPoints : kChunkPoints;
            C.cell_base = T.cell_base[f];
            C.ncells = nc;
            C.part = (int)T.part_entries;
            T.chunks.push_back(C);
            T.part_entries += nc;
        }
        if (nc > T.max_chunk_cells) T.max_chunk_cells = nc;
    }
}

}  // namespace

struct ppa_batch_plan_s {
    int nframes;
    int dim;
    int bins;
    float r_min, r_max;
    int excl;
    int64_t n_total;
    bool sort_rows;               // PPA_SORT_ROWS: rows ordered by neighbour index
    std::vector<int> point_base;  // [nframes + 1]
    ConfigTables cfg[kNumConfigs];
    int chosen;
    size_t point_base_off;
    size_t part_off;          // partial-count array of the chunked cell build
    size_t scratch_hist_off;  // autotuning histograms
    size_t bytes;
    bool uploaded;
    void* uploaded_ws;
};

struct ppa_batch_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int max_cells(const ppa_batch_plan* p)
{
    int m = 0;
    for (int c = 0; c < kNumConfigs; ++c) m = p->cfg[c].ncells > m ? p->cfg[c].ncells : m;
    return m;
}

// Workspace: 256-byte header, the global cell list (sized for the largest
// grid of any configuration), row counts and their scan state, the frame
// tables of every configuration, the point bases, and scratch histograms.
void layout(const ppa_batch_plan* p, void* base, Workspace* W)
{
    Grid g{};
    g.ncells = max_cells(p);
    workspace_layout(g, p->n_total, 0, PPA_WS_NLIST, base, W);
}

int check_ws(const ppa_batch_plan* p, const void* ws, size_t ws_bytes)
{
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < p->bytes)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         p->bytes, ws_bytes);
    if (!p->uploaded || p->uploaded_ws != ws)
        return set_error(PPA_EINVAL, "the plan's tables are not in this workspace: call "
                                     "ppa_batch_upload first");
    return PPA_OK;
}

struct RunOut {
    uint64_t* hist;
    int64_t* offsets;
    int32_t* counts;
    int32_t* point_idx;
    float* dist;
    int64_t capacity;
    int64_t* n_pairs_dev;
};

void enqueue(const ppa_batch_plan* p, int ci, const float* pts, void* ws, const RunOut& o,
             hipStream_t s)
{
    char* base = (char*)ws;
    const ConfigTables& T = p->cfg[ci];
    Workspace W{};
    layout(p, ws, &W);
    // the cell list is carved for the largest grid of any configuration;
    // this one uses its first T.ncells cells (all of it is cleared, so the
    // scan state matches the carved layout)
    Grid g{};
    g.ncells = max_cells(p);
    launch_zero(W, g, false, nullptr, 0, s);
    const FrameInfo* frames = (const FrameInfo*)(base + T.frames_off);
    const int* cell_base = (const int*)(base + T.cell_base_off);
    const int* point_base = (const int*)(base + p->point_base_off);
    launch_build_cells_batch(pts, W.pts, frames, point_base, p->nframes, T.ncells,
                             (const ChunkInfo*)(base + T.chunks_off), (int)T.chunks.size(),
                             T.max_chunk_cells, (int*)(base + p->part_off), T.global_frames,
                             W.status, s);

    PairArgs A{};
    A.cand = W.pts.local;
    A.cand_start = W.pts.cell_start;
    A.qsorted = W.pts.local;
    A.q_start = W.pts.cell_start;
    A.counts = o.counts ? o.counts : W.qry_row_counts;
    A.offsets = o.offsets;
    A.point_idx = o.point_idx;
    A.dist = o.dist;
    A.capacity = o.capacity;
    A.status = W.status;
    A.hist = (unsigned long long*)o.hist;
    A.bins = p->bins;
    A.r_min = p->r_min;
    A.inv_dr = (float)((double)p->bins / ((double)p->r_max - (double)p->r_min));
    BatchGeom B;
    B.frames = frames;
    B.cell_base = cell_base;
    B.nframes = p->nframes;
    B.ncells = T.ncells;
    B.r2max = p->r_max * p->r_max;
    B.run = kConfigs[ci].run;
    B.queue = W.counters;  // in the header, cleared by launch_zero above
    const int cap = kConfigs[ci].blocks_cap;
    const int waves = kConfigs[ci].waves;
    launch_count_batch(A, B, p->dim, p->excl, cap, waves, s);
    launch_scan_i64_total(A.counts, o.offsets, p->n_total, W.row_scan_flags, W.row_scan_ticket,
                          (unsigned long long*)o.n_pairs_dev, s);
    launch_fill_batch(A, B, p->dim, p->excl, cap, waves, s);
    if (p->sort_rows)
        launch_sort_rows(o.offsets, p->n_total, o.point_idx, o.dist, o.capacity, s);
}

int check_out(const RunOut& o)
{
    if (!o.offsets || !o.n_pairs_dev || !o.hist || (!o.point_idx && o.capacity > 0))
        return set_error(PPA_EINVAL, "hist, offsets, point_idx and n_pairs_dev are required");
    if (o.capacity < 0) return set_error(PPA_EINVAL, "capacity must be >= 0");
    return PPA_OK;
}

}  // namespace

extern "C" {

int ppa_batch_plan_create(int32_t n_frames, const ppa_box* boxes, const int64_t* frame_offsets,
                          int32_t bins, float r_min, float r_max, int32_t exclude_ii,
                          int32_t flags, ppa_batch_plan** out)
{
    if (!out) return set_error(PPA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_frames < 1 || !boxes || !frame_offsets)
        return set_error(PPA_EINVAL, "need at least one frame, its box and offsets");
    if (flags & ~PPA_SORT_ROWS) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    if (bins < 1) return set_error(PPA_EINVAL, "bins must be >= 1");
    if (!(isfinite(r_max) && r_max > 0.f && isfinite(r_min) && r_min >= 0.f && r_min < r_max))
        return set_error(PPA_EINVAL, "need 0 <= r_min < r_max");
    if (frame_offsets[0] != 0) return set_error(PPA_EINVAL, "frame_offsets[0] must be 0");
    for (int f = 0; f < n_frames; ++f)
        if (frame_offsets[f + 1] < frame_offsets[f])
            return set_error(PPA_EINVAL, "frame_offsets must not decrease (frame %d)", f);
    if (frame_offsets[n_frames] > 0x7fffffffLL)
        return set_error(PPA_EINVAL, "at most 2^31 - 1 points in a batch");
    std::vector<BoxPrep> bp(n_frames);
    for (int f = 0; f < n_frames; ++f) {
        int rc = prepare_box(&boxes[f], &bp[f]);
        if (rc == PPA_OK && bp[f].dim != bp[0].dim)
            rc = set_error(PPA_EINVAL, "frames must share a dimension");
        if (rc == PPA_OK) rc = check_cutoff(bp[f], r_max);
        if (rc) {
            char msg[400];
            snprintf(msg, sizeof(msg), "%s", ppa_last_error());
            return set_error(rc, "frame %d: %s", f, msg);
        }
    }
    ppa_batch_plan* p = new ppa_batch_plan;
    p->nframes = n_frames;
    p->dim = bp[0].dim;
    p->bins = bins;
    p->r_min = r_min;
    p->r_max = r_max;
    p->excl = exclude_ii ? 1 : 0;
    p->n_total = frame_offsets[n_frames];
    p->sort_rows = (flags & PPA_SORT_ROWS) != 0;
    p->point_base.resize(n_frames + 1);
    for (int f = 0; f <= n_frames; ++f) p->point_base[f] = (int)frame_offsets[f];
    p->chosen = 0;
    p->uploaded = false;
    p->uploaded_ws = nullptr;
    for (int c = 0; c < kNumConfigs; ++c) {
        ConfigTables& T = p->cfg[c];
        T.frames.resize(n_frames);
        T.cell_base.resize(n_frames + 1);
        int64_t cells = 0;
        for (int f = 0; f < n_frames; ++f) {
            const int64_t nf = frame_offsets[f + 1] - frame_offsets[f];
            Grid g;
            make_grid(bp[f], kConfigs[c].cell_scale * r_max, nf, &g);
            FrameInfo& F = T.frames[f];
            memset(&F, 0, sizeof(F));
            for (int r = 0; r < 3; ++r)
                for (int k = 0; k < 3; ++k) {
                    F.box.M[r][k] = bp[f].M[r][k];
                    F.box.Minv[r][k] = bp[f].Minv[r][k];
                }
            for (int k = 0; k < 3; ++k) {
                F.box.n[k] = (double)g.n[k];
                F.box.inv_n[k] = 1.0 / (double)g.n[k];
                F.box.ni[k] = g.n[k];
            }
            F.box.dim = bp[f].dim;
            F.cell_base = (int)cells;
            F.nsten = g.nsten;
            F.dot = expanded_test_ok(bp[f], g, r_max) ? 1 : 0;
            F.point_base = (int)frame_offsets[f];
            for (int t = 0; t < 27; ++t) {
                F.off[t][0] = g.off[t][0];
                F.off[t][1] = g.off[t][1];
                F.off[t][2] = g.off[t][2];
                F.off[t][3] = 0.f;
            }
            T.cell_base[f] = (int)cells;
            cells += g.ncells;
        }
        if (cells > 0x7fffffffLL) {
            delete p;
            return set_error(PPA_EINVAL, "too many cells in the batch");
        }
        T.cell_base[n_frames] = (int)cells;
        T.ncells = (int)cells;
        make_chunks(T, p->point_base, n_frames);
    }
    Workspace W{};
    layout(p, nullptr, &W);
    size_t off = align256(W.bytes);
    for (int c = 0; c < kNumConfigs; ++c) {
        p->cfg[c].frames_off = off;
        off = align256(off + sizeof(FrameInfo) * (size_t)n_frames);
        p->cfg[c].cell_base_off = off;
        off = align256(off + sizeof(int) * (size_t)(n_frames + 1));
        p->cfg[c].chunks_off = off;
        off = align256(off + sizeof(ChunkInfo) * (p->cfg[c].chunks.size() + 1));
    }
    p->point_base_off = off;
    off = align256(off + sizeof(int) * (size_t)(n_frames + 1));
    int64_t part = 1;
    for (int c = 0; c < kNumConfigs; ++c)
        part = p->cfg[c].part_entries > part ? p->cfg[c].part_entries : part;
    p->part_off = off;
    off = align256(off + sizeof(int) * (size_t)part);
    p->scratch_hist_off = off;
    off = align256(off + sizeof(uint64_t) * (size_t)n_frames * (size_t)bins);
    p->bytes = off;
    *out = p;
    return PPA_OK;
}

int ppa_batch_plan_destroy(ppa_batch_plan* plan)
{
    delete plan;
    return PPA_OK;
}

int ppa_batch_workspace_bytes(const ppa_batch_plan* plan, size_t* bytes)
{
    if (!plan || !bytes) return set_error(PPA_EINVAL, "NULL argument");
    *bytes = plan->bytes;
    return PPA_OK;
}

int ppa_batch_upload(ppa_batch_plan* p, void* ws, size_t ws_bytes, hipStream_t s)
{
    if (!p) return set_error(PPA_EINVAL, "plan is NULL");
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < p->bytes)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         p->bytes, ws_bytes);
    char* base = (char*)ws;
    int rc;
    for (int c = 0; c < kNumConfigs; ++c) {
        const ConfigTables& T = p->cfg[c];
        if ((rc = hip_check(hipMemcpyAsync(base + T.frames_off, T.frames.data(),
                                           sizeof(FrameInfo) * T.frames.size(),
                                           hipMemcpyHostToDevice, s),
                            "upload frame table")))
            return rc;
        if ((rc = hip_check(hipMemcpyAsync(base + T.cell_base_off, T.cell_base.data(),
                                           sizeof(int) * T.cell_base.size(),
                                           hipMemcpyHostToDevice, s),
                            "upload cell bases")))
            return rc;
        if (!T.chunks.empty() &&
            (rc = hip_check(hipMemcpyAsync(base + T.chunks_off, T.chunks.data(),
                                           sizeof(ChunkInfo) * T.chunks.size(),
                                           hipMemcpyHostToDevice, s),
                            "upload chunk table")))
            return rc;
    }
    if ((rc = hip_check(hipMemcpyAsync(base + p->point_base_off, p->point_base.data(),
                                       sizeof(int) * p->point_base.size(), hipMemcpyHostToDevice,
                                       s),
                        "upload point bases")))
        return rc;
    // the copies read the plan's host tables, which live as long as the plan
    p->uploaded = true;
    p->uploaded_ws = ws;
    return PPA_OK;
}

int ppa_batch_run(ppa_batch_plan* p, const float* pts, void* ws, size_t ws_bytes, uint64_t* hist,
                  int64_t* offsets, int32_t* counts, int32_t* point_idx, float* dist,
                  int64_t capacity, int64_t* n_pairs_dev, hipStream_t s)
{
    if (!p) return set_error(PPA_EINVAL, "plan is NULL");
    if (!pts && p->n_total > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    const RunOut o{hist, offsets, counts, point_idx, dist, capacity, n_pairs_dev};
    if ((rc = check_out(o))) return rc;
    enqueue(p, p->chosen, pts, ws, o, s);
    return hip_check(hipGetLastError(), "kernel launch");
}

int ppa_batch_config(ppa_batch_plan* p, int32_t index, int32_t* n_configs, int32_t* chosen,
                     double* cell_scale, int32_t* blocks_per_cu)
{
    if (!p) return set_error(PPA_EINVAL, "plan is NULL");
    if (index >= kNumConfigs) return set_error(PPA_EINVAL, "no configuration %d", index);
    if (index >= 0) p->chosen = index;
    if (n_configs) *n_configs = kNumConfigs;
    if (chosen) *chosen = p->chosen;
    if (cell_scale) *cell_scale = kConfigs[p->chosen].cell_scale;
    if (blocks_per_cu) *blocks_per_cu = kConfigs[p->chosen].blocks_cap;
    return PPA_OK;
}

int ppa_batch_config_shape(ppa_batch_plan* p, int32_t index, int32_t* cells_per_item,
                           int32_t* waves_per_workgroup)
{
    if (!p) return set_error(PPA_EINVAL, "plan is NULL");
    if (index >= kNumConfigs) return set_error(PPA_EINVAL, "no configuration %d", index);
    const int c = index >= 0 ? index : p->chosen;
    if (cells_per_item) *cells_per_item = kConfigs[c].run;
    if (waves_per_workgroup) *waves_per_workgroup = kConfigs[c].waves;
    return PPA_OK;
}

int ppa_batch_config_cells(ppa_batch_plan* p, int32_t index, int32_t* cells, int32_t* chunks,
                           int32_t* global_frames)
{
    if (!p) return set_error(PPA_EINVAL, "plan is NULL");
    if (index >= kNumConfigs) return set_error(PPA_EINVAL, "no configuration %d", index);
    const ConfigTables& T = p->cfg[index >= 0 ? index : p->chosen];
    if (cells) *cells = T.ncells;
    if (chunks) *chunks = (int32_t)T.chunks.size();
    if (global_frames) {
        int g = 0;
        for (int f = 0; f < p->nframes; ++f)
            if (T.frames[f].nchunks == 0 && p->point_base[f + 1] > p->point_base[f]) ++g;
        *global_frames = g;
    }
    return PPA_OK;
}

int ppa_batch_autotune(ppa_batch_plan* p, const float* pts, void* ws, size_t ws_bytes,
                       int64_t* offsets, int32_t* counts, int32_t* point_idx, float* dist,
                       int64_t capacity, int64_t* n_pairs_dev, int32_t reps, hipStream_t s,
                       float* ms_out)
{
    if (!p) return set_error(PPA_EINVAL, "plan is NULL");
    if (!pts && p->n_total > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    if (reps < 1) return set_error(PPA_EINVAL, "reps must be >= 1");
    uint64_t* scratch = (uint64_t*)((char*)ws + p->scratch_hist_off);
    const RunOut o{scratch, offsets, counts, point_idx, dist, capacity, n_pairs_dev};
    if ((rc = check_out(o))) return rc;
    hipEvent_t e0, e1;
    if ((rc = hip_check(hipEventCreate(&e0), "event"))) return rc;
    if ((rc = hip_check(hipEventCreate(&e1), "event"))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    int best = p->chosen;
    float best_ms = INFINITY;
    for (int c = 0; c < kNumConfigs && rc == PPA_OK; ++c) {
        enqueue(p, c, pts, ws, o, s);  // warm-up (first use of this configuration's cells)
        float ms = 0.f;
        rc = hip_check(hipEventRecord(e0, s), "event record");
        for (int r = 0; r < reps && rc == PPA_OK; ++r) enqueue(p, c, pts, ws, o, s);
        if (rc == PPA_OK) rc = hip_check(hipEventRecord(e1, s), "event record");
        if (rc == PPA_OK) rc = hip_check(hipEventSynchronize(e1), "event synchronize");
        if (rc == PPA_OK) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
        if (rc == PPA_OK) {
            ms /= (float)reps;
            if (ms_out) ms_out[c] = ms;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    p->chosen = best;
    return hip_check(hipGetLastError(), "kernel launch");
}

int ppa_batch_graph_create(ppa_batch_plan* p, const float* pts, void* ws, size_t ws_bytes,
                           uint64_t* hist, int64_t* offsets, int32_t* counts, int32_t* point_idx,
                           float* dist, int64_t capacity, int64_t* n_pairs_dev,
                           ppa_batch_graph** out)
{
    if (!out) return set_error(PPA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return set_error(PPA_EINVAL, "plan is NULL");
    if (!pts && p->n_total > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    int rc = check_ws(p, ws, ws_bytes);
    if (rc) return rc;
    const RunOut o{hist, offsets, counts, point_idx, dist, capacity, n_pairs_dev};
    if ((rc = check_out(o))) return rc;
    hipStream_t cs;
    if ((rc = hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "stream"))) return rc;
    ppa_batch_graph* g = new ppa_batch_graph;
    g->graph = nullptr;
    g->exec = nullptr;
    rc = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    if (rc == PPA_OK) {
        enqueue(p, p->chosen, pts, ws, o, cs);
        const int launch_rc = hip_check(hipGetLastError(), "kernel launch");
        rc = hip_check(hipStreamEndCapture(cs, &g->graph), "end capture");
        if (rc == PPA_OK) rc = launch_rc;
    }
    if (rc == PPA_OK)
        rc = hip_check(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0),
                       "graph instantiate");
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return rc;
    }
    *out = g;
    return PPA_OK;
}

int ppa_batch_graph_launch(ppa_batch_graph* g, hipStream_t s)
{
    if (!g) return set_error(PPA_EINVAL, "graph is NULL");
    return hip_check(hipGraphLaunch(g->exec, s), "graph launch");
}

int ppa_batch_graph_destroy(ppa_batch_graph* g)
{
    if (!g) return PPA_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return PPA_OK;
}

}  // extern "C"
