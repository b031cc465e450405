// Internal declarations shared by the host code and the HIP kernels of libppa.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ppa.h"

namespace ppa {

constexpr int kWave = 64;
constexpr int kBlock = 256;             // threads per workgroup for the pair kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxSlots = 12;           // candidate slots a wave keeps in registers
constexpr int kCandCap = kMaxSlots * kWave;
constexpr int kMaxLdsBins = 4096;       // histograms up to this size live in LDS

// Device status bits (the status word in the workspace).
constexpr unsigned kStatusNonFinite = 1u;
constexpr unsigned kStatusCapacity = 2u;
constexpr unsigned kStatusRange = 4u;   // a k-nearest row reaches half the box width
constexpr unsigned kStatusBadList = 8u; // a NeighborList offset or index out of range
constexpr unsigned kStatusTies = 16u;   // too many list entries tie at the k-th distance

// Box prepared on the host in float64.
struct BoxPrep {
    double M[3][3];     // columns are the lattice vectors a1, a2, a3 (upper triangular)
    double Minv[3][3];  // inverse (upper triangular)
    double width[3];    // perpendicular widths d_k
    int dim;
};

// Uniform cell grid in fractional coordinates: cell c covers
// u in [c/n, (c+1)/n) per axis with u = s + 1/2 the fractional coordinate.
struct Grid {
    int n[3];
    int ncells;
    int nsten;          // 27 in 3D, 9 in 2D
    float off[27][3];   // M (delta / n) for each stencil offset, delta = (dx, dy, dz)
};

// Kernel view of the box for the cell assignment (float64).
struct AssignBox {
    double M[3][3];
    double Minv[3][3];
    double n[3];
    double inv_n[3];
    int ni[3];
    int dim;
};

// One cell list (points or query points) inside the workspace.
struct CellList {
    int* cell_of;        // [n]
    int* slot;           // [n] arrival slot inside the cell
    float4* local;       // [n] position relative to its cell centre, w = index bits;
                         //     after the build: sorted by cell, then by index
    float4* sorted;      // [n] scratch (arrival order inside each cell)
    int* cell_count;     // [ncells]  (zeroed, then counts)
    int* cell_start;     // [ncells + 1]
    unsigned long long* scan_flags;  // decoupled look-back state
    int* scan_ticket;
    int64_t n;
};

struct Workspace {
    unsigned* status;             // device status bits
    unsigned long long* counters; // [24] general counters (k-NN deferred count, batch queues)
    CellList pts;
    CellList qry;                 // == pts for self queries
    // canonical-row mode: int64 exclusive scan of row counts
    unsigned long long* row_scan_flags;
    int* row_scan_ticket;
    int* qry_row_counts;          // row counts when the caller passes none
    size_t bytes;
};

// One frame of a batch as the kernels see it (a table in the workspace).
struct FrameInfo {
    AssignBox box;         // float64 box and cell grid of the frame
    int cell_base;         // first global cell id of the frame
    int nsten;             // 27 in 3D, 9 in 2D
    int dot;               // expanded in/out test allowed for this frame's cells
    int point_base;        // first global point index of the frame
    int chunk0, nchunks;   // its chunks in the chunk table (nchunks 0: global counters)
    float off[27][4];      // stencil offsets M (delta / n), float32
};

// The batch cell build counts the points of a frame per cell in LDS, one
// workgroup per chunk of at most kChunkPoints consecutive points of one
// frame, instead of with global atomics (one per point, on cells in random
// order when the points are): each chunk writes its per-cell counts to its
// own row of a partial-count array; then each chunk sums the rows of the
// frame's earlier chunks into its first slot in every cell, and a point's
// slot in its cell is that plus its slot inside the chunk.  Frames with
// more than kChunkMaxCells cells (counted as 16-bit halves of 32-bit LDS
// words; the first slots take 4 bytes a cell of LDS) use the global
// counters.
struct ChunkInfo {
    int frame;
    int first;      // first point
    int n;          // points
    int cell_base;  // the frame's first cell
    int ncells;     // the frame's cells
    int part;       // first entry of this chunk's row in the partial-count array
};
constexpr int kChunkPoints = 16384;
constexpr int kChunkMaxCells = 32768;

// Per-workgroup partial arrays are summed in two stages; the first sums
// kPartialRowsPer of them at a time into one row of first-stage sums.
constexpr int kPartialRowsPer = 32;
inline int partial_rows(int G) { return (G + kPartialRowsPer - 1) / kPartialRowsPer; }

// Host helpers (api.hip).
int prepare_box(const ppa_box* box, BoxPrep* out);
int make_grid(const BoxPrep& b, double r_cut, int64_t n_hint, Grid* g);
size_t workspace_layout(const Grid& g, int64_t n, int64_t nq, int32_t flags, void* base,
                        Workspace* ws);
int set_error(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);

// Launchers (cells.hip).
void launch_zero(Workspace& ws, const Grid& g, bool separate_queries, void* extra,
                 size_t extra_bytes, hipStream_t s);
void launch_build_cells(const float* pts, CellList& cl, const BoxPrep& b, const Grid& g,
                        unsigned* status, hipStream_t s);
void launch_scan_i64(const int* in, int64_t* out, int64_t n, unsigned long long* flags,
                     int* ticket, hipStream_t s);
void launch_scan_i64_total(const int* in, int64_t* out, int64_t n, unsigned long long* flags,
                           int* ticket, unsigned long long* total, hipStream_t s);
size_t scan_flag_count(int64_t n);
// Batch: cells of every frame in one global list (cells.hip).
// chunks: the chunk table ([nchunks], device); part: the partial-count
// array its rows index; global_frames: whether any frame uses the global
// counters.
void launch_build_cells_batch(const float* pts, CellList& cl, const FrameInfo* frames,
                              const int* point_base, int nframes,
                              int ncells, const ChunkInfo* chunks, int nchunks, int max_chunk_cells,
                              int* part, bool global_frames, unsigned* status, hipStream_t s);
bool expanded_test_ok(const BoxPrep& bp, const Grid& g, double r);
int check_cutoff(const BoxPrep& bp, double r);

// Geometry of a pair query (pairs.hip).
struct PairGeom {
    int n[3];
    int ncells;
    int nsten;
    int center;          // stencil slot of the home cell itself
    float off[27][3];    // stencil offsets M (delta / n)
    float r2max;
    int dot;             // 1: expanded in/out test (its error bound passed on the host)
    int split;           // ball query: wavefronts sharing a home cell's queries (0, 1: one)
};

struct PairArgs {
    const float4* cand;      // points sorted by cell
    const int* cand_start;   // [ncells + 1]
    const float4* qsorted;   // query points sorted by cell
    const int* q_start;      // [ncells + 1]
    PairGeom geom;
    int32_t* counts;         // row lengths (count pass)
    const int64_t* offsets;  // CSR row pointer (fill pass)
    int32_t* point_idx;
    float* dist;
    int64_t capacity;
    unsigned* status;
    unsigned long long* hist;
    int bins;
    float r_min;
    float inv_dr;
};

// Batch pair kernels: frames[] and cell_base[nframes + 1] in device memory.
struct BatchGeom {
    const FrameInfo* frames;
    const int* cell_base;
    int nframes;
    int ncells;        // all frames
    float r2max;
    int run;           // home cells per work-queue item
    unsigned long long* queue;  // [16] zeroed counters: 8 per-XCD queues per pass
};
// waves: wavefronts per workgroup (2 or 4)
void launch_count_batch(const PairArgs& a, const BatchGeom& b, int dim, int excl, int blocks_cap,
                        int waves, hipStream_t s);
void launch_fill_batch(const PairArgs& a, const BatchGeom& b, int dim, int excl, int blocks_cap,
                       int waves, hipStream_t s);

// excl: 0 keep i == j, 1 points query themselves (drop the query's own
// entry), 2 separate query points (drop j == i by index).
// Compute units of the current device (queried once per device; 256 if the
// query fails).  Safe to call from several host threads.
int device_cus();

void launch_count(const PairArgs& a, int dim, int excl, hipStream_t s);
void launch_fill(const PairArgs& a, int dim, int excl, bool nl, bool hist, hipStream_t s);
// Orders every complete row of a CSR list by neighbour index (distances follow).
void launch_sort_rows(const int64_t* offsets, int64_t nq, int32_t* idx, float* dist,
                      int64_t capacity, hipStream_t s);

// k nearest neighbours (knn.hip).
struct KnnGeom {
    float minv[3][3];   // M^-1 in float32 (upper triangular)
    float nf[3];        // cells per axis
    float cellw[3];     // perpendicular cell widths d_k / n_k
    double M[3][3];     // lattice vectors, for the offsets of far shells
    float lim2;         // squared search limit: min(r_guard, half the smallest width)^2
    float t0;           // first threshold guess (r^2)
    int guard;          // 1: r_guard limits the rows (rows may be short)
    int excl;           // 1: drop the point whose index is the query's
    int k;
    int n_points;
    int smax;           // last shell of the far search (its radius passes the limit)
};

struct KnnArgs {
    const float4* cand;       // points sorted by cell
    const int* cand_start;    // [ncells + 1]
    const float4* qsorted;    // query points sorted by cell
    const int* q_start;       // [ncells + 1]
    const int* q_cell_of;     // [nq] home cell of each query (by query index)
    PairGeom geom;
    KnnGeom knn;
    int32_t* out_idx;         // rows at stride k
    float* out_dist;          // rows at stride k, or NULL
    int32_t* row_len;         // [nq] or NULL
    int* deferred;            // [nq] sorted positions of queries for the shell search
    unsigned long long* n_deferred;
    unsigned* status;
};

void launch_knn(const KnnArgs& a, int dim, hipStream_t s);
void launch_knn_offsets(int64_t* offsets, int64_t nq, int k, int64_t* n_pairs, hipStream_t s);
void launch_knn_pack(int64_t nq, int k, const int32_t* row_len, const int64_t* offsets,
                     const int32_t* st_idx, const float* st_dist, int32_t* point_idx, float* dist,
                     hipStream_t s);

// 2D PMFT (pmft.hip).  Bins of the histogram a bond shorter than r_max can
// reach, row by row: row ix keeps bins iy in [lo[ix], lo[ix] + base[ix+1] -
// base[ix]) at LDS words base[ix] onwards.
constexpr int kPmftMaxRows = 256;

struct PmftTable {
    int lo[kPmftMaxRows];
    int base[kPmftMaxRows + 1];
};

struct PmftArgs {
    const float4* cand;       // points sorted by cell
    const int* cand_start;    // [ncells + 1]
    const float4* qsorted;    // query points sorted by cell
    const int* q_start;       // [ncells + 1]
    const float* angles;      // [nq] orientation of each query point (radians)
    PairGeom geom;
    int excl;                 // 1: drop the point whose index is the query's
    int nbx, nby;
    float x_max, y_max;
    float inv_dx, inv_dy;     // bins per unit length
    int words;                // LDS words of the compacted histogram (0: global atomics)
    int entries;              // bins the compacted histogram holds
    int packed;               // 1: two 16-bit counters per LDS word
    unsigned* partial;        // [gridDim.x][entries] per-workgroup histograms
    unsigned* level2;         // [ceil(gridDim.x / 32)][entries] first-stage sums
    unsigned* counts;         // [nbx * nby] accumulated
    PmftTable table;
};

// Returns the number of workgroups launched (partials needed), or a negative
// PPA error when the launch failed.
int pmft_blocks_per_cu(int words, int packed);
int pmft_workgroups(int words, int packed);
size_t pmft_lds_limit();  // bytes of LDS a workgroup may give the histogram
void launch_pmft(const PmftArgs& a, int blocks, hipStream_t s);

// PMFT over three pair coordinates (pmft3.hip): XYT in 2D, XYZ in 3D.
constexpr int kPmftXyt = 0;
constexpr int kPmftXyz = 1;

struct Pmft3Args {
    const float4* cand;       // points sorted by cell
    const int* cand_start;    // [ncells + 1]
    const float4* qsorted;    // query points sorted by cell
    const int* q_start;       // [ncells + 1]
    const float* q_orient;    // XYT: [nq] angles; XYZ: [nq][4] quaternions (w, x, y, z)
    const float* p_orient;    // XYT: [n] angles of the points; XYZ: unused
    PairGeom geom;
    int mode;                 // kPmftXyt or kPmftXyz
    int excl;                 // 1: drop the point whose index is the query's
    int nb[3];                // bins per coordinate
    float max[3];             // x_max, y_max, z_max (unused for t)
    float inv_w[3];           // bins per unit of each coordinate
    unsigned* counts;         // [nb0 * nb1 * nb2] accumulated
    unsigned* status;         // workspace status word
};

void launch_pmft3(const Pmft3Args& a, hipStream_t s);

// Spatial correlation function of per-particle values (corr.hip).
constexpr int kCorrMaxBins = 4096;

struct CorrArgs {
    const float4* cand;       // points sorted by cell
    const int* cand_start;    // [ncells + 1]
    const float4* qsorted;    // query points sorted by cell
    const int* q_start;       // [ncells + 1]
    const float2* pval;       // [n] complex value of each point
    const float2* qval;       // [nq] complex value of each query point
    PairGeom geom;
    int excl;                 // 1: drop the point whose index is the query's
    int bins;
    float r_min;
    float inv_dr;             // bins / (r_max - r_min)
    double* psum;             // [blocks][2 bins] per-workgroup sums (re, im)
    unsigned long long* pcnt; // [blocks][bins] per-workgroup counts
    double* lsum;             // [rows][2 bins] first-stage sums
    unsigned long long* lcnt; // [rows][bins]
    double* sums;             // [bins][2] accumulated
    unsigned long long* counts;  // [bins] accumulated
    unsigned* status;
};

size_t corr_lds_bytes(int bins);
int corr_workgroups(int dim, int bins, long long ncells);
void launch_corr(const CorrArgs& a, int dim, int blocks, hipStream_t s);

// Steinhardt order parameters of NeighborList rows (steinhardt.hip).
constexpr int kSteinMaxL = 12;

struct SteinArgs {
    const float* pts;         // [n][3]
    const float* qpts;        // [nq][3] (pts when the points query themselves)
    const int64_t* offsets;   // [nq + 1]
    const int32_t* idx;       // [capacity]
    long long n, nq, capacity;
    int l;
    int dim;
    double m[3][3];           // box matrix (columns a1, a2, a3)
    double minv[3][3];
    const double* w3j;        // [(2l+1)^2] (l l l; m1 m2 -m1-m2), or NULL without W
    double* ql;               // [nq]
    double* wl;               // [nq] or NULL
    unsigned* status;
};

void launch_steinhardt_setup(int l, bool want_w, double* table, unsigned* status, hipStream_t s);
void launch_steinhardt(const SteinArgs& a, hipStream_t s);

// Clusters: connected components of NeighborList bonds (cluster.hip).
constexpr int kClusterRounds = 12;  // hooking rounds at most (flags in the header)

struct ClusterArgs {
    const int64_t* offsets;   // [n + 1]
    const int32_t* idx;       // [capacity]
    long long n, capacity;
    int* labels;              // [n] out: smallest index of the component
    int32_t* cluster_idx;     // [n] or NULL
    int32_t* sizes;           // [n] or NULL (first n_clusters entries used)
    int64_t* n_clusters;      // device or NULL
    unsigned* status;         // workspace header
    int* ticket;              // scan tile ticket (workspace header)
    int* round_flags;         // [kClusterRounds] changes per hooking round (header)
    int* giant;               // root of the sampled largest component (header)
    int symmetric;            // every bond is listed in both rows
    unsigned long long* scan_flags;
    int* is_root;             // [n]
    int64_t* rank;            // [n + 1]
    unsigned* zero;           // start of the region cleared per call
    size_t zero_bytes;
};

void launch_cluster(const ClusterArgs& a, hipStream_t s);

// k nearest selected from a stored NeighborList (knn_list.hip).
struct KnnListArgs {
    const int64_t* offsets;   // [nq + 1]
    const int32_t* idx;       // [capacity]
    const float* dist;        // [capacity]
    long long nq, capacity;
    int k;
    int32_t* row_len;         // [nq] out: min(k, row length)
    int32_t* out_idx;         // [nq * k] rows at stride k
    float* out_dist;          // [nq * k]
    unsigned* status;
};

int knn_list_workgroups(long long nq);
void launch_zero_words(unsigned* p, long long words, hipStream_t s);
void launch_knn_list(const KnnListArgs& a, int blocks, hipStream_t s);

// Gaussian-smoothed RDF and its adjoint (smooth.hip).
constexpr int kSmoothMaxBins = 4096;

struct SmoothArgs {
    const float4* cand;       // points sorted by cell (they are also the queries)
    const int* cand_start;    // [ncells + 1]
    PairGeom geom;            // r2max = (r_max + 8 sigma)^2 in float
    double offd[27][3];       // stencil offsets in float64
    int bins;
    double dr;                // r_max / bins
    double w8;                // window half-width 8 sigma
    float inv_dr;             // bins / r_max
    float k2;                 // log2(e) / (2 sigma^2)
    float step2;              // 2^(-2 k2 dr^2): ratio of consecutive bins' Gaussian factors
    float hscale;             // dr / (sigma sqrt(2 pi)): forward weight of exp(-u^2/2s^2)
    float gscale;             // dr / (sigma^3 sqrt(2 pi)): adjoint weight of u exp(-u^2/2s^2)
    int split;                // work units per home cell (its queries in parts)
    double* partial;          // forward: [gridDim.x][bins]
    double* level2;           // forward: [ceil(gridDim.x / 32)][bins] first-stage sums
    double* h;                // forward: [bins], accumulated
    const double* grad_h;     // adjoint: dL/dh [bins]
    float* grad;              // adjoint: dL/dp [n][3], written
};

int smooth_workgroups(bool adjoint, int dim, int bins);
void launch_smooth_fwd(const SmoothArgs& a, int dim, int blocks, hipStream_t s);
void launch_smooth_bwd(const SmoothArgs& a, int dim, int blocks, hipStream_t s);

void launch_hist_from_dist(const float* dist, const int64_t* n_pairs, int64_t capacity, int bins,
                           float r_min, float inv_dr, unsigned long long* hist, hipStream_t s);

}  // namespace ppa
