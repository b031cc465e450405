// C ABI of libppa: argument checks, box preparation in float64, workspace
// layout and the sequence of kernel launches for each entry point.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "internal.hpp"

namespace ppa {

static thread_local char g_err[512] = "";
struct ProfileEvents {
    hipEvent_t ev[4];
};
static thread_local ProfileEvents g_prof = {{nullptr, nullptr, nullptr, nullptr}};

// One-shot profiling events: before/after the count pass, before/after the
// fill pass of the next query call.
static ProfileEvents take_profile_events()
{
    ProfileEvents p = g_prof;
    g_prof = ProfileEvents{{nullptr, nullptr, nullptr, nullptr}};
    return p;
}

static void record(hipEvent_t e, hipStream_t s)
{
    if (e) (void)hipEventRecord(e, s);
}

int set_error(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_check(hipError_t e, const char* what)
{
    if (e == hipSuccess) return PPA_OK;
    return set_error(PPA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Box matrix M with columns a1 = (Lx,0,0), a2 = (xy Ly, Ly, 0),
// a3 = (xz Lz, yz Lz, Lz); its inverse; and the perpendicular widths
// d_k = 1 / |row k of M^-1| (the distance between opposite faces).
int prepare_box(const ppa_box* box, BoxPrep* out)
{
    if (!box) return set_error(PPA_EINVAL, "box is NULL");
    if (box->dim != 2 && box->dim != 3) return set_error(PPA_EINVAL, "dim must be 2 or 3");
    const int dim = box->dim;
    for (int k = 0; k < dim; ++k)
        if (!(isfinite(box->L[k]) && box->L[k] > 0.0))
            return set_error(PPA_EBOX, "box length L[%d] must be finite and positive", k);
    for (int k = 0; k < 3; ++k)
        if (!isfinite(box->tilt[k])) return set_error(PPA_EBOX, "tilt[%d] is not finite", k);
    const double Lx = box->L[0], Ly = box->L[1], Lz = dim == 3 ? box->L[2] : 1.0;
    const double xy = box->tilt[0], xz = dim == 3 ? box->tilt[1] : 0.0,
                 yz = dim == 3 ? box->tilt[2] : 0.0;
    double(*M)[3] = out->M;
    double(*I)[3] = out->Minv;
    memset(out, 0, sizeof(*out));
    M[0][0] = Lx; M[0][1] = xy * Ly; M[0][2] = xz * Lz;
    M[1][1] = Ly; M[1][2] = yz * Lz;
    M[2][2] = Lz;
    I[0][0] = 1.0 / Lx; I[0][1] = -xy / Lx; I[0][2] = (xy * yz - xz) / Lx;
    I[1][1] = 1.0 / Ly; I[1][2] = -yz / Ly;
    I[2][2] = 1.0 / Lz;
    for (int k = 0; k < 3; ++k) {
        const double r = sqrt(I[k][0] * I[k][0] + I[k][1] * I[k][1] + I[k][2] * I[k][2]);
        out->width[k] = 1.0 / r;
    }
    if (dim == 2) out->width[2] = INFINITY;
    out->dim = dim;
    return PPA_OK;
}

// Cells of width >= r_cut (1 + 1e-5) per axis, so a pair closer than r_cut is
// always in the 27-cell (9-cell) stencil even when rounding puts a point on
// the wrong side of a cell face.  The count is capped near the number of
// points: larger cells are always valid, only slower.
int make_grid(const BoxPrep& b, double r_cut, int64_t n_hint, Grid* g)
{
    const int dim = b.dim;
    double nk[3] = {1, 1, 1};
    for (int k = 0; k < dim; ++k) {
        double v = floor(b.width[k] / (r_cut * (1.0 + 1e-5)));
        nk[k] = v < 1.0 ? 1.0 : v;
    }
    const double cap = fmax(64.0, 2.0 * (double)n_hint);
    double total = nk[0] * nk[1] * nk[2];
    if (total > cap) {
        const double f = pow(cap / total, 1.0 / dim);
        for (int k = 0; k < dim; ++k) nk[k] = fmax(1.0, floor(nk[k] * f));
    }
    for (int k = 0; k < 3; ++k) g->n[k] = (int)nk[k];
    g->ncells = g->n[0] * g->n[1] * g->n[2];
    g->nsten = dim == 3 ? 27 : 9;
    // slot 0 is the home cell: it swaps places with offset code 0
    const int centre = g->nsten / 2;
    for (int s = 0; s < 27; ++s) {
        const int code = s == 0 ? centre : (s == centre ? 0 : s);
        double d[3] = {(double)(code % 3 - 1), (double)((code / 3) % 3 - 1),
                       dim == 3 ? (double)(code / 9 - 1) : 0.0};
        if (s >= g->nsten) d[0] = d[1] = d[2] = 0.0;
        double f[3] = {d[0] / g->n[0], d[1] / g->n[1], d[2] / g->n[2]};
        g->off[s][0] = (float)(b.M[0][0] * f[0] + b.M[0][1] * f[1] + b.M[0][2] * f[2]);
        g->off[s][1] = (float)(b.M[1][1] * f[1] + b.M[1][2] * f[2]);
        g->off[s][2] = dim == 3 ? (float)(b.M[2][2] * f[2]) : 0.f;
    }
    return PPA_OK;
}

// Grid of the ball query and PMFT: cells of width >= r_cut, widened (by at
// most 2x per axis) while they would hold fewer than kPairTargetPpc points on
// average.  One wavefront works on one home cell, so very sparse cells leave
// most lanes idle; wider cells give each wavefront more queries and more
// candidates per stencil walk.
constexpr double kPairTargetPpc = 6.0;

static void pair_grid(const BoxPrep& b, double r_cut, int64_t n, Grid* g)
{
    make_grid(b, r_cut, n, g);
    if (n <= 0) return;
    const double ppc = (double)n / g->ncells;
    if (ppc >= kPairTargetPpc) return;
    const double s = fmin(2.0, pow(kPairTargetPpc / ppc, 1.0 / b.dim));
    make_grid(b, r_cut * s, n, g);
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

static void carve_cells(char* base, size_t& off, const Grid& g, int64_t n, CellList* cl)
{
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    cl->n = n;
    cl->cell_of = (int*)take(sizeof(int) * (size_t)n);
    cl->slot = (int*)take(sizeof(int) * (size_t)n);
    cl->local = (float4*)take(sizeof(float4) * (size_t)n);
    cl->sorted = (float4*)take(sizeof(float4) * (size_t)n);
    cl->cell_count = (int*)take(sizeof(int) * (size_t)g.ncells);
    cl->cell_start = (int*)take(sizeof(int) * ((size_t)g.ncells + 1));
    const size_t nf = scan_flag_count(g.ncells);
    cl->scan_flags = (unsigned long long*)take(sizeof(unsigned long long) * nf + 256);
    cl->scan_ticket = cl->scan_flags ? (int*)(cl->scan_flags + nf) : nullptr;
}

// Workspace: 256-byte header (status word, counters), the points' cell list,
// the query points' cell list when they differ, and for query-ordered rows a
// row-count array plus the scan state for the row offsets.
size_t workspace_layout(const Grid& g, int64_t n, int64_t nq, int32_t flags, void* base_v,
                        Workspace* ws)
{
    char* base = (char*)base_v;
    size_t off = 0;
    ws->status = base ? (unsigned*)base : nullptr;
    ws->counters = base ? (unsigned long long*)(base + 64) : nullptr;
    off = 256;
    carve_cells(base, off, g, n, &ws->pts);
    if (nq > 0) {
        carve_cells(base, off, g, nq, &ws->qry);
    } else {
        ws->qry = ws->pts;
    }
    ws->row_scan_flags = nullptr;
    ws->row_scan_ticket = nullptr;
    ws->qry_row_counts = nullptr;
    const int64_t nrow = nq > 0 ? nq : n;
    if (flags & PPA_WS_NLIST) {  // row counts and the scan state of the row offsets
        const size_t nf = scan_flag_count(nrow);
        void* rc = base ? base + off : nullptr;
        off = align_up(off + sizeof(int) * (size_t)nrow);
        ws->row_scan_flags = base ? (unsigned long long*)(base + off) : nullptr;
        ws->row_scan_ticket = base ? (int*)(ws->row_scan_flags + nf) : nullptr;
        off = align_up(off + sizeof(unsigned long long) * nf + 256);
        ws->qry_row_counts = (int*)rc;
    }
    ws->bytes = off;
    return off;
}

int check_cutoff(const BoxPrep& bp, double r)
{
    const double half = 0.5 * fmin(bp.width[0], fmin(bp.width[1], bp.width[2]));
    if (!(r < half))
        return set_error(PPA_ERANGE,
                         "cutoff %.9g must be below half the smallest perpendicular box width "
                         "(%.9g)",
                         r, half);
    return PPA_OK;
}

// Whether the expanded in/out test |c|^2 - 2 c.q < r^2 - |q|^2 is accurate
// enough in float32: its worst-case rounding error, for a query anywhere in
// its cell (|q| <= the cell's centre-to-corner distance) and a candidate
// near the cutoff (|c| <= |q| + r), must stay below half the parity band
// (1e-5 r^2) so that every pair outside the band is decided exactly.
bool expanded_test_ok(const BoxPrep& bp, const Grid& g, double r)
{
    double qmax = 0.0;
    for (int sx = -1; sx <= 1; sx += 2)
        for (int sy = -1; sy <= 1; sy += 2)
            for (int sz = -1; sz <= 1; sz += 2) {
                const double f[3] = {0.5 * sx / g.n[0], 0.5 * sy / g.n[1],
                                     bp.dim == 3 ? 0.5 * sz / g.n[2] : 0.0};
                const double x = bp.M[0][0] * f[0] + bp.M[0][1] * f[1] + bp.M[0][2] * f[2];
                const double y = bp.M[1][1] * f[1] + bp.M[1][2] * f[2];
                const double z = bp.M[2][2] * f[2];
                qmax = fmax(qmax, sqrt(x * x + y * y + z * z));
            }
    const double cmax = qmax + r;
    const double u = ldexp(1.0, -24);  // unit roundoff of float32
    const double err = u * (3 * cmax * cmax + 3 * (cmax * cmax + 2 * cmax * qmax) +
                            3 * qmax * qmax + (r * r + qmax * qmax));
    return err <= 0.5e-5 * r * r;
}

int device_cus()
{
    constexpr int kMaxDevices = 64;
    static std::atomic<int> cache[kMaxDevices];  // 0: not queried yet
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
    if (dev >= kMaxDevices) {
        hipDeviceProp_t prop;
        return hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.multiProcessorCount : 256;
    }
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        hipDeviceProp_t prop;
        v = hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0
                ? prop.multiProcessorCount
                : 256;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Wavefronts sharing each home cell's queries in the ball query's passes.
// One wavefront per cell leaves most of the chip idle when there are few
// cells (a small system, or a cutoff that is large against the box): then
// each cell's queries are split between several wavefronts, each loading
// the cell's stencil, up to about 8192 wavefronts in all and down to about
// four queries per wavefront.
int pair_split(long long ncells, long long nq)
{
    constexpr long long kTargetWaves = 8192;
    if (ncells <= 0 || ncells >= kTargetWaves) return 1;
    long long s = kTargetWaves / ncells;
    const long long by_queries = nq / ncells / 4;
    if (s > by_queries) s = by_queries;
    if (s > 16) s = 16;
    return s < 1 ? 1 : (int)s;
}

}  // namespace ppa

using namespace ppa;

namespace {

struct QueryCall {
    const ppa_box* box;
    const float* pts;
    int64_t n;
    const float* qpts;
    int64_t nq;
    float r_max;
    int32_t exclude_ii;
    int32_t flags;
    void* ws;
    size_t ws_bytes;
    bool want_nl;
    int64_t* offsets;
    int32_t* counts;
    int32_t* point_idx;
    float* dist;
    int64_t capacity;
    int64_t* n_pairs_dev;
    bool want_hist;
    int32_t bins;
    float r_min;
    uint64_t* hist;
    hipStream_t stream;
};

int run_pairs(const QueryCall& c)
{
    if (!c.pts && c.n > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    if (c.n < 0 || c.nq < 0) return set_error(PPA_EINVAL, "negative point count");
    if (c.n > 0x7fffffffLL || c.nq > 0x7fffffffLL)
        return set_error(PPA_EINVAL, "point counts are limited to 2^31 - 1");
    if (!c.qpts && c.nq != c.n)
        return set_error(PPA_EINVAL, "nq must equal n when query points are NULL");
    if (!(isfinite(c.r_max) && c.r_max > 0.f))
        return set_error(PPA_EINVAL, "r_max must be finite and positive");
    if (c.flags & ~PPA_SORT_ROWS) return set_error(PPA_EINVAL, "unknown flags 0x%x", c.flags);
    if (c.want_nl) {
        if (!c.offsets || !c.n_pairs_dev || (!c.point_idx && c.capacity > 0))
            return set_error(PPA_EINVAL, "offsets, point_idx and n_pairs_dev are required");
        if (c.capacity < 0) return set_error(PPA_EINVAL, "capacity must be >= 0");
    }
    if (c.want_hist) {
        if (!c.hist) return set_error(PPA_EINVAL, "histogram pointer is NULL");
        if (c.bins < 1) return set_error(PPA_EINVAL, "bins must be >= 1");
        if (!(isfinite(c.r_min) && c.r_min >= 0.f && c.r_min < c.r_max))
            return set_error(PPA_EINVAL, "need 0 <= r_min < r_max");
    }
    BoxPrep bp;
    int rc = prepare_box(c.box, &bp);
    if (rc) return rc;
    if ((rc = check_cutoff(bp, c.r_max))) return rc;
    Grid g;
    pair_grid(bp, c.r_max, c.n, &g);
    Workspace W{};
    const int64_t nq_sep = c.qpts ? c.nq : 0;
    const int32_t lay_flags = c.want_nl ? PPA_WS_NLIST : 0;
    const size_t need = workspace_layout(g, c.n, nq_sep, lay_flags, nullptr, &W);
    if (!c.ws || ((uintptr_t)c.ws & 255) || c.ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, c.ws_bytes);
    workspace_layout(g, c.n, nq_sep, lay_flags, c.ws, &W);
    hipStream_t s = c.stream;

    // n_pairs_dev doubles as the reservation counter of the one-pass mode
    launch_zero(W, g, c.qpts != nullptr, nullptr, 0, s);
    launch_build_cells(c.pts, W.pts, bp, g, W.status, s);
    if (c.qpts) launch_build_cells(c.qpts, W.qry, bp, g, W.status, s);

    PairArgs A{};
    A.cand = W.pts.local;
    A.cand_start = W.pts.cell_start;
    A.qsorted = W.qry.local;
    A.q_start = W.qry.cell_start;
    for (int k = 0; k < 3; ++k) A.geom.n[k] = g.n[k];
    A.geom.ncells = g.ncells;
    A.geom.nsten = g.nsten;
    A.geom.center = 0;
    memcpy(A.geom.off, g.off, sizeof(A.geom.off));
    A.geom.r2max = c.r_max * c.r_max;
    A.geom.dot = expanded_test_ok(bp, g, c.r_max) ? 1 : 0;
    A.geom.split = pair_split(g.ncells, c.nq);
    A.offsets = c.offsets;
    A.point_idx = c.point_idx;
    A.dist = c.dist;
    A.capacity = c.capacity;
    A.status = W.status;
    A.hist = (unsigned long long*)c.hist;
    A.bins = c.want_hist ? c.bins : 0;
    A.r_min = c.r_min;
    A.inv_dr = c.want_hist ? (float)((double)c.bins / ((double)c.r_max - (double)c.r_min)) : 0.f;
    const int dim = bp.dim;
    const int excl = !c.exclude_ii ? 0 : (c.qpts ? 2 : 1);

    ProfileEvents pe = take_profile_events();
    if (c.want_nl) {
        A.counts = c.counts ? c.counts : W.qry_row_counts;
        record(pe.ev[0], s);
        launch_count(A, dim, excl, s);
        record(pe.ev[1], s);
        launch_scan_i64_total(A.counts, c.offsets, c.nq, W.row_scan_flags, W.row_scan_ticket,
                              (unsigned long long*)c.n_pairs_dev, s);
    }
    record(pe.ev[2], s);
    launch_fill(A, dim, excl, c.want_nl, c.want_hist, s);
    record(pe.ev[3], s);
    if (c.want_nl && (c.flags & PPA_SORT_ROWS))
        launch_sort_rows(c.offsets, c.nq, c.point_idx, c.dist, c.capacity, s);
    return hip_check(hipGetLastError(), "kernel launch");
}

// ---------------------------------------------------------------------------
// k nearest neighbours: plan, workspace and launch sequence.
// ---------------------------------------------------------------------------
constexpr double kKnnCellScale = 1.15;  // cell width / expected k-th neighbour distance
constexpr int kKnnMaxK = 64;

struct KnnPlan {
    Grid g;
    bool full;     // every row has exactly k entries: written in place at k i
    double lim;    // search limit: min(r_guard, half the smallest width)
    double r_est;  // expected k-th neighbour distance at the points' density
};

int knn_plan(const BoxPrep& bp, int64_t n, int32_t k, float r_guard, KnnPlan* P)
{
    if (k < 1 || k > kKnnMaxK) return set_error(PPA_EINVAL, "k must be in [1, %d]", kKnnMaxK);
    if (!(isfinite(r_guard) && r_guard >= 0.f))
        return set_error(PPA_EINVAL, "r_guard must be finite and >= 0");
    int rc;
    if (r_guard > 0.f && (rc = check_cutoff(bp, r_guard))) return rc;
    const double half = 0.5 * fmin(bp.width[0], fmin(bp.width[1], bp.width[2]));
    // two images of one point are at least the smallest width apart, so below
    // half of it (less a margin for rounding) a point appears at most once
    P->lim = half * (1.0 - 2e-6);
    if (r_guard > 0.f) P->lim = fmin(P->lim, (double)r_guard);
    const double vol = bp.M[0][0] * bp.M[1][1] * (bp.dim == 3 ? bp.M[2][2] : 1.0);
    const double rho = (double)(n > 0 ? n : 1) / vol;
    const double unit = bp.dim == 3 ? 4.0 / 3.0 * M_PI : M_PI;
    P->r_est = pow((double)k / (rho * unit), 1.0 / bp.dim);
    double cell = kKnnCellScale * P->r_est;
    if (r_guard > 0.f) cell = fmin(cell, (double)r_guard);  // every row then fits in the block
    cell = fmin(cell, half);
    make_grid(bp, cell, n, &P->g);
    P->full = r_guard == 0.f && n - 1 >= k;
    return PPA_OK;
}

// Workspace of a k-nearest query: the cell lists, the deferred-query list
// and, for rows that may be short, rows staged at stride k plus the scan
// state of their offsets.
struct KnnSpace {
    Workspace W;
    int* deferred;
    int32_t* st_idx;
    float* st_dist;
    size_t bytes;
};

size_t knn_layout(const KnnPlan& P, int64_t n, int64_t nq_sep, int32_t k, void* base_v,
                  KnnSpace* S)
{
    char* base = (char*)base_v;
    size_t off = workspace_layout(P.g, n, nq_sep, P.full ? 0 : PPA_WS_NLIST, base_v, &S->W);
    const int64_t nrow = nq_sep > 0 ? nq_sep : n;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off = (off + bytes + 255) & ~(size_t)255;
        return p;
    };
    S->deferred = (int*)take(sizeof(int) * (size_t)(nrow > 0 ? nrow : 1));
    S->st_idx = nullptr;
    S->st_dist = nullptr;
    if (!P.full) {
        S->st_idx = (int32_t*)take(sizeof(int32_t) * (size_t)nrow * (size_t)k);
        S->st_dist = (float*)take(sizeof(float) * (size_t)nrow * (size_t)k);
    }
    S->bytes = off;
    return off;
}

int run_knn(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
            int32_t k, float r_guard, int32_t exclude_ii, int32_t flags, void* ws,
            size_t ws_bytes, int64_t* offsets, int32_t* counts, int32_t* point_idx, float* dist,
            int64_t* n_pairs_dev, hipStream_t s)
{
    if (!pts && n > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    if (n < 0 || nq < 0) return set_error(PPA_EINVAL, "negative point count");
    if (n > 0x7fffffffLL || nq > 0x7fffffffLL || (int64_t)k * (nq > n ? nq : n) > (1LL << 40))
        return set_error(PPA_EINVAL, "point counts are limited to 2^31 - 1");
    if (!qpts && nq != n) return set_error(PPA_EINVAL, "nq must equal n when query points are NULL");
    if (flags != 0) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    if (!offsets || !n_pairs_dev || (!point_idx && nq > 0))
        return set_error(PPA_EINVAL, "offsets, point_idx and n_pairs_dev are required");
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    KnnPlan P;
    if ((rc = knn_plan(bp, n, k, r_guard, &P))) return rc;
    const int64_t nq_sep = qpts ? nq : 0;
    KnnSpace S{};
    const size_t need = knn_layout(P, n, nq_sep, k, nullptr, &S);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, ws_bytes);
    knn_layout(P, n, nq_sep, k, ws, &S);
    Workspace& W = S.W;
    const Grid& g = P.g;

    launch_zero(W, g, qpts != nullptr, nullptr, 0, s);  // also clears the deferred counter
    launch_build_cells(pts, W.pts, bp, g, W.status, s);
    if (qpts) launch_build_cells(qpts, W.qry, bp, g, W.status, s);

    KnnArgs A{};
    A.cand = W.pts.local;
    A.cand_start = W.pts.cell_start;
    A.qsorted = W.qry.local;
    A.q_start = W.qry.cell_start;
    A.q_cell_of = W.qry.cell_of;
    for (int d = 0; d < 3; ++d) A.geom.n[d] = g.n[d];
    A.geom.ncells = g.ncells;
    A.geom.nsten = g.nsten;
    memcpy(A.geom.off, g.off, sizeof(A.geom.off));
    KnnGeom& K = A.knn;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            K.minv[r][c] = (float)bp.Minv[r][c];
            K.M[r][c] = bp.M[r][c];
        }
    for (int d = 0; d < 3; ++d) {
        K.nf[d] = (float)g.n[d];
        K.cellw[d] = (float)(bp.width[d] / g.n[d]);
    }
    if (bp.dim == 2) K.cellw[2] = INFINITY;
    {
        double wmin = INFINITY;
        for (int d = 0; d < bp.dim; ++d) wmin = fmin(wmin, bp.width[d] / g.n[d]);
        K.smax = (int)ceil(P.lim / wmin) + 2;
    }
    K.lim2 = (float)(P.lim * P.lim);
    K.t0 = (float)fmin(1.44 * P.r_est * P.r_est, P.lim * P.lim);
    K.guard = r_guard > 0.f ? 1 : 0;
    K.excl = exclude_ii ? 1 : 0;
    K.k = k;
    K.n_points = (int)n;
    A.row_len = P.full ? counts : (counts ? counts : W.qry_row_counts);
    A.out_idx = P.full ? point_idx : S.st_idx;
    A.out_dist = P.full ? dist : (dist ? S.st_dist : nullptr);
    A.deferred = S.deferred;
    A.n_deferred = W.counters;
    A.status = W.status;

    ProfileEvents pe = take_profile_events();
    record(pe.ev[2], s);
    if (nq > 0) launch_knn(A, bp.dim, s);
    record(pe.ev[3], s);
    if (P.full) {
        launch_knn_offsets(offsets, nq, k, n_pairs_dev, s);
    } else {
        launch_scan_i64_total(A.row_len, offsets, nq, W.row_scan_flags, W.row_scan_ticket,
                              (unsigned long long*)n_pairs_dev, s);
        launch_knn_pack(nq, k, A.row_len, offsets, S.st_idx, S.st_dist, point_idx, dist, s);
    }
    return hip_check(hipGetLastError(), "kernel launch");
}

// ---------------------------------------------------------------------------
// 2D PMFT: plan (reachable-bin table, launch shape), workspace, launches.
// ---------------------------------------------------------------------------
struct PmftPlan {
    Grid g;
    PmftTable table;
    int words;    // LDS histogram words (0: global atomics)
    int entries;  // bins of the LDS histogram
    int packed;   // two 16-bit counters per word
    int blocks;
};

int pmft_plan(const BoxPrep& bp, int64_t n, int32_t nbx, int32_t nby, float x_max, float y_max,
              float r_max, PmftPlan* P)
{
    if (bp.dim != 2) return set_error(PPA_EINVAL, "the 2D PMFT needs a 2D box");
    if (nbx < 1 || nby < 1 || (int64_t)nbx * nby > 0x7fffffffLL)
        return set_error(PPA_EINVAL, "bad bin counts %d x %d", nbx, nby);
    if (!(isfinite(x_max) && x_max > 0.f && isfinite(y_max) && y_max > 0.f))
        return set_error(PPA_EINVAL, "x_max and y_max must be finite and positive");
    if (!(isfinite(r_max) && r_max > 0.f)) return set_error(PPA_EINVAL, "r_max must be positive");
    int rc;
    if ((rc = check_cutoff(bp, r_max))) return rc;
    pair_grid(bp, r_max, n, &P->g);
    // bins a bond shorter than r_max can reach: per row ix, the iy range
    // covering |y| < sqrt(r_max^2 - min|x|^2), widened by a bin each side
    P->words = 0;
    P->entries = 0;
    P->packed = 0;
    if (nbx <= kPmftMaxRows) {
        const double dx = 2.0 * x_max / nbx, dy = 2.0 * y_max / nby, r = r_max;
        int base = 0;
        for (int ix = 0; ix < nbx; ++ix) {
            const double x0 = -(double)x_max + ix * dx, x1 = x0 + dx;
            const double mx = (x0 <= 0.0 && x1 >= 0.0) ? 0.0 : fmin(fabs(x0), fabs(x1));
            int lo = 0, hi = 0;
            if (mx < r * (1.0 + 1e-4)) {
                const double ym = sqrt(fmax(0.0, r * r - mx * mx)) * (1.0 + 1e-4) + 1e-6 * r;
                lo = (int)fmax(0.0, floor((y_max - ym) / dy) - 1.0);
                hi = (int)fmin((double)nby, floor((y_max + ym) / dy) + 2.0);
                if (hi < lo) hi = lo;
            }
            P->table.lo[ix] = lo;
            P->table.base[ix] = base;
            base += hi - lo;
        }
        P->table.base[nbx] = base;
        // 32-bit counters, or two 16-bit counters per word when that is the
        // only way to fit the LDS or lets more workgroups share a CU
        const int half = (base + 1) / 2;
        const bool fit32 = (size_t)base * sizeof(unsigned) <= pmft_lds_limit();
        const bool fit16 = (size_t)half * sizeof(unsigned) <= pmft_lds_limit();
        if (base > 0 && fit16) {
            P->entries = base;
            if (!fit32 || pmft_blocks_per_cu(half, 1) > pmft_blocks_per_cu(base, 0)) {
                P->packed = 1;
                P->words = half;
            } else {
                P->words = base;
            }
        }
    }
    P->blocks = pmft_workgroups(P->words, P->packed);
    return PPA_OK;
}

size_t pmft_layout(const PmftPlan& P, int64_t n, int64_t nq_sep, void* base_v, Workspace* W,
                   unsigned** partial, unsigned** level2)
{
    char* base = (char*)base_v;
    size_t off = workspace_layout(P.g, n, nq_sep, 0, base_v, W);
    *partial = base ? (unsigned*)(base + off) : nullptr;
    off = (off + sizeof(unsigned) * (size_t)P.blocks * (size_t)P.entries + 255) & ~(size_t)255;
    *level2 = base ? (unsigned*)(base + off) : nullptr;
    off += sizeof(unsigned) * (size_t)partial_rows(P.blocks) * (size_t)P.entries;
    return (off + 255) & ~(size_t)255;
}

int run_pmft(const ppa_box* box, const float* pts, int64_t n, const float* qpts,
             const float* angles, int64_t nq, int32_t nbx, int32_t nby, float x_max, float y_max,
             float r_max, int32_t exclude_ii, int32_t flags, void* ws, size_t ws_bytes,
             uint32_t* counts, hipStream_t s)
{
    if (!pts && n > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    if (n < 0 || nq < 0) return set_error(PPA_EINVAL, "negative point count");
    if (n > 0x7fffffffLL || nq > 0x7fffffffLL)
        return set_error(PPA_EINVAL, "point counts are limited to 2^31 - 1");
    if (!qpts && nq != n) return set_error(PPA_EINVAL, "nq must equal n when query points are NULL");
    if (!angles && nq > 0) return set_error(PPA_EINVAL, "orientations pointer is NULL");
    if (!counts) return set_error(PPA_EINVAL, "counts pointer is NULL");
    if (flags != 0) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    PmftPlan P;
    if ((rc = pmft_plan(bp, n, nbx, nby, x_max, y_max, r_max, &P))) return rc;
    const int64_t nq_sep = qpts ? nq : 0;
    Workspace W{};
    unsigned* partial = nullptr;
    unsigned* level2 = nullptr;
    const size_t need = pmft_layout(P, n, nq_sep, nullptr, &W, &partial, &level2);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, ws_bytes);
    pmft_layout(P, n, nq_sep, ws, &W, &partial, &level2);
    if (nq == 0) return PPA_OK;
    const Grid& g = P.g;
    launch_zero(W, g, qpts != nullptr, nullptr, 0, s);
    launch_build_cells(pts, W.pts, bp, g, W.status, s);
    if (qpts) launch_build_cells(qpts, W.qry, bp, g, W.status, s);

    PmftArgs A{};
    A.cand = W.pts.local;
    A.cand_start = W.pts.cell_start;
    A.qsorted = W.qry.local;
    A.q_start = W.qry.cell_start;
    A.angles = angles;
    for (int d = 0; d < 3; ++d) A.geom.n[d] = g.n[d];
    A.geom.ncells = g.ncells;
    A.geom.nsten = g.nsten;
    memcpy(A.geom.off, g.off, sizeof(A.geom.off));
    A.geom.r2max = r_max * r_max;
    A.excl = exclude_ii ? 1 : 0;
    A.nbx = nbx;
    A.nby = nby;
    A.x_max = x_max;
    A.y_max = y_max;
    A.inv_dx = (float)((double)nbx / (2.0 * x_max));
    A.inv_dy = (float)((double)nby / (2.0 * y_max));
    A.words = P.words;
    A.entries = P.entries;
    A.packed = P.packed;
    A.partial = partial;
    A.level2 = level2;
    A.counts = counts;
    A.table = P.table;
    ProfileEvents pe = take_profile_events();
    record(pe.ev[2], s);
    launch_pmft(A, P.blocks, s);
    record(pe.ev[3], s);
    return hip_check(hipGetLastError(), "kernel launch");
}

// ---------------------------------------------------------------------------
// PMFT over three pair coordinates (XYT in 2D, XYZ in 3D): validation,
// workspace (the cell lists alone) and launch.
// ---------------------------------------------------------------------------
struct Pmft3Call {
    int mode;
    const ppa_box* box;
    const float* pts;
    const float* p_orient;
    int64_t n;
    const float* qpts;
    const float* q_orient;
    int64_t nq;
    int32_t nb[3];
    float max[3];
    float r_max;
};

int pmft3_check(const Pmft3Call& c, BoxPrep* bp, Grid* g)
{
    const int dim = c.mode == kPmftXyt ? 2 : 3;
    if (c.n < 0 || c.nq < 0) return set_error(PPA_EINVAL, "negative point count");
    if (c.n > 0x7fffffffLL || c.nq > 0x7fffffffLL)
        return set_error(PPA_EINVAL, "point counts are limited to 2^31 - 1");
    const int64_t nbins = (int64_t)c.nb[0] * c.nb[1] * c.nb[2];
    if (c.nb[0] < 1 || c.nb[1] < 1 || c.nb[2] < 1 || nbins > 0x7fffffffLL)
        return set_error(PPA_EINVAL, "bad bin counts %d x %d x %d", c.nb[0], c.nb[1], c.nb[2]);
    for (int k = 0; k < (dim == 3 ? 3 : 2); ++k)
        if (!(isfinite(c.max[k]) && c.max[k] > 0.f))
            return set_error(PPA_EINVAL, "the coordinate ranges must be finite and positive");
    if (!(isfinite(c.r_max) && c.r_max > 0.f)) return set_error(PPA_EINVAL, "r_max must be positive");
    int rc = prepare_box(c.box, bp);
    if (rc) return rc;
    if (bp->dim != dim)
        return set_error(PPA_EINVAL, dim == 2 ? "the XYT PMFT needs a 2D box"
                                              : "the XYZ PMFT needs a 3D box");
    if ((rc = check_cutoff(*bp, c.r_max))) return rc;
    pair_grid(*bp, c.r_max, c.n, g);
    return PPA_OK;
}

int pmft3_workspace(const Pmft3Call& c, size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    BoxPrep bp;
    Grid g;
    int rc = pmft3_check(c, &bp, &g);
    if (rc) return rc;
    Workspace W{};
    *bytes = workspace_layout(g, c.n, c.nq, 0, nullptr, &W);
    return PPA_OK;
}

int run_pmft3(const Pmft3Call& c, int32_t exclude_ii, int32_t flags, void* ws, size_t ws_bytes,
              uint32_t* counts, hipStream_t s)
{
    if (!c.pts && c.n > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    if (!c.qpts && c.nq != c.n)
        return set_error(PPA_EINVAL, "nq must equal n when query points are NULL");
    if (!c.q_orient && c.nq > 0) return set_error(PPA_EINVAL, "orientations pointer is NULL");
    if (c.mode == kPmftXyt && !c.p_orient && c.n > 0)
        return set_error(PPA_EINVAL, "orientations of the points are NULL");
    if (c.mode == kPmftXyz && ((uintptr_t)c.q_orient & 15))
        return set_error(PPA_EINVAL, "quaternions must be 16-byte aligned");
    if (!counts) return set_error(PPA_EINVAL, "counts pointer is NULL");
    if (flags != 0) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    BoxPrep bp;
    Grid g;
    int rc = pmft3_check(c, &bp, &g);
    if (rc) return rc;
    const int64_t nq_sep = c.qpts ? c.nq : 0;
    Workspace W{};
    const size_t need = workspace_layout(g, c.n, nq_sep, 0, nullptr, &W);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, ws_bytes);
    workspace_layout(g, c.n, nq_sep, 0, ws, &W);
    if (c.nq == 0) return PPA_OK;
    launch_zero(W, g, c.qpts != nullptr, nullptr, 0, s);
    launch_build_cells(c.pts, W.pts, bp, g, W.status, s);
    if (c.qpts) launch_build_cells(c.qpts, W.qry, bp, g, W.status, s);

    Pmft3Args A{};
    A.cand = W.pts.local;
    A.cand_start = W.pts.cell_start;
    A.qsorted = W.qry.local;
    A.q_start = W.qry.cell_start;
    A.q_orient = c.q_orient;
    A.p_orient = c.p_orient;
    for (int d = 0; d < 3; ++d) A.geom.n[d] = g.n[d];
    A.geom.ncells = g.ncells;
    A.geom.nsten = g.nsten;
    memcpy(A.geom.off, g.off, sizeof(A.geom.off));
    A.geom.r2max = c.r_max * c.r_max;
    A.mode = c.mode;
    A.excl = exclude_ii ? 1 : 0;
    for (int k = 0; k < 3; ++k) {
        A.nb[k] = c.nb[k];
        A.max[k] = c.max[k];
        // the angle spans [0, 2 pi); lengths span [-max, max)
        const double span = (c.mode == kPmftXyt && k == 2) ? 2.0 * M_PI : 2.0 * (double)c.max[k];
        A.inv_w[k] = (float)((double)c.nb[k] / span);
    }
    A.counts = counts;
    A.status = W.status;
    ProfileEvents pe = take_profile_events();
    record(pe.ev[2], s);
    launch_pmft3(A, s);
    record(pe.ev[3], s);
    return hip_check(hipGetLastError(), "kernel launch");
}

// ---------------------------------------------------------------------------
// Spatial correlation function: plan, workspace and launches.
// ---------------------------------------------------------------------------
struct CorrPlan {
    Grid g;
    int blocks;
};

int corr_plan(const BoxPrep& bp, int64_t n, int32_t bins, float r_min, float r_max, CorrPlan* P)
{
    if (bins < 1 || bins > kCorrMaxBins)
        return set_error(PPA_EINVAL, "bins must be in [1, %d]", kCorrMaxBins);
    if (!(isfinite(r_min) && isfinite(r_max) && r_min >= 0.f && r_min < r_max))
        return set_error(PPA_EINVAL, "need 0 <= r_min < r_max");
    int rc;
    if ((rc = check_cutoff(bp, r_max))) return rc;
    pair_grid(bp, r_max, n, &P->g);
    P->blocks = corr_workgroups(bp.dim, bins, P->g.ncells);
    return PPA_OK;
}

size_t corr_layout(const CorrPlan& P, int64_t n, int64_t nq_sep, int32_t bins, void* base_v,
                   Workspace* W, CorrArgs* A)
{
    char* base = (char*)base_v;
    size_t off = workspace_layout(P.g, n, nq_sep, 0, base_v, W);
    const size_t rows = (size_t)partial_rows(P.blocks);
    auto take = [&](size_t bytes) {
        void* p = base ? (void*)(base + off) : nullptr;
        off = (off + bytes + 255) & ~(size_t)255;
        return p;
    };
    A->psum = (double*)take(sizeof(double) * 2 * (size_t)bins * P.blocks);
    A->pcnt = (unsigned long long*)take(sizeof(unsigned long long) * (size_t)bins * P.blocks);
    A->lsum = (double*)take(sizeof(double) * 2 * (size_t)bins * rows);
    A->lcnt = (unsigned long long*)take(sizeof(unsigned long long) * (size_t)bins * rows);
    return off;
}

int run_corr(const ppa_box* box, const float* pts, const float* values, int64_t n,
             const float* qpts, const float* qvalues, int64_t nq, int32_t bins, float r_min,
             float r_max, int32_t exclude_ii, int32_t flags, void* ws, size_t ws_bytes,
             double* sums, uint64_t* counts, hipStream_t s)
{
    if (!pts && n > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    if (n < 0 || nq < 0) return set_error(PPA_EINVAL, "negative point count");
    if (n > 0x7fffffffLL || nq > 0x7fffffffLL)
        return set_error(PPA_EINVAL, "point counts are limited to 2^31 - 1");
    if (!qpts && nq != n) return set_error(PPA_EINVAL, "nq must equal n when query points are NULL");
    if (!values && n > 0) return set_error(PPA_EINVAL, "values pointer is NULL");
    if (qpts && !qvalues && nq > 0) return set_error(PPA_EINVAL, "query values pointer is NULL");
    if (((uintptr_t)values & 7) || ((uintptr_t)qvalues & 7))
        return set_error(PPA_EINVAL, "values must be 8-byte aligned");
    if (!sums || !counts) return set_error(PPA_EINVAL, "output pointer is NULL");
    if (flags != 0) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    CorrPlan P;
    if ((rc = corr_plan(bp, n, bins, r_min, r_max, &P))) return rc;
    const int64_t nq_sep = qpts ? nq : 0;
    Workspace W{};
    CorrArgs A{};
    const size_t need = corr_layout(P, n, nq_sep, bins, nullptr, &W, &A);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, ws_bytes);
    corr_layout(P, n, nq_sep, bins, ws, &W, &A);
    if (nq == 0) return PPA_OK;
    const Grid& g = P.g;
    launch_zero(W, g, qpts != nullptr, nullptr, 0, s);
    launch_build_cells(pts, W.pts, bp, g, W.status, s);
    if (qpts) launch_build_cells(qpts, W.qry, bp, g, W.status, s);

    A.cand = W.pts.local;
    A.cand_start = W.pts.cell_start;
    A.qsorted = W.qry.local;
    A.q_start = W.qry.cell_start;
    A.pval = (const float2*)values;
    A.qval = (const float2*)(qvalues ? qvalues : values);
    for (int d = 0; d < 3; ++d) A.geom.n[d] = g.n[d];
    A.geom.ncells = g.ncells;
    A.geom.nsten = g.nsten;
    memcpy(A.geom.off, g.off, sizeof(A.geom.off));
    A.geom.r2max = r_max * r_max;
    A.excl = exclude_ii ? 1 : 0;
    A.bins = bins;
    A.r_min = r_min;
    A.inv_dr = (float)((double)bins / ((double)r_max - (double)r_min));
    A.sums = sums;
    A.counts = (unsigned long long*)counts;
    A.status = W.status;
    ProfileEvents pe = take_profile_events();
    record(pe.ev[2], s);
    launch_corr(A, bp.dim, P.blocks, s);
    record(pe.ev[3], s);
    return hip_check(hipGetLastError(), "kernel launch");
}

// ---------------------------------------------------------------------------
// Gaussian-smoothed RDF: plan, workspace and launches.
// ---------------------------------------------------------------------------
struct SmoothPlan {
    Grid g;
    double r_s;  // pair cutoff r_max + 8 sigma
    int blocks;
};

int smooth_plan(const BoxPrep& bp, int64_t n, int32_t bins, float r_max, float sigma, bool adjoint,
                SmoothPlan* P)
{
    if (bins < 1 || bins > kSmoothMaxBins)
        return set_error(PPA_EINVAL, "bins must be in [1, %d]", kSmoothMaxBins);
    if (!(isfinite(r_max) && r_max > 0.f)) return set_error(PPA_EINVAL, "r_max must be positive");
    if (!(isfinite(sigma) && sigma > 0.f)) return set_error(PPA_EINVAL, "sigma must be positive");
    P->r_s = (double)r_max + 8.0 * (double)sigma;
    int rc;
    if ((rc = check_cutoff(bp, P->r_s))) return rc;
    make_grid(bp, P->r_s, n, &P->g);
    P->blocks = smooth_workgroups(adjoint, bp.dim, bins);
    return PPA_OK;
}

size_t smooth_layout(const SmoothPlan& P, int64_t n, int32_t bins, void* base_v, Workspace* W,
                     double** partial, double** level2)
{
    char* base = (char*)base_v;
    size_t off = workspace_layout(P.g, n, 0, 0, base_v, W);
    *partial = base ? (double*)(base + off) : nullptr;
    off = (off + sizeof(double) * (size_t)P.blocks * (size_t)bins + 255) & ~(size_t)255;
    *level2 = base ? (double*)(base + off) : nullptr;
    off += sizeof(double) * (size_t)partial_rows(P.blocks) * (size_t)bins;
    return (off + 255) & ~(size_t)255;
}

int run_smooth(const ppa_box* box, const float* pts, int64_t n, int32_t bins, float r_max,
               float sigma, const double* grad_h, int32_t flags, void* ws, size_t ws_bytes,
               double* h, float* grad, hipStream_t s)
{
    const bool adjoint = grad != nullptr;
    if (!pts && n > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    if (n < 0 || n > 0x7fffffffLL) return set_error(PPA_EINVAL, "bad point count");
    if (flags != 0) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    if (adjoint ? !grad_h : !h) return set_error(PPA_EINVAL, "output or gradient pointer is NULL");
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    SmoothPlan P;
    if ((rc = smooth_plan(bp, n, bins, r_max, sigma, adjoint, &P))) return rc;
    Workspace W{};
    double* partial = nullptr;
    double* level2 = nullptr;
    const size_t need = smooth_layout(P, n, bins, nullptr, &W, &partial, &level2);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, ws_bytes);
    smooth_layout(P, n, bins, ws, &W, &partial, &level2);
    if (n == 0) return PPA_OK;
    const Grid& g = P.g;
    launch_zero(W, g, false, nullptr, 0, s);
    launch_build_cells(pts, W.pts, bp, g, W.status, s);

    SmoothArgs A{};
    A.cand = W.pts.local;
    A.cand_start = W.pts.cell_start;
    for (int d = 0; d < 3; ++d) A.geom.n[d] = g.n[d];
    A.geom.ncells = g.ncells;
    A.geom.nsten = g.nsten;
    memcpy(A.geom.off, g.off, sizeof(A.geom.off));
    A.geom.r2max = (float)(P.r_s * P.r_s);
    // the stencil offsets again in float64, for the exact pair vectors
    for (int t = 0; t < 27; ++t) {
        const int centre = g.nsten / 2;
        const int code = t == 0 ? centre : (t == centre ? 0 : t);
        double d[3] = {(double)(code % 3 - 1), (double)((code / 3) % 3 - 1),
                       bp.dim == 3 ? (double)(code / 9 - 1) : 0.0};
        if (t >= g.nsten) d[0] = d[1] = d[2] = 0.0;
        const double f[3] = {d[0] / g.n[0], d[1] / g.n[1], d[2] / g.n[2]};
        A.offd[t][0] = bp.M[0][0] * f[0] + bp.M[0][1] * f[1] + bp.M[0][2] * f[2];
        A.offd[t][1] = bp.M[1][1] * f[1] + bp.M[1][2] * f[2];
        A.offd[t][2] = bp.dim == 3 ? bp.M[2][2] * f[2] : 0.0;
    }
    A.bins = bins;
    A.dr = (double)r_max / bins;
    A.w8 = 8.0 * (double)sigma;
    A.inv_dr = (float)((double)bins / (double)r_max);
    const double sg = sigma;
    A.k2 = (float)(1.4426950408889634 / (2.0 * sg * sg));
    const double drf = (double)(float)A.dr;  // the step the kernel adds
    A.step2 = (float)exp2(-2.0 * (double)A.k2 * drf * drf);
    A.hscale = (float)(A.dr / (sg * sqrt(2.0 * M_PI)));
    A.gscale = (float)(A.dr / (sg * sg * sg * sqrt(2.0 * M_PI)));
    A.partial = partial;
    A.level2 = level2;
    A.h = h;
    A.grad_h = grad_h;
    A.grad = grad;
    // enough work units for four per resident wavefront: split home cells
    // into parts of their query lists when cells are fewer than that
    const long long waves = (long long)P.blocks * kWavesPerBlock;
    long long split = (4 * waves + g.ncells - 1) / g.ncells;
    const long long per_cell = n / (g.ncells > 0 ? g.ncells : 1);
    if (split > per_cell / 8) split = per_cell / 8;  // keep >= 8 queries per unit
    A.split = (int)(split < 1 ? 1 : (split > 16 ? 16 : split));
    long long want = ((long long)g.ncells * A.split + kWavesPerBlock - 1) / kWavesPerBlock;
    int blocks = (int)(want < P.blocks ? (want + 7) / 8 * 8 : P.blocks);
    if (blocks > P.blocks) blocks = P.blocks;
    ProfileEvents pe = take_profile_events();
    record(pe.ev[2], s);
    if (adjoint)
        launch_smooth_bwd(A, bp.dim, blocks, s);
    else
        launch_smooth_fwd(A, bp.dim, blocks, s);
    record(pe.ev[3], s);
    return hip_check(hipGetLastError(), "kernel launch");
}

}  // namespace

extern "C" {

int ppa_box_from_matrix(const double m[9], int32_t dim, ppa_box* out)
{
    if (!m || !out) return set_error(PPA_EINVAL, "NULL argument");
    if (dim != 2 && dim != 3) return set_error(PPA_EINVAL, "dim must be 2 or 3");
    for (int i = 0; i < 9; ++i)
        if (!isfinite(m[i])) return set_error(PPA_EBOX, "matrix has a non-finite entry");
    if (m[3] != 0.0 || m[6] != 0.0 || m[7] != 0.0)
        return set_error(PPA_EBOX, "matrix must be upper triangular (rotate it first)");
    const double Lx = m[0], Ly = m[4], Lz = dim == 3 ? m[8] : 1.0;
    if (!(Lx > 0 && Ly > 0 && Lz > 0)) return set_error(PPA_EBOX, "diagonal must be positive");
    out->L[0] = Lx;
    out->L[1] = Ly;
    out->L[2] = dim == 3 ? Lz : 1.0;
    out->tilt[0] = m[1] / Ly;
    out->tilt[1] = dim == 3 ? m[2] / Lz : 0.0;
    out->tilt[2] = dim == 3 ? m[5] / Lz : 0.0;
    out->dim = dim;
    return PPA_OK;
}

int ppa_box_widths(const ppa_box* box, double widths[3])
{
    if (!widths) return set_error(PPA_EINVAL, "widths is NULL");
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    for (int k = 0; k < 3; ++k) widths[k] = bp.width[k];
    return PPA_OK;
}

int ppa_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, float r_cut, int32_t flags,
                        size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    if (n < 0 || nq < 0) return set_error(PPA_EINVAL, "negative point count");
    if (!(isfinite(r_cut) && r_cut > 0.f)) return set_error(PPA_EINVAL, "r_cut must be positive");
    if (flags & ~PPA_WS_NLIST) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    if ((rc = check_cutoff(bp, r_cut))) return rc;
    Grid g;
    pair_grid(bp, r_cut, n, &g);
    Workspace W{};
    *bytes = workspace_layout(g, n, nq, flags, nullptr, &W);
    return PPA_OK;
}

int ppa_query_ball(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
                   float r_max, int32_t exclude_ii, int32_t flags, void* ws, size_t ws_bytes,
                   int64_t* offsets, int32_t* counts, int32_t* point_idx, float* dist,
                   int64_t capacity, int64_t* n_pairs_dev, hipStream_t stream)
{
    QueryCall c{box, pts, n, qpts, nq, r_max, exclude_ii, flags, ws, ws_bytes, true, offsets,
                counts, point_idx, dist, capacity, n_pairs_dev, false, 0, 0.f, nullptr, stream};
    return run_pairs(c);
}

}  // extern "C"

// Scratch of ppa_rdf_static: a fixed device array, so that call allocates
// nothing.  Its address is looked up once per device (each device holds its
// own copy of the array) and kept; host code uses only that address.
namespace ppa {
namespace {
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

int static_scratch(void** out, bool create)
{
    int dev = 0;
    int rc = hip_check(hipGetDevice(&dev), "get device");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return set_error(PPA_EDEVICE, "device ordinal %d", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        if (!create) return set_error(PPA_EINVAL, "workspace is NULL");
        void* p = nullptr;
        rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "static scratch address");
        if (rc) return rc;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PPA_OK;
}
}  // namespace
}  // namespace ppa

extern "C" {

int ppa_rdf_static(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
                   int32_t bins, float r_min, float r_max, int32_t exclude_ii, int32_t flags,
                   uint64_t* counts_hist, int64_t* offsets, int32_t* counts, int32_t* point_idx,
                   float* dist, int64_t capacity, int64_t* n_pairs_dev, hipStream_t stream)
{
    size_t need = 0;
    int rc = ppa_workspace_bytes(box, n, qpts ? nq : 0, r_max, offsets ? PPA_WS_NLIST : 0, &need);
    if (rc) return rc;
    if (need > kStaticScratchBytes)
        return set_error(PPA_EWORKSPACE,
                         "the call needs %zu bytes of scratch, more than the static %zu bytes; "
                         "use ppa_rdf with a workspace",
                         need, kStaticScratchBytes);
    void* ws = nullptr;
    if ((rc = static_scratch(&ws, true))) return rc;
    QueryCall c{box,      pts,    n,        qpts,      nq,       r_max,       exclude_ii, flags,
                ws,       kStaticScratchBytes, offsets != nullptr, offsets, counts, point_idx,
                dist,     capacity, n_pairs_dev, true, bins, r_min, counts_hist, stream};
    return run_pairs(c);
}

int ppa_rdf(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
            int32_t bins, float r_min, float r_max, int32_t exclude_ii, int32_t flags, void* ws,
            size_t ws_bytes, uint64_t* counts_hist, int64_t* offsets, int32_t* counts,
            int32_t* point_idx, float* dist, int64_t capacity, int64_t* n_pairs_dev,
            hipStream_t stream)
{
    QueryCall c{box,     pts,    n,        qpts,      nq,       r_max,       exclude_ii, flags,
                ws,      ws_bytes, offsets != nullptr, offsets, counts, point_idx, dist,
                capacity, n_pairs_dev, true, bins, r_min, counts_hist, stream};
    return run_pairs(c);
}

int ppa_rdf_from_nlist(const float* dist, const int64_t* n_pairs_dev, int64_t capacity,
                       int32_t bins, float r_min, float r_max, uint64_t* counts_hist,
                       hipStream_t stream)
{
    if (!n_pairs_dev || !counts_hist || (!dist && capacity > 0))
        return set_error(PPA_EINVAL, "NULL argument");
    if (bins < 1) return set_error(PPA_EINVAL, "bins must be >= 1");
    if (!(isfinite(r_min) && isfinite(r_max) && r_min >= 0.f && r_min < r_max))
        return set_error(PPA_EINVAL, "need 0 <= r_min < r_max");
    const float inv_dr = (float)((double)bins / ((double)r_max - (double)r_min));
    launch_hist_from_dist(dist, n_pairs_dev, capacity, bins, r_min, inv_dr,
                          (unsigned long long*)counts_hist, stream);
    return hip_check(hipGetLastError(), "kernel launch");
}

int ppa_knn_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t k, float r_guard,
                            size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    if (n < 0 || nq < 0) return set_error(PPA_EINVAL, "negative point count");
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    KnnPlan P;
    if ((rc = knn_plan(bp, n, k, r_guard, &P))) return rc;
    KnnSpace S{};
    *bytes = knn_layout(P, n, nq, k, nullptr, &S);
    return PPA_OK;
}

int ppa_query_knn(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
                  int32_t k, float r_guard, int32_t exclude_ii, int32_t flags, void* ws,
                  size_t ws_bytes, int64_t* offsets, int32_t* counts, int32_t* point_idx,
                  float* dist, int64_t* n_pairs_dev, hipStream_t stream)
{
    return run_knn(box, pts, n, qpts, nq, k, r_guard, exclude_ii, flags, ws, ws_bytes, offsets,
                   counts, point_idx, dist, n_pairs_dev, stream);
}

int ppa_pmft2d_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t nbx, int32_t nby,
                               float x_max, float y_max, float r_max, size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    if (n < 0 || nq < 0) return set_error(PPA_EINVAL, "negative point count");
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    PmftPlan P;
    if ((rc = pmft_plan(bp, n, nbx, nby, x_max, y_max, r_max, &P))) return rc;
    Workspace W{};
    unsigned* partial = nullptr;
    unsigned* level2 = nullptr;
    *bytes = pmft_layout(P, n, nq, nullptr, &W, &partial, &level2);
    return PPA_OK;
}

int ppa_pmft2d(const ppa_box* box, const float* pts, int64_t n, const float* qpts,
               const float* angles, int64_t nq, int32_t nbx, int32_t nby, float x_max,
               float y_max, float r_max, int32_t exclude_ii, int32_t flags, void* ws,
               size_t ws_bytes, uint32_t* counts, hipStream_t stream)
{
    return run_pmft(box, pts, n, qpts, angles, nq, nbx, nby, x_max, y_max, r_max, exclude_ii,
                    flags, ws, ws_bytes, counts, stream);
}

int ppa_correlation_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t bins,
                                    float r_min, float r_max, size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    if (n < 0 || nq < 0) return set_error(PPA_EINVAL, "negative point count");
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    CorrPlan P;
    if ((rc = corr_plan(bp, n, bins, r_min, r_max, &P))) return rc;
    Workspace W{};
    CorrArgs A{};
    *bytes = corr_layout(P, n, nq, bins, nullptr, &W, &A);
    return PPA_OK;
}

int ppa_correlation(const ppa_box* box, const float* pts, const float* values, int64_t n,
                    const float* qpts, const float* qvalues, int64_t nq, int32_t bins,
                    float r_min, float r_max, int32_t exclude_ii, int32_t flags, void* ws,
                    size_t ws_bytes, double* sums, uint64_t* counts, hipStream_t stream)
{
    return run_corr(box, pts, values, n, qpts, qvalues, nq, bins, r_min, r_max, exclude_ii, flags,
                    ws, ws_bytes, sums, counts, stream);
}

int ppa_steinhardt_workspace_bytes(int32_t l, int32_t flags, size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    if (l < 0 || l > kSteinMaxL) return set_error(PPA_EINVAL, "l must be in [0, %d]", kSteinMaxL);
    if (flags != 0) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    const size_t w = 2 * (size_t)l + 1;
    *bytes = 256 + ((sizeof(double) * w * w + 255) & ~(size_t)255);
    return PPA_OK;
}

int ppa_steinhardt(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
                   const int64_t* offsets, const int32_t* point_idx, int64_t capacity, int32_t l,
                   int32_t flags, void* ws, size_t ws_bytes, double* ql, double* wl,
                   hipStream_t stream)
{
    if (n < 0 || nq < 0 || capacity < 0) return set_error(PPA_EINVAL, "negative size");
    if (!pts && n > 0) return set_error(PPA_EINVAL, "points pointer is NULL");
    if (!qpts && nq != n) return set_error(PPA_EINVAL, "nq must equal n when query points are NULL");
    if (!offsets) return set_error(PPA_EINVAL, "offsets pointer is NULL");
    if (!point_idx && capacity > 0) return set_error(PPA_EINVAL, "point_idx pointer is NULL");
    if (!ql && nq > 0) return set_error(PPA_EINVAL, "output pointer is NULL");
    size_t need = 0;
    int rc = ppa_steinhardt_workspace_bytes(l, flags, &need);
    if (rc) return rc;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, ws_bytes);
    BoxPrep bp;
    if ((rc = prepare_box(box, &bp))) return rc;
    unsigned* status = (unsigned*)ws;
    double* table = (double*)((char*)ws + 256);
    launch_steinhardt_setup(l, wl != nullptr, table, status, stream);
    SteinArgs A{};
    A.pts = pts;
    A.qpts = qpts ? qpts : pts;
    A.offsets = offsets;
    A.idx = point_idx;
    A.n = n;
    A.nq = nq;
    A.capacity = capacity;
    A.l = l;
    A.dim = bp.dim;
    memcpy(A.m, bp.M, sizeof(A.m));
    memcpy(A.minv, bp.Minv, sizeof(A.minv));
    A.w3j = wl ? table : nullptr;
    A.ql = ql;
    A.wl = wl;
    A.status = status;
    ProfileEvents pe = take_profile_events();
    record(pe.ev[2], stream);
    launch_steinhardt(A, stream);
    record(pe.ev[3], stream);
    return hip_check(hipGetLastError(), "kernel launch");
}

static size_t cluster_layout(int64_t n, void* base_v, ClusterArgs* A)
{
    char* base = (char*)base_v;
    size_t off = 256;  // header: status word at 0, scan ticket at 64, round flags at 128
    const size_t flag_bytes = sizeof(unsigned long long) * scan_flag_count(n) + 256;
    A->status = (unsigned*)base;
    A->ticket = base ? (int*)(base + 64) : nullptr;
    A->round_flags = base ? (int*)(base + 128) : nullptr;  // kClusterRounds ints
    static_assert(128 + 4 * kClusterRounds <= 192, "round flags exceed their part of the header");
    A->giant = base ? (int*)(base + 192) : nullptr;
    A->scan_flags = base ? (unsigned long long*)(base + off) : nullptr;
    off = (off + flag_bytes + 255) & ~(size_t)255;
    A->zero = (unsigned*)base;
    A->zero_bytes = off;
    A->is_root = base ? (int*)(base + off) : nullptr;
    off = (off + sizeof(int) * (size_t)n + 255) & ~(size_t)255;
    A->rank = base ? (int64_t*)(base + off) : nullptr;
    off = (off + sizeof(int64_t) * (size_t)(n + 1) + 255) & ~(size_t)255;
    return off;
}

int ppa_cluster_workspace_bytes(int64_t n, size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    if (n < 0 || n > 0x7fffffffLL) return set_error(PPA_EINVAL, "bad point count");
    ClusterArgs A{};
    *bytes = cluster_layout(n, nullptr, &A);
    return PPA_OK;
}

int ppa_cluster(const int64_t* offsets, const int32_t* point_idx, int64_t n, int64_t capacity,
                int32_t flags, void* ws, size_t ws_bytes, int32_t* labels, int32_t* cluster_idx,
                int32_t* sizes, int64_t* n_clusters_dev, hipStream_t stream)
{
    if (n < 0 || n > 0x7fffffffLL || capacity < 0) return set_error(PPA_EINVAL, "bad size");
    if (!offsets) return set_error(PPA_EINVAL, "offsets pointer is NULL");
    if (!point_idx && capacity > 0) return set_error(PPA_EINVAL, "point_idx pointer is NULL");
    if (!labels && n > 0) return set_error(PPA_EINVAL, "labels pointer is NULL");
    if (flags & ~PPA_CLUSTER_SYMMETRIC) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    ClusterArgs A{};
    const size_t need = cluster_layout(n, nullptr, &A);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, ws_bytes);
    cluster_layout(n, ws, &A);
    A.offsets = offsets;
    A.idx = point_idx;
    A.n = n;
    A.capacity = capacity;
    A.labels = labels;
    A.cluster_idx = cluster_idx;
    A.sizes = sizes;
    A.n_clusters = n_clusters_dev;
    A.symmetric = (flags & PPA_CLUSTER_SYMMETRIC) ? 1 : 0;
    ProfileEvents pe = take_profile_events();
    record(pe.ev[2], stream);
    launch_cluster(A, stream);
    record(pe.ev[3], stream);
    return hip_check(hipGetLastError(), "kernel launch");
}

static size_t knn_list_layout(int64_t nq, int32_t k, void* base_v, KnnListArgs* A,
                              unsigned long long** flags, int** ticket, size_t* zero_bytes)
{
    char* base = (char*)base_v;
    size_t off = 256;  // header: status word at 0, scan ticket at 64
    A->status = (unsigned*)base;
    *ticket = base ? (int*)(base + 64) : nullptr;
    *flags = base ? (unsigned long long*)(base + off) : nullptr;
    off = (off + sizeof(unsigned long long) * scan_flag_count(nq) + 256 + 255) & ~(size_t)255;
    *zero_bytes = off;
    A->row_len = base ? (int32_t*)(base + off) : nullptr;
    off = (off + sizeof(int32_t) * (size_t)nq + 255) & ~(size_t)255;
    A->out_idx = base ? (int32_t*)(base + off) : nullptr;
    off = (off + sizeof(int32_t) * (size_t)nq * (size_t)k + 255) & ~(size_t)255;
    A->out_dist = base ? (float*)(base + off) : nullptr;
    off = (off + sizeof(float) * (size_t)nq * (size_t)k + 255) & ~(size_t)255;
    return off;
}

int ppa_knn_from_nlist_workspace_bytes(int64_t nq, int32_t k, size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    if (nq < 0 || nq > 0x7fffffffLL) return set_error(PPA_EINVAL, "bad row count");
    if (k < 1 || k > 64) return set_error(PPA_EINVAL, "k must be in [1, 64]");
    KnnListArgs A{};
    unsigned long long* flags = nullptr;
    int* ticket = nullptr;
    size_t zb = 0;
    *bytes = knn_list_layout(nq, k, nullptr, &A, &flags, &ticket, &zb);
    return PPA_OK;
}

int ppa_knn_from_nlist(const int64_t* offsets, const int32_t* point_idx, const float* dist,
                       int64_t nq, int64_t capacity, int32_t k, int32_t flags, void* ws,
                       size_t ws_bytes, int64_t* out_offsets, int32_t* out_counts,
                       int32_t* out_idx, float* out_dist, int64_t* n_pairs_dev,
                       hipStream_t stream)
{
    size_t need = 0;
    int rc = ppa_knn_from_nlist_workspace_bytes(nq, k, &need);
    if (rc) return rc;
    if (capacity < 0) return set_error(PPA_EINVAL, "negative capacity");
    if (!offsets) return set_error(PPA_EINVAL, "offsets pointer is NULL");
    if ((!point_idx || !dist) && capacity > 0)
        return set_error(PPA_EINVAL, "point_idx and dist of the list are required");
    if (!out_offsets || !n_pairs_dev || (!out_idx && nq > 0))
        return set_error(PPA_EINVAL, "out_offsets, out_idx and n_pairs_dev are required");
    if (flags != 0) return set_error(PPA_EINVAL, "unknown flags 0x%x", flags);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return set_error(PPA_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                         need, ws_bytes);
    KnnListArgs A{};
    unsigned long long* scan_flags = nullptr;
    int* ticket = nullptr;
    size_t zb = 0;
    knn_list_layout(nq, k, ws, &A, &scan_flags, &ticket, &zb);
    if (out_counts) A.row_len = out_counts;
    A.offsets = offsets;
    A.idx = point_idx;
    A.dist = dist;
    A.nq = nq;
    A.capacity = capacity;
    A.k = k;
    launch_zero_words((unsigned*)ws, (long long)(zb / 4), stream);
    ProfileEvents pe = take_profile_events();
    record(pe.ev[2], stream);
    launch_knn_list(A, knn_list_workgroups(nq), stream);
    record(pe.ev[3], stream);
    launch_scan_i64_total(A.row_len, out_offsets, nq, scan_flags, ticket,
                          (unsigned long long*)n_pairs_dev, stream);
    launch_knn_pack(nq, k, A.row_len, out_offsets, A.out_idx, A.out_dist, out_idx, out_dist,
                    stream);
    return hip_check(hipGetLastError(), "kernel launch");
}

int ppa_pmft_xyt_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t nbx,
                                 int32_t nby, int32_t nbt, float x_max, float y_max, float r_max,
                                 size_t* bytes)
{
    const Pmft3Call c{kPmftXyt, box, nullptr, nullptr, n, nullptr, nullptr, nq,
                      {nbx, nby, nbt}, {x_max, y_max, 1.f}, r_max};
    return pmft3_workspace(c, bytes);
}

int ppa_pmft_xyt(const ppa_box* box, const float* pts, const float* angles, int64_t n,
                 const float* qpts, const float* qangles, int64_t nq, int32_t nbx, int32_t nby,
                 int32_t nbt, float x_max, float y_max, float r_max, int32_t exclude_ii,
                 int32_t flags, void* ws, size_t ws_bytes, uint32_t* counts, hipStream_t stream)
{
    const Pmft3Call c{kPmftXyt, box, pts, angles, n, qpts, qpts ? qangles : angles, nq,
                      {nbx, nby, nbt}, {x_max, y_max, 1.f}, r_max};
    return run_pmft3(c, exclude_ii, flags, ws, ws_bytes, counts, stream);
}

int ppa_pmft_xyz_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t nbx,
                                 int32_t nby, int32_t nbz, float x_max, float y_max, float z_max,
                                 float r_max, size_t* bytes)
{
    const Pmft3Call c{kPmftXyz, box, nullptr, nullptr, n, nullptr, nullptr, nq,
                      {nbx, nby, nbz}, {x_max, y_max, z_max}, r_max};
    return pmft3_workspace(c, bytes);
}

int ppa_pmft_xyz(const ppa_box* box, const float* pts, int64_t n, const float* qpts,
                 const float* qquats, int64_t nq, int32_t nbx, int32_t nby, int32_t nbz,
                 float x_max, float y_max, float z_max, float r_max, int32_t exclude_ii,
                 int32_t flags, void* ws, size_t ws_bytes, uint32_t* counts, hipStream_t stream)
{
    const Pmft3Call c{kPmftXyz, box, pts, nullptr, n, qpts, qquats, nq,
                      {nbx, nby, nbz}, {x_max, y_max, z_max}, r_max};
    return run_pmft3(c, exclude_ii, flags, ws, ws_bytes, counts, stream);
}

int ppa_smooth_rdf_workspace_bytes(const ppa_box* box, int64_t n, int32_t bins, float r_max,
                                   float sigma, size_t* bytes)
{
    if (!bytes) return set_error(PPA_EINVAL, "bytes is NULL");
    if (n < 0) return set_error(PPA_EINVAL, "negative point count");
    BoxPrep bp;
    int rc = prepare_box(box, &bp);
    if (rc) return rc;
    SmoothPlan P, Pb;
    if ((rc = smooth_plan(bp, n, bins, r_max, sigma, false, &P))) return rc;
    if ((rc = smooth_plan(bp, n, bins, r_max, sigma, true, &Pb))) return rc;
    Workspace W{};
    double* partial = nullptr;
    double* level2 = nullptr;
    const size_t a = smooth_layout(P, n, bins, nullptr, &W, &partial, &level2);
    const size_t b = smooth_layout(Pb, n, bins, nullptr, &W, &partial, &level2);
    *bytes = a > b ? a : b;
    return PPA_OK;
}

int ppa_smooth_rdf_fwd(const ppa_box* box, const float* pts, int64_t n, int32_t bins, float r_max,
                       float sigma, int32_t flags, void* ws, size_t ws_bytes, double* h,
                       hipStream_t stream)
{
    return run_smooth(box, pts, n, bins, r_max, sigma, nullptr, flags, ws, ws_bytes, h, nullptr,
                      stream);
}

int ppa_smooth_rdf_bwd(const ppa_box* box, const float* pts, int64_t n, int32_t bins, float r_max,
                       float sigma, const double* grad_h, int32_t flags, void* ws,
                       size_t ws_bytes, float* grad_pts, hipStream_t stream)
{
    if (!grad_pts) return set_error(PPA_EINVAL, "grad_pts is NULL");
    return run_smooth(box, pts, n, bins, r_max, sigma, grad_h, flags, ws, ws_bytes, nullptr,
                      grad_pts, stream);
}

int ppa_sync_status(const void* ws, hipStream_t stream)
{
    int rc;
    if (!ws) {  // the static scratch of ppa_rdf_static on the current device
        void* p = nullptr;
        if ((rc = static_scratch(&p, false))) return rc;
        ws = p;
    }
    rc = hip_check(hipStreamSynchronize(stream), "stream synchronize");
    if (rc) return rc;
    unsigned st = 0;
    rc = hip_check(hipMemcpy(&st, ws, sizeof(st), hipMemcpyDeviceToHost), "read status");
    if (rc) return rc;
    if (st & kStatusNonFinite) return set_error(PPA_ENONFINITE, "input has a non-finite coordinate");
    if (st & kStatusCapacity) return set_error(PPA_ECAPACITY, "more pairs than the output capacity");
    if (st & kStatusBadList)
        return set_error(PPA_EINVAL, "a NeighborList offset or point index is out of range");
    if (st & kStatusTies)
        return set_error(PPA_ERANGE,
                         "more than 256 entries of a NeighborList row tie at the k-th distance");
    if (st & kStatusRange)
        return set_error(PPA_ERANGE,
                         "a k-nearest row needs a neighbour at or beyond half the smallest "
                         "perpendicular box width");
    return PPA_OK;
}

int ppa_profile_next(hipEvent_t count_start, hipEvent_t count_stop, hipEvent_t fill_start,
                     hipEvent_t fill_stop)
{
    g_prof = ProfileEvents{{count_start, count_stop, fill_start, fill_stop}};
    return PPA_OK;
}

const char* ppa_last_error(void) { return g_err; }

const char* ppa_version(void) { return "ppa 0.1.0 (gfx950)"; }

}  // extern "C"
