/*
 * ppa: periodic pair analysis on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libppa.so: neighbor queries in periodic triclinic boxes, the
 * per-bond histograms built from them (RDF, 2D PMFT, the PMFT over three
 * pair coordinates, the spatial correlation function) and analyses of a
 * NeighborList (Steinhardt order parameters, clusters), after the neighbor
 * machinery and analysis modules of the freud paper (arXiv:1906.06317,
 * sections "Implementation" and "Features"); plus batched analysis of many
 * frames and a Gaussian-smoothed RDF with its adjoint.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Box.  ppa_box holds the edge lengths L = (Lx, Ly, Lz), the tilt factors
 *   (xy, xz, yz) and the dimension (2 or 3).  Its lattice vectors are
 *   a1 = (Lx, 0, 0), a2 = (xy Ly, Ly, 0), a3 = (xz Lz, yz Lz, Lz), and the box
 *   is centred on the origin.  The paper builds a box from three edge lengths
 *   or a 3x3 matrix ("Implementation"); ppa_box_from_matrix accepts the
 *   latter in upper-triangular form.  In 2D, Lz, xz, yz and z are ignored.
 * Points.  Positions are N x 3 float32, row-major (x, y, z), the paper's
 *   "N x 3 array".  Points may lie outside the box; they are folded in.
 * Minimum image.  Every query needs r_max < min_k(d_k)/2, where d_k is the
 *   perpendicular width of the box across face k.  Then the pair vector is
 *   the unique periodic image shorter than r_max.
 * Memory.  Every pointer argument named *_dev or documented as "device" is
 *   device memory owned by the caller; the library allocates nothing on the
 *   device.  The scratch space each call needs is the caller's workspace
 *   `ws` of `ws_bytes` bytes (size from ppa_workspace_bytes, 256-byte
 *   aligned).  Inputs must stay valid until the stream work is done.
 * Streams.  All compute calls are asynchronous on the given hipStream_t and
 *   return after enqueueing.  Errors found on the host are returned at
 *   once; errors found on the device (non-finite input, output capacity)
 *   are recorded in a status word inside `ws` and returned by
 *   ppa_sync_status, which waits for the stream.  The status word sits at
 *   the start of every workspace.
 * Histograms are accumulated into (+=), as the paper's reset=False
 *   accumulation over frames ("Implementation"); zero them to start over.
 * Return value: PPA_OK or a negative PPA_E* code; ppa_last_error() gives a
 *   message for the calling thread's last failure.
 */
#ifndef PPA_H
#define PPA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double L[3];    /* Lx, Ly, Lz (> 0, finite) */
    double tilt[3]; /* xy, xz, yz (finite) */
    int32_t dim;    /* 2 or 3 */
} ppa_box;

enum {
    PPA_OK = 0,
    PPA_EINVAL = -1,     /* null pointer, negative size, bad bins/k/flags, r_max <= r_min */
    PPA_EBOX = -2,       /* non-finite or non-positive box, or matrix not upper triangular */
    PPA_ERANGE = -3,     /* cutoff at or beyond half the smallest perpendicular width */
    PPA_EWORKSPACE = -4, /* ws null, misaligned or smaller than ppa_workspace_bytes */
    PPA_EDEVICE = -5,    /* a HIP call failed */
    PPA_ECAPACITY = -6,  /* more pairs than the output capacity (device status) */
    PPA_ENONFINITE = -7  /* a NaN or infinite coordinate (device status) */
};

/* Workspace flag: the call writes a NeighborList (adds room for the row
 * counts and the scan of the row offsets). */
#define PPA_WS_NLIST 1

/* Query flag (ppa_query_ball, ppa_rdf with a list): each row of the
 * NeighborList ordered by neighbour index j, distances moved with their
 * indices (the paper's promise that the Python API may sort the resulting
 * neighbours, "Implementation").  Without it a row is in the fixed stencil
 * order described at ppa_query_ball.  Rows beyond an exceeded capacity are
 * left as written. */
#define PPA_SORT_ROWS 2

/* Box from a 3x3 matrix whose columns are the lattice vectors (row-major
 * m[r*3+c]).  The matrix must be upper triangular with a positive diagonal;
 * a general matrix must be rotated into that form by the caller. */
int ppa_box_from_matrix(const double m[9], int32_t dim, ppa_box* out);

/* Perpendicular widths d_k of the box (host only, no device work). */
int ppa_box_widths(const ppa_box* box, double widths[3]);

/* Workspace bytes for a query on n points (and nq separate query points,
 * 0 when the points query themselves) with cutoff r_cut.  flags is
 * PPA_WS_NLIST for calls that write a NeighborList, else 0.  Host only.
 * Returns PPA_ERANGE for an over-long cutoff. */
int ppa_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, float r_cut, int32_t flags,
                        size_t* bytes);

/* Ball query: the NeighborList of all (i, j) with |p_j - q_i| < r_max
 * (minimum image), excluding i == j when exclude_ii is set (the paper's
 * query API with an r_max query argument and exclude_ii, "Implementation"
 * and the common-neighbor example; the NeighborList of "General
 * Utilities").
 *   pts [n x 3] device; qpts [nq x 3] device, or NULL to query pts with
 *     themselves (then nq must equal n).
 *   flags: 0 or PPA_SORT_ROWS.
 *   offsets [nq + 1] int64 device: CSR row pointer, rows in query order
 *     (the paper's promise of sorted query order); offsets[nq] = pairs.
 *   counts [nq] int32 device or NULL: row lengths.
 *   point_idx [capacity] int32 device: neighbour point index j per pair.
 *   dist [capacity] float32 device or NULL: |p_j - q_i| per pair.
 *   n_pairs_dev: int64 device, receives the pair count (also when it
 *     exceeds capacity, in which case the status is PPA_ECAPACITY and
 *     point_idx/dist hold an incomplete list).
 * Within a row, pairs are in a fixed order for a given input (stencil cell
 * by stencil cell, then by point index), or by point index with
 * PPA_SORT_ROWS; the output is deterministic.
 * Two passes: row lengths, a prefix scan into offsets, then the fill. */
int ppa_query_ball(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
                   float r_max, int32_t exclude_ii, int32_t flags, void* ws, size_t ws_bytes,
                   int64_t* offsets, int32_t* counts, int32_t* point_idx, float* dist,
                   int64_t capacity, int64_t* n_pairs_dev, hipStream_t stream);

/* RDF pair histogram: counts[b] += number of ball pairs with
 * r_min + b dr <= r < r_min + (b+1) dr, dr = (r_max - r_min)/bins (the
 * density module's RDF configured by bins, r_max, r_min, "Analysis
 * Modules" and the LAMMPS example).  Pairs are the ball pairs of
 * ppa_query_ball with cutoff r_max.  When offsets is non-NULL the same
 * pass also writes the NeighborList exactly as ppa_query_ball does
 * (neighbours found once, used twice: the paper's lazy iteration of pairs
 * inside the analysis).  counts [bins] uint64 device, accumulated.
 * flags: 0 or PPA_SORT_ROWS (acts on the list only). */
int ppa_rdf(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
            int32_t bins, float r_min, float r_max, int32_t exclude_ii, int32_t flags, void* ws,
            size_t ws_bytes, uint64_t* counts_hist, int64_t* offsets, int32_t* counts,
            int32_t* point_idx, float* dist, int64_t capacity, int64_t* n_pairs_dev,
            hipStream_t stream);

/* ppa_rdf for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same call without a workspace argument.  Its scratch is a static device
 * array of the library, 64 MiB per device, held from the first call on a
 * device until the process ends; the call allocates nothing and calls no
 * allocating routine.  Arguments, outputs and results are those of ppa_rdf.
 * A call whose workspace (ppa_workspace_bytes with PPA_WS_NLIST when
 * offsets is non-NULL) would exceed 64 MiB returns PPA_EWORKSPACE before
 * any device work (about 1.4 million points for the self-query ball list).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (different streams or threads) race and must be serialised by
 * the caller.  The device status of the last call is read with
 * ppa_sync_status(NULL, stream) on the same device. */
int ppa_rdf_static(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
                   int32_t bins, float r_min, float r_max, int32_t exclude_ii, int32_t flags,
                   uint64_t* counts_hist, int64_t* offsets, int32_t* counts, int32_t* point_idx,
                   float* dist, int64_t capacity, int64_t* n_pairs_dev, hipStream_t stream);

/* RDF histogram from a stored NeighborList's distances (the paper's reuse of
 * a NeighborList across analyses, "Implementation").  dist [*n_pairs_dev]
 * float32 device, at most `capacity` are read; counts_hist accumulated. */
int ppa_rdf_from_nlist(const float* dist, const int64_t* n_pairs_dev, int64_t capacity,
                       int32_t bins, float r_min, float r_max, uint64_t* counts_hist,
                       hipStream_t stream);

/* Workspace bytes for a k-nearest query (ppa_query_knn) on n points and nq
 * separate query points (0 when the points query themselves).  Host only.
 * Returns PPA_EINVAL for k outside [1, 64] and PPA_ERANGE for an r_guard at
 * or beyond half the smallest perpendicular width. */
int ppa_knn_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t k, float r_guard,
                            size_t* bytes);

/* k-nearest query: for every query point q_i, the k points nearest to it
 * (minimum image), excluding j == i when exclude_ii is set (the paper's
 * query API with a num_neighbors query argument, "Implementation" and the
 * Steinhardt example).  Neighbours are ordered by (r^2, j): increasing
 * distance, ties by point index.
 *   k in [1, 64].
 *   r_guard: 0 for none; otherwise only points with r < r_guard qualify and
 *     a row may hold fewer than k (r_guard must be below half the smallest
 *     perpendicular width).
 *   pts, qpts, nq, exclude_ii: as for ppa_query_ball.
 *   flags: reserved, must be 0.
 *   offsets [nq + 1] int64 device: CSR row pointer in query order.  Without
 *     r_guard and with n - 1 >= k every row holds exactly k pairs and
 *     offsets[i] = k i.
 *   counts [nq] int32 device or NULL: row lengths.
 *   point_idx [nq * k] int32 device, dist [nq * k] float32 device or NULL:
 *     the pairs, row after row (offsets[nq] of them are written).
 *   n_pairs_dev: int64 device, receives offsets[nq].
 * Without r_guard a row must reach min(k, number of eligible points); if
 * that needs a neighbour at or beyond half the smallest perpendicular width
 * (where the minimum image stops being unique), the device status becomes
 * PPA_ERANGE and the row is incomplete. */
int ppa_query_knn(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
                  int32_t k, float r_guard, int32_t exclude_ii, int32_t flags, void* ws,
                  size_t ws_bytes, int64_t* offsets, int32_t* counts, int32_t* point_idx,
                  float* dist, int64_t* n_pairs_dev, hipStream_t stream);

/* Workspace bytes for ppa_knn_from_nlist on nq rows with this k (host only). */
int ppa_knn_from_nlist_workspace_bytes(int64_t nq, int32_t k, size_t* bytes);

/* k nearest neighbours selected from a stored NeighborList (the paper's
 * reuse of a NeighborList across analyses, "Implementation"): each row keeps
 * its min(k, row length) entries of smallest (distance, point index), in that
 * order.  For a ball list with cutoff r_max whose rows all hold at least k
 * entries this equals ppa_query_knn (nothing outside the ball is nearer);
 * in general it is the k-nearest query guarded at r_max.
 *   offsets [nq + 1] int64, point_idx [capacity] int32, dist [capacity]
 *     float32 (all device): the list; an offset outside [0, capacity] or
 *     decreasing offsets make the row empty and set PPA_EINVAL in the device
 *     status.
 *   k in [1, 64]; flags: reserved, must be 0.
 *   out_offsets [nq + 1] int64 device: CSR row pointer of the result.
 *   out_counts [nq] int32 device or NULL: row lengths.
 *   out_idx [nq * k] int32 device, out_dist [nq * k] float32 device or NULL:
 *     the selected pairs, row after row (out_offsets[nq] of them).
 *   n_pairs_dev: int64 device, receives out_offsets[nq].
 * Rows in which more than 256 entries tie at the k-th distance are left
 * empty and set PPA_ERANGE in the device status. */
int ppa_knn_from_nlist(const int64_t* offsets, const int32_t* point_idx, const float* dist,
                       int64_t nq, int64_t capacity, int32_t k, int32_t flags, void* ws,
                       size_t ws_bytes, int64_t* out_offsets, int32_t* out_counts,
                       int32_t* out_idx, float* out_dist, int64_t* n_pairs_dev,
                       hipStream_t stream);

/* Workspace bytes for ppa_pmft2d with these arguments (nq: separate query
 * points, 0 when the points query themselves).  Queries the current device
 * (its compute-unit count and LDS size set the launch) but does no device
 * work.  Same error codes as ppa_pmft2d's host checks. */
int ppa_pmft2d_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t nbx, int32_t nby,
                               float x_max, float y_max, float r_max, size_t* bytes);

/* 2D PMFT histogram (the paper's PMFT section, in 2D: positions of the
 * other particles seen from each particle's own frame).  For every ball pair
 * (i, j) with |p_j - q_i| < r_max (minimum image), excluding j == i when
 * exclude_ii is set, the bond d = p_j - q_i is rotated by -theta_i:
 *     x' =  cos(theta_i) d_x + sin(theta_i) d_y,
 *     y' = -sin(theta_i) d_x + cos(theta_i) d_y,
 * and counted in bin (ix, iy) = (floor((x' + x_max) / dx),
 * floor((y' + y_max) / dy)), dx = 2 x_max / nbx, dy = 2 y_max / nby, when
 * both lie in range.  counts[ix * nby + iy] += the count (uint32, device,
 * accumulated; it wraps past 2^32).
 *   box: dim must be 2 (PPA_EINVAL otherwise).
 *   pts [n x 3], qpts [nq x 3] or NULL, exclude_ii: as for ppa_query_ball.
 *   angles [nq] float32 device: orientation theta of each query point in
 *     radians (of pts when qpts is NULL).
 *   nbx, nby >= 1; x_max, y_max > 0; r_max below half the smallest width.
 *   flags: reserved, must be 0.
 * The PMFT itself is minus the log of the normalised counts (host side). */
int ppa_pmft2d(const ppa_box* box, const float* pts, int64_t n, const float* qpts,
               const float* angles, int64_t nq, int32_t nbx, int32_t nby, float x_max,
               float y_max, float r_max, int32_t exclude_ii, int32_t flags, void* ws,
               size_t ws_bytes, uint32_t* counts, hipStream_t stream);

/* Workspace bytes for ppa_pmft_xyt / ppa_pmft_xyz with these arguments (nq:
 * separate query points, 0 when the points query themselves): the cell
 * lists of the points (and queries).  No device work.  Same error codes as
 * the calls' host checks. */
int ppa_pmft_xyt_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t nbx,
                                 int32_t nby, int32_t nbt, float x_max, float y_max, float r_max,
                                 size_t* bytes);
int ppa_pmft_xyz_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t nbx,
                                 int32_t nby, int32_t nbz, float x_max, float y_max, float z_max,
                                 float r_max, size_t* bytes);

/* 2D PMFT with the relative orientation (the paper's PMFT section: in 2D
 * the full PMFT is three-dimensional, since the second particle's
 * orientation relative to the first is a coordinate too).  For every ball
 * pair (i, j) as in ppa_pmft2d, (x', y') is the bond in the query's frame
 * exactly as there, and t = (theta_j - theta_i) mod 2 pi in [0, 2 pi).  The
 * bond is counted in bin (ix, iy, it), it = floor(t nbt / (2 pi)), when ix
 * and iy lie in range (t always does):
 *     counts[(ix * nby + iy) * nbt + it] += the count (uint32, device,
 *     accumulated; it wraps past 2^32).
 *   box: dim must be 2 (PPA_EINVAL otherwise).
 *   pts [n x 3], qpts [nq x 3] or NULL, exclude_ii: as for ppa_query_ball.
 *   angles [n] float32 device: orientation of every point in radians.
 *   qangles [nq] float32 device: orientation of every query point (ignored,
 *     and may be NULL, when qpts is NULL: the points' angles are used).
 *   nbx, nby, nbt >= 1 (product below 2^31); x_max, y_max > 0; r_max below
 *     half the smallest width.
 *   flags: reserved, must be 0.
 * Non-finite angles set PPA_ENONFINITE in the device status.  Bonds go to
 * the histogram with global atomics: it may be of any size. */
int ppa_pmft_xyt(const ppa_box* box, const float* pts, const float* angles, int64_t n,
                 const float* qpts, const float* qangles, int64_t nq, int32_t nbx, int32_t nby,
                 int32_t nbt, float x_max, float y_max, float r_max, int32_t exclude_ii,
                 int32_t flags, void* ws, size_t ws_bytes, uint32_t* counts, hipStream_t stream);

/* 3D PMFT over the bond's position in the query particle's frame (the
 * paper's PMFT section: the translational degrees of freedom of a 3D
 * PMFT).  For every ball pair (i, j), |p_j - q_i| < r_max (minimum image),
 * excluding j == i when exclude_ii is set, the bond d = p_j - q_i is turned
 * into the query's frame, d' = R(q_i)^T d, with R the rotation matrix of the
 * query's unit quaternion q_i = (w, x, y, z), and counted in bin
 * (ix, iy, iz) = floor((d' + max) nb / (2 max)) per axis when all three lie
 * in range:
 *     counts[(ix * nby + iy) * nbz + iz] += the count (uint32, device,
 *     accumulated; it wraps past 2^32).
 *   box: dim must be 3 (PPA_EINVAL otherwise).
 *   pts [n x 3], qpts [nq x 3] or NULL, exclude_ii: as for ppa_query_ball.
 *   qquats [nq x 4] float32 device, 16-byte aligned: orientation of every
 *     query point (of pts when qpts is NULL) as a quaternion (w, x, y, z);
 *     each is normalised first.
 *   nbx, nby, nbz >= 1 (product below 2^31); x_max, y_max, z_max > 0;
 *     r_max below half the smallest perpendicular width.
 *   flags: reserved, must be 0.
 * A zero or non-finite quaternion sets PPA_ENONFINITE in the device
 * status.  Bonds go to the histogram with global atomics. */
int ppa_pmft_xyz(const ppa_box* box, const float* pts, int64_t n, const float* qpts,
                 const float* qquats, int64_t nq, int32_t nbx, int32_t nby, int32_t nbz,
                 float x_max, float y_max, float z_max, float r_max, int32_t exclude_ii,
                 int32_t flags, void* ws, size_t ws_bytes, uint32_t* counts, hipStream_t stream);

/* Workspace bytes for ppa_correlation with these arguments (nq: separate
 * query points, 0 when the points query themselves).  Queries the current
 * device (its compute units and LDS set the launch) but does no device
 * work.  Same error codes as ppa_correlation's host checks. */
int ppa_correlation_workspace_bytes(const ppa_box* box, int64_t n, int64_t nq, int32_t bins,
                                    float r_min, float r_max, size_t* bytes);

/* Spatial correlation function of per-particle values (the density
 * module's correlation functions of arbitrary quantities, "Analysis
 * Modules"; the paper's overview figure shows that of the hexatic order
 * parameter).  For every ball pair (i, j), |p_j - q_i| < r_max (minimum
 * image), excluding j == i when exclude_ii is set, with r_min <= r and bin
 * b = floor((r - r_min) / dr), dr = (r_max - r_min) / bins:
 *     sums[2b] + i sums[2b + 1] += conj(f_i) g_j,   counts[b] += 1,
 * where g_j = values[j] and f_i = qvalues[i] are complex.  The correlation
 * is C_b = (sums[2b] + i sums[2b + 1]) / counts[b] (ppa_correlation_finalize).  Each term
 * is formed in float64 from the float32 values (exact products, one
 * rounding); bins' sums are float64, accumulated per workgroup in LDS and
 * then summed in a fixed order.
 *   pts [n x 3], qpts [nq x 3] or NULL, exclude_ii: as for ppa_query_ball.
 *   values [n x 2] float32 device, 8-byte aligned: (re, im) per point (a
 *     real quantity has im = 0).
 *   qvalues [nq x 2] float32 device, 8-byte aligned: values of the query
 *     points; may be NULL when qpts is NULL (the points' values are used).
 *   bins in [1, 4096]; 0 <= r_min < r_max, r_max below half the smallest
 *     perpendicular width.
 *   flags: reserved, must be 0.
 *   sums [bins x 2] float64 device, counts [bins] uint64 device: accumulated.
 * Non-finite values set PPA_ENONFINITE in the device status. */
int ppa_correlation(const ppa_box* box, const float* pts, const float* values, int64_t n,
                    const float* qpts, const float* qvalues, int64_t nq, int32_t bins,
                    float r_min, float r_max, int32_t exclude_ii, int32_t flags, void* ws,
                    size_t ws_bytes, double* sums, uint64_t* counts, hipStream_t stream);

/* Workspace bytes for ppa_steinhardt with degree l (host only). */
int ppa_steinhardt_workspace_bytes(int32_t l, int32_t flags, size_t* bytes);

/* Steinhardt bond-orientational order parameters of the rows of a
 * NeighborList (the paper's order-parameter features; its example computes
 * Q6 on the 12-nearest-neighbour list, definitions after Steinhardt, Nelson
 * and Ronchetti).  For query i with bonds d_ij = p_j - q_i over its row
 * (minimum image; bonds of length 0 are skipped, N_b counts the others):
 *     q_lm(i) = (1 / N_b) sum_j Y_lm(d_ij),
 *     ql[i] = Q_l(i) = sqrt(4 pi / (2l + 1) sum_m |q_lm|^2),
 *     wl[i] = sum_{m1+m2+m3=0} (l l l; m1 m2 m3) q_lm1 q_lm2 q_lm3
 *             / (sum_m |q_lm|^2)^(3/2)      (the normalised W-hat),
 * with Y_lm the orthonormal spherical harmonics (polar angle from +z).
 * Rows without bonds give 0.  Computed in float64.
 *   pts [n x 3], qpts [nq x 3] or NULL (the points are the queries):
 *     float32 device, the positions the list was built from.
 *   offsets [nq + 1] int64 device, point_idx [capacity] int32 device: the
 *     NeighborList (any CSR list, e.g. from ppa_query_knn or
 *     ppa_query_ball).  An offset outside [0, capacity], decreasing offsets
 *     or an index outside [0, n) is skipped and sets the device status to
 *     PPA_EINVAL.  Bonds are taken as the image in the centred box cell, the
 *     minimum image for every bond shorter than half the smallest width.
 *   l in [0, 12]; flags: reserved, must be 0.
 *   ws: ppa_steinhardt_workspace_bytes(l) bytes (status and 3j table).
 *   ql [nq] float64 device; wl [nq] float64 device or NULL (Q_l only). */
int ppa_steinhardt(const ppa_box* box, const float* pts, int64_t n, const float* qpts, int64_t nq,
                   const int64_t* offsets, const int32_t* point_idx, int64_t capacity, int32_t l,
                   int32_t flags, void* ws, size_t ws_bytes, double* ql, double* wl,
                   hipStream_t stream);

/* Cluster flag: the list is symmetric (j in row i exactly when i is in row
 * j, as in a ball query of the points with themselves).  The hooking rounds
 * then sample two bonds per row and the closing union pass skips the points
 * of the largest sampled component.  The labels are the same; with a list
 * that is not symmetric they may be wrong. */
#define PPA_CLUSTER_SYMMETRIC 1

/* Workspace bytes for ppa_cluster on n points (host only). */
int ppa_cluster_workspace_bytes(int64_t n, size_t* bytes);

/* Clusters (the cluster module, "Analysis Modules": membership defined by
 * neighbour bonds): the connected components of the undirected graph on the
 * n points whose edges are the pairs (i, point_idx[e]) of every row i of a
 * NeighborList over these points (a bond listed in one direction only, as
 * in a k-nearest list, still joins both points).
 *   offsets [n + 1] int64 device, point_idx [capacity] int32 device: the
 *     list, row i belonging to point i (e.g. ppa_query_ball of the points
 *     with themselves).  An offset outside [0, capacity], decreasing
 *     offsets or an index outside [0, n) is skipped and sets the device
 *     status to PPA_EINVAL.
 *   flags: 0 or PPA_CLUSTER_SYMMETRIC.
 *   labels [n] int32 device: the smallest point index of each point's
 *     component (deterministic, independent of scheduling).
 *   cluster_idx [n] int32 device or NULL: components numbered 0, 1, ... in
 *     order of their smallest point index.
 *   sizes [n] int32 device or NULL: sizes[c] = points of component c for
 *     c < number of components (the rest 0).
 *   n_clusters_dev int64 device or NULL: the number of components.
 * Lock-free union-find on the device (compare-and-swap linking of the
 * larger root under the smaller, path halving); no host synchronisation. */
int ppa_cluster(const int64_t* offsets, const int32_t* point_idx, int64_t n, int64_t capacity,
                int32_t flags, void* ws, size_t ws_bytes, int32_t* labels, int32_t* cluster_idx,
                int32_t* sizes, int64_t* n_clusters_dev, hipStream_t stream);

/* Gaussian-smoothed RDF (an extension beyond the paper: a differentiable
 * form of the density module's RDF histogram).  With bins of width
 * dr = r_max / bins centred at c_b = (b + 1/2) dr and
 * phi(u) = exp(-u^2 / (2 sigma^2)) / (sigma sqrt(2 pi)):
 *     h_b += dr * sum over ordered pairs (i, j), i != j, r_ij < r_max + 8 sigma
 *            (minimum image), of phi(c_b - r_ij), for |c_b - r_ij| <= 8 sigma.
 * The points query themselves; g_b = h_b / (N rho dV_b) as for the RDF.
 *   bins in [1, 4096]; r_max + 8 sigma below half the smallest width.
 *   h [bins] float64 device, accumulated.
 *   flags: reserved, must be 0.
 * Pair vectors enter the Gaussian in float64; its terms are float32 and are
 * summed in float64. */
int ppa_smooth_rdf_fwd(const ppa_box* box, const float* pts, int64_t n, int32_t bins, float r_max,
                       float sigma, int32_t flags, void* ws, size_t ws_bytes, double* h,
                       hipStream_t stream);

/* Adjoint of ppa_smooth_rdf_fwd: given grad_h[b] = dL/dh_b (float64
 * device), writes grad_pts[k] = dL/dp_k (float32 [n x 3] device):
 *     dL/dp_k = sum over j != k of 2 A(r_kj) (p_k - p_j) / r_kj,
 *     A(r) = sum_b grad_h[b] dr (c_b - r) / sigma^2 phi(c_b - r)
 * over the same window; pairs at r = 0 add nothing.  The pairs are found
 * again (nothing is kept from the forward); each row is summed in float64
 * by the one wavefront that owns it. */
int ppa_smooth_rdf_bwd(const ppa_box* box, const float* pts, int64_t n, int32_t bins, float r_max,
                       float sigma, const double* grad_h, int32_t flags, void* ws,
                       size_t ws_bytes, float* grad_pts, hipStream_t stream);

/* Workspace bytes for ppa_smooth_rdf_fwd and ppa_smooth_rdf_bwd (the larger
 * of the two).  Queries the current device, no device work. */
int ppa_smooth_rdf_workspace_bytes(const ppa_box* box, int64_t n, int32_t bins, float r_max,
                                   float sigma, size_t* bytes);

/* ---- Normalisation of accumulated histograms (float64, device) ------------
 * The paper reads the RDF as g(r) = exp(-beta F(r)), the potential of mean
 * force in units of kT, and defines the PMFT as minus the logarithm of the
 * histogram of neighbour positions in each particle's own frame ("PMFT");
 * histograms accumulate over frames before they are averaged
 * ("Implementation", reset=False).  These calls divide each bin by the count
 * an ideal gas of the same density would give it, summed over the frames:
 *     D = sum_f N_q,f * N_p,f / V_f   (V: volume in 3D, area Lx Ly in 2D),
 * from per-frame host arrays boxes[n_frames], n_points[n_frames] (N_p, the
 * points searched) and n_query[n_frames] (N_q, the query points; equal to
 * N_p for a self-query).  D is formed on the host in float64 (PPA_EINVAL
 * when it is 0, or a count is negative; PPA_EBOX for a bad box); one kernel
 * on `stream` then writes every bin in float64.  Outputs are device arrays
 * owned by the caller, overwritten (not accumulated).  -ln of an empty bin
 * is +inf.  The additive constant of the PMF and PMFT (the paper defines them
 * up to a constant) is fixed by this normalisation: an ideal gas gives
 * g = pcf = 1 up to the (N-1)/N of a self-query. */

/* RDF: g[b] = counts[b] / (D dV_b), dV_b the volume of the shell between the
 * bin's edges e_b = r_min + b (r_max - r_min) / bins (4/3 pi (e1^3 - e0^3) in
 * 3D, pi (e1^2 - e0^2) in 2D; the dimension is boxes[0].dim and every frame
 * must share it); pmf[b] = -ln g[b] when pmf is non-NULL.
 *   counts [bins] uint64 device; g [bins] float64 device; pmf [bins] float64
 *   device or NULL. */
int ppa_rdf_normalize(const uint64_t* counts, int32_t bins, double r_min, double r_max,
                      int32_t n_frames, const ppa_box* boxes, const int64_t* n_points,
                      const int64_t* n_query, double* g, double* pmf, hipStream_t stream);

/* The RDF's per-bin factor alone: scale[b] = 1 / (D dV_b), so g = h * scale
 * for any numerator h (the smoothed RDF's float64 h, whose gradient then
 * passes through the same factor).  scale [bins] float64 device. */
int ppa_rdf_bin_scale(int32_t bins, double r_min, double r_max, int32_t n_frames,
                      const ppa_box* boxes, const int64_t* n_points, const int64_t* n_query,
                      double* scale, hipStream_t stream);

/* 2D PMFT (ppa_pmft2d counts [nbx][nby], bins of dx = 2 x_max / nbx by
 * dy = 2 y_max / nby): pcf = counts / (D dx dy), pmft = -ln pcf (NULL to
 * skip).  2D boxes only.  counts uint32 device; pcf, pmft float64 device. */
int ppa_pmft2d_normalize(const uint32_t* counts, int32_t nbx, int32_t nby, double x_max,
                         double y_max, int32_t n_frames, const ppa_box* boxes,
                         const int64_t* n_points, const int64_t* n_query, double* pcf,
                         double* pmft, hipStream_t stream);

/* PMFT XYT (ppa_pmft_xyt counts [nbx][nby][nbt]): the orientation bin is
 * weighted by its share 1 / nbt of the full turn, pcf = counts /
 * (D dx dy / nbt), so an ideal gas gives 1.  2D boxes only. */
int ppa_pmft_xyt_normalize(const uint32_t* counts, int32_t nbx, int32_t nby, int32_t nbt,
                           double x_max, double y_max, int32_t n_frames, const ppa_box* boxes,
                           const int64_t* n_points, const int64_t* n_query, double* pcf,
                           double* pmft, hipStream_t stream);

/* PMFT XYZ (ppa_pmft_xyz counts [nbx][nby][nbz]): pcf = counts /
 * (D dx dy dz), dz = 2 z_max / nbz.  3D boxes only. */
int ppa_pmft_xyz_normalize(const uint32_t* counts, int32_t nbx, int32_t nby, int32_t nbz,
                           double x_max, double y_max, double z_max, int32_t n_frames,
                           const ppa_box* boxes, const int64_t* n_points, const int64_t* n_query,
                           double* pcf, double* pmft, hipStream_t stream);

/* Correlation function from ppa_correlation's accumulated sums and counts
 * (the density module's correlation of arbitrary quantities, "Analysis
 * Modules"): corr[2b] + i corr[2b+1] = (sums[2b] + i sums[2b+1]) / counts[b],
 * 0 for an empty bin.  sums, corr [bins x 2] float64 device; counts [bins]
 * uint64 device. */
int ppa_correlation_finalize(const double* sums, const uint64_t* counts, int32_t bins,
                             double* corr, hipStream_t stream);

/* ---- Batched analysis (an extension beyond the paper) --------------------
 * Many frames (a trajectory, or many systems of uneven size each with its
 * own box) analysed together: for every frame the ball-query NeighborList
 * and the RDF, as ppa_rdf computes them for that frame alone, in one fixed
 * sequence of launches over one cell list holding every frame's cells.  The
 * paper accumulates an RDF over frames by calling compute once per frame
 * (reset=False); a batch does all frames at once and keeps one histogram
 * per frame. */
typedef struct ppa_batch_plan_s ppa_batch_plan;
typedef struct ppa_batch_graph_s ppa_batch_graph;

/* Plan for n_frames frames: boxes[f] (host), and the points of frame f are
 * rows frame_offsets[f] .. frame_offsets[f+1] - 1 of one [N x 3] float32
 * array (frame_offsets: host, n_frames + 1 entries, starting at 0,
 * non-decreasing, N = frame_offsets[n_frames] < 2^31).  All frames share
 * the dimension, bins, r_min, r_max and exclude_ii (each frame's points
 * query themselves).  r_max must be below half the smallest perpendicular
 * width of every frame (PPA_ERANGE names the frame).  flags: 0 or
 * PPA_SORT_ROWS (every run orders each row by frame-local neighbour index).
 * Host only; free with ppa_batch_plan_destroy. */
int ppa_batch_plan_create(int32_t n_frames, const ppa_box* boxes, const int64_t* frame_offsets,
                          int32_t bins, float r_min, float r_max, int32_t exclude_ii,
                          int32_t flags, ppa_batch_plan** out);
int ppa_batch_plan_destroy(ppa_batch_plan* plan);

/* Workspace bytes a plan needs (every launch configuration fits in it). */
int ppa_batch_workspace_bytes(const ppa_batch_plan* plan, size_t* bytes);

/* Copies the plan's frame tables into the workspace (asynchronous on the
 * stream; the plan owns the host copies).  Needed once per workspace,
 * before ppa_batch_run, ppa_batch_autotune or ppa_batch_graph_create. */
int ppa_batch_upload(ppa_batch_plan* plan, void* ws, size_t ws_bytes, hipStream_t stream);

/* One batched run in the plan's current configuration.
 *   pts [N x 3] float32 device.
 *   hist [n_frames x bins] uint64 device, accumulated: row f is frame f's RDF
 *     pair histogram (as ppa_rdf with that frame's points and box).
 *   offsets [N + 1] int64 device: one CSR over all frames' rows in point
 *     order; counts [N] int32 device or NULL.
 *   point_idx [capacity] int32: neighbour indices local to the frame (0 is
 *     the frame's first point); dist [capacity] float32 or NULL.
 *   n_pairs_dev: int64 device, total pairs (PPA_ECAPACITY when above
 *     capacity, reported by ppa_sync_status).
 * Only kernels are launched (no copies, no memsets, no allocation), so a
 * run can be captured in a HIP graph. */
int ppa_batch_run(ppa_batch_plan* plan, const float* pts, void* ws, size_t ws_bytes,
                  uint64_t* hist, int64_t* offsets, int32_t* counts, int32_t* point_idx,
                  float* dist, int64_t capacity, int64_t* n_pairs_dev, hipStream_t stream);

/* Launch configurations: index >= 0 selects one, -1 only queries.  Returns
 * the number of configurations, the current one, and its cell width
 * (cell_scale * r_max at least) and resident workgroups per CU of the pair
 * kernels (0: as many as fit).  Any pointer may be NULL. */
int ppa_batch_config(ppa_batch_plan* plan, int32_t index, int32_t* n_configs, int32_t* chosen,
                     double* cell_scale, int32_t* blocks_per_cu);

/* Block shape of configuration `index` (-1: the chosen one), which
 * ppa_batch_config does not report: home cells per work-queue item and
 * wavefronts per workgroup of the pair kernels.  Either pointer may be
 * NULL.  Host only; does not change the chosen configuration. */
int ppa_batch_config_shape(ppa_batch_plan* plan, int32_t index, int32_t* cells_per_item,
                           int32_t* waves_per_workgroup);

/* Cell grid of configuration `index` (-1: the chosen one) as the cell build
 * sees it: the cells of all frames, and how they are counted.  Frames with
 * at most 32768 cells are counted per chunk of 16384 points in LDS
 * (`chunks`: the number of such chunks over all frames); the others with
 * one global atomic per point (`global_frames`: their number).  Any pointer
 * may be NULL.  Host only. */
int ppa_batch_config_cells(ppa_batch_plan* plan, int32_t index, int32_t* cells, int32_t* chunks,
                           int32_t* global_frames);

/* Autotuner: runs every configuration (one warm-up and `reps` timed runs,
 * HIP events on the stream, which it synchronizes) and selects the fastest
 * for later runs and graphs.  The NeighborList arguments are used as
 * scratch (they hold the last trial's list); histograms go to scratch in the
 * workspace.  ms_out [n_configs] host or NULL receives the mean times. */
int ppa_batch_autotune(ppa_batch_plan* plan, const float* pts, void* ws, size_t ws_bytes,
                       int64_t* offsets, int32_t* counts, int32_t* point_idx, float* dist,
                       int64_t capacity, int64_t* n_pairs_dev, int32_t reps, hipStream_t stream,
                       float* ms_out);

/* Captures one ppa_batch_run with these arguments (the plan's current
 * configuration) into an instantiated HIP graph; ppa_batch_graph_launch
 * replays it on a stream with one launch.  The arguments must stay valid
 * for the graph's life. */
int ppa_batch_graph_create(ppa_batch_plan* plan, const float* pts, void* ws, size_t ws_bytes,
                           uint64_t* hist, int64_t* offsets, int32_t* counts, int32_t* point_idx,
                           float* dist, int64_t capacity, int64_t* n_pairs_dev,
                           ppa_batch_graph** out);
int ppa_batch_graph_launch(ppa_batch_graph* graph, hipStream_t stream);
int ppa_batch_graph_destroy(ppa_batch_graph* graph);

/* Profiling hook: the next ppa_query_ball / ppa_rdf call made by this
 * thread records, on its stream, count_start / count_stop around its
 * row-count kernel and fill_start / fill_stop around its fill kernel (the
 * kernel that writes the list and the histogram; for ppa_query_knn, the two
 * selection kernels; for ppa_pmft2d, the binning and the sum of the
 * per-workgroup histograms; for the smoothed RDF, its pair kernel and, in
 * the forward, the sum of the partial histograms), then forgets them.  Any
 * event may be NULL; the events belong to the caller.  Used to time single
 * kernels inside a longer stream of work. */
int ppa_profile_next(hipEvent_t count_start, hipEvent_t count_stop, hipEvent_t fill_start,
                     hipEvent_t fill_stop);

/* Measurement hook: launches `blocks` workgroups of 256 threads that each
 * add 1 to pseudo-random bins of an LDS histogram of 2^log2_bins 32-bit
 * counters, 8 x iters atomics per thread (log2_bins in [1, 14]), then add
 * their totals to *out_dev (uint32 device, accumulated).  Timed by the
 * caller, it gives the device's LDS atomic rate, the reference for the
 * histogram kernels' binning rates. */
int ppa_probe_lds_atomics(int32_t log2_bins, int32_t iters, int32_t blocks, uint32_t* out_dev,
                          hipStream_t stream);

/* Measurement hook: launches `blocks` workgroups of 256 threads that each
 * add 1 (32-bit atomics without return value) to pseudo-random words of
 * hist_dev[0 .. 2^log2_words - 1] (uint32 device, accumulated; the caller
 * provides 2^log2_words words), 8 x iters atomics per thread (log2_words in
 * [1, 28]).  Timed by the caller, it gives the device's global atomic rate
 * for a histogram of that size, the reference for the kernels that bin into
 * device memory. */
int ppa_probe_global_atomics(int32_t log2_words, int32_t iters, int32_t blocks,
                             uint32_t* hist_dev, hipStream_t stream);

/* Waits for the stream and returns the device status of the last call that
 * used this workspace (ws NULL: the static scratch of ppa_rdf_static on the
 * current device, PPA_EINVAL if no such call was made there) (PPA_OK, PPA_ECAPACITY, PPA_ENONFINITE, for a
 * k-nearest query PPA_ERANGE, and for ppa_steinhardt / ppa_cluster /
 * ppa_knn_from_nlist PPA_EINVAL when a NeighborList offset or index was out
 * of range, PPA_ERANGE for too many ties in ppa_knn_from_nlist). */
int ppa_sync_status(const void* ws, hipStream_t stream);

/* Message describing the calling thread's last error. */
const char* ppa_last_error(void);

/* Library version string. */
const char* ppa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PPA_H */
