/*
 * FP64 reference oracle for periodic neighbor queries, the RDF, the 2D PMFT,
 * the 2D PMFT with relative orientation and the 3D PMFT, the spatial
 * correlation function of per-particle values, and a Gaussian-smoothed RDF
 * with its gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header or constant with
 * the GPU library, and the GPU library never calls it.
 *
 * Every routine is the plain definition written out: each query point is
 * compared with every point (O(N*M) brute force), in double precision, from
 * the same FP32 input arrays converted exactly to double.  There is no cell
 * list, blocking or reordering; loops over query rows run in parallel with
 * OpenMP, each row writing only its own outputs or a thread-private
 * histogram (the paper's thread-local-storage pattern, Implementation
 * section), so results do not depend on the thread count except for the
 * rounding order of double-precision sums.
 *
 * Box convention (the paper only says "3 linearly independent basis
 * vectors", Implementation section): an upper-triangular box matrix with
 * columns a1 = (Lx,0,0), a2 = (xy*Ly, Ly, 0), a3 = (xz*Lz, yz*Lz, Lz),
 * centered at the origin.  In 2D, z, Lz, xz and yz are ignored.
 *
 * Parity status of each function is stated above it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double L[3];    /* Lx, Ly, Lz */
    double tilt[3]; /* xy, xz, yz */
    int32_t dim;    /* 2 or 3 */
} orc_box;

/* Minimum image of a displacement (General Utilities section: periodicity
 * is handled for arbitrary triclinic boxes).  Back-substitution through the
 * upper-triangular box matrix: remove whole a3's to bring z into
 * [-Lz/2, Lz/2], then whole a2's for y, then whole a1's for x.  The result
 * lies in the rectangular fundamental domain |d_k| <= L_k/2, which contains
 * every image shorter than half the smallest perpendicular box width, so any
 * image inside that radius is the one returned. */
static void minimum_image(const orc_box* b, double d[3])
{
    const double Lx = b->L[0], Ly = b->L[1], Lz = b->L[2];
    const double xy = b->tilt[0], xz = b->tilt[1], yz = b->tilt[2];
    if (b->dim == 3) {
        double nz = rint(d[2] / Lz);
        d[0] -= nz * xz * Lz;
        d[1] -= nz * yz * Lz;
        d[2] -= nz * Lz;
    } else {
        d[2] = 0.0;
    }
    double ny = rint(d[1] / Ly);
    d[0] -= ny * xy * Ly;
    d[1] -= ny * Ly;
    double nx = rint(d[0] / Lx);
    d[0] -= nx * Lx;
}

/* Exported for the pin tests (minimum image against an explicit search over
 * images).  d is n x 3, modified in place. */
void orc_minimum_image(const orc_box* b, double* d, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) minimum_image(b, d + 3 * i);
}

static inline double pair_r2(const orc_box* b, const float* pj, const float* qi, double d[3])
{
    d[0] = (double)pj[0] - (double)qi[0];
    d[1] = (double)pj[1] - (double)qi[1];
    d[2] = (b->dim == 3) ? (double)pj[2] - (double)qi[2] : 0.0;
    minimum_image(b, d);
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Ball query (query API with a distance cutoff, General Utilities and
 * Implementation sections): the set of (i, j) with i a query point, j a
 * point, not (exclude_ii and i == j), and minimum-image |p_j - q_i|^2 <
 * r2_limit.  Callers pass r2_limit slightly above r_max^2 to also see the
 * pairs in the ambiguity band.  Rows are in query order, and within a row
 * the points are in ascending index order.  Pinned by: explicit image search
 * on tiny boxes, SciPy cKDTree on cubic boxes, perfect-FCC shell counts and
 * pair symmetry.
 * ---------------------------------------------------------------------- */
int orc_ball_count(const orc_box* b, const float* pts, int64_t n, const float* q, int64_t nq,
                   double r2_limit, int32_t exclude_ii, int64_t* counts)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        int64_t c = 0;
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (exclude_ii && i == j) continue;
            if (pair_r2(b, pts + 3 * j, q + 3 * i, d) < r2_limit) ++c;
        }
        counts[i] = c;
    }
    return 0;
}

int orc_ball_fill(const orc_box* b, const float* pts, int64_t n, const float* q, int64_t nq,
                  double r2_limit, int32_t exclude_ii, const int64_t* offsets, int32_t* idx,
                  double* r2_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        int64_t o = offsets[i];
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (exclude_ii && i == j) continue;
            double r2 = pair_r2(b, pts + 3 * j, q + 3 * i, d);
            if (r2 < r2_limit) {
                idx[o] = (int32_t)j;
                r2_out[o] = r2;
                ++o;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Histogram bin of a squared distance x over edges e_b = r_min + b*dr,
 * b = 0..bins: the b with e_b^2 <= x < e_{b+1}^2, or -1 below r_min^2, or
 * `bins` at or above r_max^2.  The first guess from the square root is
 * corrected against the squared edges so the comparison is exact in FP64.
 * ---------------------------------------------------------------------- */
static int64_t bin_of(double x, double r_min, double dr, int64_t bins)
{
    double e0 = r_min;
    double eB = r_min + (double)bins * dr;
    if (x < e0 * e0) return -1;
    if (x >= eB * eB) return bins;
    int64_t b = (int64_t)floor((sqrt(x) - r_min) / dr);
    if (b < 0) b = 0;
    if (b > bins - 1) b = bins - 1;
    while (b > 0 && x < (r_min + (double)b * dr) * (r_min + (double)b * dr)) --b;
    while (b < bins - 1 && x >= (r_min + (double)(b + 1) * dr) * (r_min + (double)(b + 1) * dr)) ++b;
    return b;
}

/* ------------------------------------------------------------------------
 * RDF pair-distance histogram (Analysis Modules: the density module's RDF;
 * PMFT section: g(r) = exp(-beta F(r))).  Bins are half-open and uniform in
 * r on [r_min, r_max).  For grading a single-precision implementation, each
 * pair whose squared distance lies within rel_band of the square of any bin
 * edge (r_min and r_max included) is "ambiguous": it adds to hi[] for every
 * bin it could fall in and to n_amb, and not to lo[].  Every other pair adds
 * to both lo[b] and hi[b].  An exact implementation satisfies
 * lo <= counts <= hi.  Pinned by: brute-force numpy binning on tiny inputs,
 * FCC shell multiplicities, and the ideal-gas limit g -> (N-1)/N.
 * ---------------------------------------------------------------------- */
/* One pair's contribution to the RDF bounds: the bins its squared distance
 * x can reach within the band; a single bin counts in lo and hi, a range is
 * ambiguous and counts in hi only (and in *amb). */
static void rdf_add_pair(double x, double r_min, double dr, int64_t bins, double rel_band,
                         uint64_t* tlo, uint64_t* thi, uint64_t* amb)
{
    const int64_t blo = bin_of(x / (1.0 + rel_band), r_min, dr, bins);
    const int64_t bhi = bin_of(x / (1.0 - rel_band), r_min, dr, bins);
    if (blo == bhi) {
        if (blo >= 0 && blo < bins) { tlo[blo]++; thi[blo]++; }
    } else {
        ++*amb;
        for (int64_t k = blo; k <= bhi; ++k)
            if (k >= 0 && k < bins) thi[k]++;
    }
}

int orc_rdf(const orc_box* b, const float* pts, int64_t n, const float* q, int64_t nq,
            int64_t bins, double r_min, double r_max, int32_t exclude_ii, double rel_band,
            uint64_t* lo, uint64_t* hi, uint64_t* n_amb)
{
    const double dr = (r_max - r_min) / (double)bins;
    const double r2_lim = r_max * r_max * (1.0 + rel_band);
    memset(lo, 0, sizeof(uint64_t) * bins);
    memset(hi, 0, sizeof(uint64_t) * bins);
    uint64_t amb_total = 0;
#pragma omp parallel
    {
        uint64_t* tlo = (uint64_t*)calloc((size_t)bins, sizeof(uint64_t));
        uint64_t* thi = (uint64_t*)calloc((size_t)bins, sizeof(uint64_t));
        uint64_t tamb = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < nq; ++i) {
            double d[3];
            for (int64_t j = 0; j < n; ++j) {
                if (exclude_ii && i == j) continue;
                double x = pair_r2(b, pts + 3 * j, q + 3 * i, d);
                if (x >= r2_lim) continue;
                rdf_add_pair(x, r_min, dr, bins, rel_band, tlo, thi, &tamb);
            }
        }
#pragma omp critical
        {
            for (int64_t k = 0; k < bins; ++k) { lo[k] += tlo[k]; hi[k] += thi[k]; }
            amb_total += tamb;
        }
        free(tlo);
        free(thi);
    }
    *n_amb = amb_total;
    return 0;
}

/* ------------------------------------------------------------------------
 * The ball query and the RDF bounds of the same pairs in one sweep over all
 * (query, point) pairs: the two definitions above evaluated together, so a
 * large system is checked with one brute-force pass instead of three.
 * Query row i is q[i] with global index q_first + i (exclude_ii drops
 * j == q_first + i).  The row's points with r^2 < r2_limit go, in ascending
 * j with their r^2, to idx / r2_out at i * cap onwards; counts[i] is the full
 * row length, and a row longer than cap is cut there and makes the return
 * value 1.  Every pair with r^2 < r_max^2 (1 + rel_band) is binned exactly as
 * orc_rdf bins it into lo / hi and n_amb, which accumulate (the caller
 * zeroes them), so row ranges can be swept one after another.  Pinned by:
 * equality with orc_ball_count / orc_ball_fill and orc_rdf.
 * ---------------------------------------------------------------------- */
int orc_ball_rdf_rows(const orc_box* b, const float* pts, int64_t n, const float* q, int64_t nq,
                      int64_t q_first, double r2_limit, int32_t exclude_ii, int64_t cap,
                      int32_t* idx, double* r2_out, int64_t* counts, int64_t bins, double r_min,
                      double r_max, double rel_band, uint64_t* lo, uint64_t* hi, uint64_t* n_amb)
{
    const double dr = (r_max - r_min) / (double)bins;
    const double r2_hist = r_max * r_max * (1.0 + rel_band);
    int cut = 0;
    uint64_t amb_total = 0;
#pragma omp parallel
    {
        uint64_t* tlo = (uint64_t*)calloc((size_t)bins, sizeof(uint64_t));
        uint64_t* thi = (uint64_t*)calloc((size_t)bins, sizeof(uint64_t));
        uint64_t tamb = 0;
        int tcut = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < nq; ++i) {
            const int64_t self = q_first + i;
            int64_t c = 0;
            double d[3];
            for (int64_t j = 0; j < n; ++j) {
                if (exclude_ii && j == self) continue;
                const double x = pair_r2(b, pts + 3 * j, q + 3 * i, d);
                if (x < r2_limit) {
                    if (c < cap) {
                        idx[i * cap + c] = (int32_t)j;
                        r2_out[i * cap + c] = x;
                    } else {
                        tcut = 1;
                    }
                    ++c;
                }
                if (x < r2_hist) rdf_add_pair(x, r_min, dr, bins, rel_band, tlo, thi, &tamb);
            }
            counts[i] = c;
        }
#pragma omp critical
        {
            for (int64_t k = 0; k < bins; ++k) { lo[k] += tlo[k]; hi[k] += thi[k]; }
            amb_total += tamb;
            cut |= tcut;
        }
        free(tlo);
        free(thi);
    }
    *n_amb += amb_total;
    return cut;
}

/* ------------------------------------------------------------------------
 * Spatial correlation function of per-particle values (Analysis Modules:
 * the density module's correlation functions of arbitrary quantities; the
 * overview figure's correlation of the hexatic order parameter).  Values
 * are complex (re, im as two floats); for every ball pair (i, j), query i
 * with value f_i and point j with value g_j, r_min <= r < r_max, the term
 * conj(f_i) g_j is added to bin b and the pair counted there; the
 * correlation is C_b = S_b / N_b.  Terms are formed in double from the
 * float inputs (the products are exact, the sum of two rounds once).
 * Bin assignment and ambiguity follow the RDF: a pair within rel_band of a
 * bin edge (in r^2) is ambiguous; it adds 1 to hi[k] and |Re term| + |Im
 * term| to amb_mass[k] for every bin k it may reach, and nothing to
 * sum_cert.  Certain pairs add to lo, hi and sum_cert[2b], sum_cert[2b+1].
 * An exact implementation satisfies lo <= N <= hi and, per component,
 * |S_b - sum_cert_b| <= amb_mass_b up to double rounding.  Pinned by:
 * constant values (C_b = |c|^2, counts equal to the RDF's), a numpy brute
 * force with explicit image search, a hand-computed complex pair (which
 * side is conjugated) and the Hermitian symmetry of self-queries.
 * ---------------------------------------------------------------------- */
int orc_correlation(const orc_box* b, const float* pts, const float* vals, int64_t n,
                    const float* q, const float* qvals, int64_t nq, int64_t bins, double r_min,
                    double r_max, int32_t exclude_ii, double rel_band, double* sum_cert,
                    double* amb_mass, uint64_t* lo, uint64_t* hi, uint64_t* n_amb)
{
    const double dr = (r_max - r_min) / (double)bins;
    const double r2_lim = r_max * r_max * (1.0 + rel_band);
    memset(sum_cert, 0, sizeof(double) * 2 * bins);
    memset(amb_mass, 0, sizeof(double) * bins);
    memset(lo, 0, sizeof(uint64_t) * bins);
    memset(hi, 0, sizeof(uint64_t) * bins);
    uint64_t amb_total = 0;
#pragma omp parallel
    {
        double* ts = (double*)calloc((size_t)(2 * bins), sizeof(double));
        double* tm = (double*)calloc((size_t)bins, sizeof(double));
        uint64_t* tlo = (uint64_t*)calloc((size_t)bins, sizeof(uint64_t));
        uint64_t* thi = (uint64_t*)calloc((size_t)bins, sizeof(uint64_t));
        uint64_t tamb = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < nq; ++i) {
            const double fr = qvals[2 * i], fi = qvals[2 * i + 1];
            double d[3];
            for (int64_t j = 0; j < n; ++j) {
                if (exclude_ii && i == j) continue;
                const double x = pair_r2(b, pts + 3 * j, q + 3 * i, d);
                if (x >= r2_lim) continue;
                const double gr = vals[2 * j], gi = vals[2 * j + 1];
                /* conj(f) g = (fr - i fi)(gr + i gi) */
                const double re = fr * gr + fi * gi;
                const double im = fr * gi - fi * gr;
                const int64_t blo = bin_of(x / (1.0 + rel_band), r_min, dr, bins);
                const int64_t bhi = bin_of(x / (1.0 - rel_band), r_min, dr, bins);
                if (blo == bhi) {
                    if (blo >= 0 && blo < bins) {
                        tlo[blo]++;
                        thi[blo]++;
                        ts[2 * blo] += re;
                        ts[2 * blo + 1] += im;
                    }
                } else {
                    ++tamb;
                    for (int64_t k = blo; k <= bhi; ++k)
                        if (k >= 0 && k < bins) {
                            thi[k]++;
                            tm[k] += fabs(re) + fabs(im);
                        }
                }
            }
        }
#pragma omp critical
        {
            for (int64_t k = 0; k < bins; ++k) {
                lo[k] += tlo[k];
                hi[k] += thi[k];
                amb_mass[k] += tm[k];
                sum_cert[2 * k] += ts[2 * k];
                sum_cert[2 * k + 1] += ts[2 * k + 1];
            }
            amb_total += tamb;
        }
        free(ts);
        free(tm);
        free(tlo);
        free(thi);
    }
    *n_amb = amb_total;
    return 0;
}

/* ------------------------------------------------------------------------
 * k nearest neighbors (query API with a neighbor count, General Utilities
 * section and the common-neighbor example).  Row i holds the first m =
 * k + extra candidates in the order (r^2, j), excluding j == i under
 * exclude_ii and, when r2_guard > 0, candidates with r^2 >= r2_guard.  Rows
 * shorter than m are padded with index -1.  The caller keeps the first k and
 * uses the extra entries to detect near-ties at rank k.  Selection keeps a
 * sorted buffer of the m best seen so far (insertion), which is the partial
 * sort of the definition.  Pinned by: perfect FCC (12 neighbors at a/sqrt2)
 * and a full numpy sort on tiny inputs.
 * ---------------------------------------------------------------------- */
int orc_knn(const orc_box* b, const float* pts, int64_t n, const float* q, int64_t nq, int32_t k,
            int32_t extra, int32_t exclude_ii, double r2_guard, int32_t* idx, double* r2_out,
            int32_t* row_len)
{
    const int32_t m = k + extra;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        int32_t* ri = idx + i * m;
        double* rr = r2_out + i * m;
        int32_t len = 0;
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (exclude_ii && i == j) continue;
            double x = pair_r2(b, pts + 3 * j, q + 3 * i, d);
            if (r2_guard > 0.0 && x >= r2_guard) continue;
            /* (x, j) is larger than every earlier j at equal x, so ties keep
             * ascending j by inserting after equal keys */
            if (len == m && !(x < rr[m - 1])) continue;
            int32_t pos = (len < m) ? len : m - 1;
            while (pos > 0 && x < rr[pos - 1]) {
                rr[pos] = rr[pos - 1];
                ri[pos] = ri[pos - 1];
                --pos;
            }
            rr[pos] = x;
            ri[pos] = (int32_t)j;
            if (len < m) ++len;
        }
        for (int32_t t = len; t < m; ++t) { ri[t] = -1; rr[t] = INFINITY; }
        row_len[i] = len;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * 2D PMFT histogram (PMFT section: a histogram of the positions of all other
 * particles in each particle's own frame; the PMFT is minus the log of it).
 * For each ball pair (i, j) in 2D, the bond d = minimum image of p_j - q_i is
 * rotated into the frame of i by -theta_i:
 *     x' =  cos(theta_i) d_x + sin(theta_i) d_y
 *     y' = -sin(theta_i) d_x + cos(theta_i) d_y
 * and binned on [-x_max, x_max) x [-y_max, y_max) with nbx x nby uniform
 * bins, counts[ix * nby + iy].  Ambiguity for grading: r^2 within rel_band
 * of r_max^2, or x' (y') within abs_band of any x (y) edge.  Pinned by:
 * theta = 0 against numpy.histogram2d of bond vectors, theta = pi/2 as an
 * index rotation, and total count = number of ball pairs in range.
 * ---------------------------------------------------------------------- */
static int64_t edge_bin(double x, double lo, double width, int64_t nb)
{
    double t = floor((x - lo) / width);
    if (t < 0.0) return -1;
    if (t >= (double)nb) return nb;
    return (int64_t)t;
}

int orc_pmft2d(const orc_box* b, const float* pts, int64_t n, const float* q, const float* q_theta,
               int64_t nq, int64_t nbx, int64_t nby, double x_max, double y_max, double r_max,
               int32_t exclude_ii, double rel_band, double abs_band, uint64_t* lo, uint64_t* hi,
               uint64_t* n_amb)
{
    const double dx = 2.0 * x_max / (double)nbx;
    const double dy = 2.0 * y_max / (double)nby;
    const double r2_in = r_max * r_max * (1.0 - rel_band);
    const double r2_lim = r_max * r_max * (1.0 + rel_band);
    const int64_t nbins = nbx * nby;
    memset(lo, 0, sizeof(uint64_t) * nbins);
    memset(hi, 0, sizeof(uint64_t) * nbins);
    uint64_t amb_total = 0;
#pragma omp parallel
    {
        uint64_t* tlo = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
        uint64_t* thi = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
        uint64_t tamb = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < nq; ++i) {
            const double th = (double)q_theta[i];
            const double c = cos(th), s = sin(th);
            double d[3];
            for (int64_t j = 0; j < n; ++j) {
                if (exclude_ii && i == j) continue;
                double r2 = pair_r2(b, pts + 3 * j, q + 3 * i, d);
                if (r2 >= r2_lim) continue;
                double xr = c * d[0] + s * d[1];
                double yr = -s * d[0] + c * d[1];
                int64_t ix0 = edge_bin(xr - abs_band, -x_max, dx, nbx);
                int64_t ix1 = edge_bin(xr + abs_band, -x_max, dx, nbx);
                int64_t iy0 = edge_bin(yr - abs_band, -y_max, dy, nby);
                int64_t iy1 = edge_bin(yr + abs_band, -y_max, dy, nby);
                int certain_in_ball = r2 < r2_in;
                if (certain_in_ball && ix0 == ix1 && iy0 == iy1) {
                    if (ix0 >= 0 && ix0 < nbx && iy0 >= 0 && iy0 < nby) {
                        tlo[ix0 * nby + iy0]++;
                        thi[ix0 * nby + iy0]++;
                    }
                } else {
                    ++tamb;
                    for (int64_t ix = ix0; ix <= ix1; ++ix)
                        for (int64_t iy = iy0; iy <= iy1; ++iy)
                            if (ix >= 0 && ix < nbx && iy >= 0 && iy < nby) thi[ix * nby + iy]++;
                }
            }
        }
#pragma omp critical
        {
            for (int64_t t = 0; t < nbins; ++t) { lo[t] += tlo[t]; hi[t] += thi[t]; }
            amb_total += tamb;
        }
        free(tlo);
        free(thi);
    }
    *n_amb = amb_total;
    return 0;
}

/* ------------------------------------------------------------------------
 * Three-dimensional PMFT histograms (PMFT section: in 2D the full PMFT also
 * resolves the orientation of the second particle relative to the first; in
 * 3D the translational part alone is three-dimensional).  Both bin the bond
 * d = minimum image of p_j - q_i of every pair closer than r_max, seen from
 * the query particle's own frame, in a uniform histogram:
 *
 *   XYT (2D): (x', y') = R(-theta_i) d as in the 2D PMFT, and the relative
 *     orientation t = (theta_j - theta_i) mod 2 pi in [0, 2 pi), binned into
 *     nbt equal bins; counts[(ix * nby + iy) * nbt + it].
 *   XYZ (3D): d' = R(q_i)^T d, the bond in the frame of the query's unit
 *     quaternion q_i = (w, x, y, z) (normalised here), with the rotation
 *     matrix of a unit quaternion; counts[(ix * nby + iy) * nbz + iz] on
 *     [-x_max, x_max) x [-y_max, y_max) x [-z_max, z_max).
 *
 * lo/hi bound the histogram over the ambiguous pairs exactly as in the 2D
 * PMFT: a pair within rel_band of r_max^2, or within the absolute band of a
 * bin edge in any coordinate (t_band for the angle, whose edges wrap), adds
 * 1 to hi in every bin it may reach and is counted in n_amb.  Pinned by:
 * theta = 0 (XYT) and identity quaternions (XYZ) reducing to numpy's
 * histogramdd of minimum-image displacements, the marginal over t equal to
 * the 2D PMFT, hand-computed bins of a two-particle system with a general
 * angle and a general quaternion, and rotations about z in 3D matching the
 * 2D PMFT.
 * ---------------------------------------------------------------------- */
static void bins3_add(uint64_t* tlo, uint64_t* thi, uint64_t* tamb, int certain,
                      const int64_t b0[3], const int64_t b1[3], const int64_t nb[3], int wrap2)
{
    if (certain && b0[0] == b1[0] && b0[1] == b1[1] && b0[2] == b1[2]) {
        int64_t k2 = b0[2];
        if (wrap2) k2 = ((k2 % nb[2]) + nb[2]) % nb[2];
        if (b0[0] >= 0 && b0[0] < nb[0] && b0[1] >= 0 && b0[1] < nb[1] && k2 >= 0 && k2 < nb[2]) {
            const int64_t t = (b0[0] * nb[1] + b0[1]) * nb[2] + k2;
            tlo[t]++;
            thi[t]++;
        }
        return;
    }
    ++*tamb;
    for (int64_t i0 = b0[0]; i0 <= b1[0]; ++i0) {
        if (i0 < 0 || i0 >= nb[0]) continue;
        for (int64_t i1 = b0[1]; i1 <= b1[1]; ++i1) {
            if (i1 < 0 || i1 >= nb[1]) continue;
            for (int64_t i2 = b0[2]; i2 <= b1[2]; ++i2) {
                int64_t k2 = i2;
                if (wrap2) k2 = ((k2 % nb[2]) + nb[2]) % nb[2];
                if (k2 < 0 || k2 >= nb[2]) continue;
                thi[(i0 * nb[1] + i1) * nb[2] + k2]++;
            }
        }
    }
}

int orc_pmft_xyt(const orc_box* b, const float* pts, const float* theta, int64_t n,
                 const float* q, const float* q_theta, int64_t nq, int64_t nbx, int64_t nby,
                 int64_t nbt, double x_max, double y_max, double r_max, int32_t exclude_ii,
                 double rel_band, double abs_band, double t_band, uint64_t* lo, uint64_t* hi,
                 uint64_t* n_amb)
{
    const double two_pi = 2.0 * M_PI;
    const double w[3] = {2.0 * x_max / (double)nbx, 2.0 * y_max / (double)nby,
                         two_pi / (double)nbt};
    const double org[3] = {-x_max, -y_max, 0.0};
    const int64_t nb[3] = {nbx, nby, nbt};
    const double r2_in = r_max * r_max * (1.0 - rel_band);
    const double r2_lim = r_max * r_max * (1.0 + rel_band);
    const int64_t nbins = nbx * nby * nbt;
    memset(lo, 0, sizeof(uint64_t) * nbins);
    memset(hi, 0, sizeof(uint64_t) * nbins);
    uint64_t amb_total = 0;
#pragma omp parallel
    {
        uint64_t* tlo = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
        uint64_t* thi = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
        uint64_t tamb = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < nq; ++i) {
            const double th = (double)q_theta[i];
            const double c = cos(th), s = sin(th);
            double d[3];
            for (int64_t j = 0; j < n; ++j) {
                if (exclude_ii && i == j) continue;
                const double r2 = pair_r2(b, pts + 3 * j, q + 3 * i, d);
                if (r2 >= r2_lim) continue;
                double t = fmod((double)theta[j] - th, two_pi);
                if (t < 0.0) t += two_pi;
                const double v[3] = {c * d[0] + s * d[1], -s * d[0] + c * d[1], t};
                const double band[3] = {abs_band, abs_band, t_band};
                int64_t b0[3], b1[3];
                for (int k = 0; k < 3; ++k) {
                    b0[k] = (int64_t)floor((v[k] - band[k] - org[k]) / w[k]);
                    b1[k] = (int64_t)floor((v[k] + band[k] - org[k]) / w[k]);
                }
                bins3_add(tlo, thi, &tamb, r2 < r2_in, b0, b1, nb, 1);
            }
        }
#pragma omp critical
        {
            for (int64_t t = 0; t < nbins; ++t) { lo[t] += tlo[t]; hi[t] += thi[t]; }
            amb_total += tamb;
        }
        free(tlo);
        free(thi);
    }
    *n_amb = amb_total;
    return 0;
}

int orc_pmft_xyz(const orc_box* b, const float* pts, int64_t n, const float* q,
                 const float* q_quat, int64_t nq, int64_t nbx, int64_t nby, int64_t nbz,
                 double x_max, double y_max, double z_max, double r_max, int32_t exclude_ii,
                 double rel_band, double abs_band, uint64_t* lo, uint64_t* hi, uint64_t* n_amb)
{
    const double w[3] = {2.0 * x_max / (double)nbx, 2.0 * y_max / (double)nby,
                         2.0 * z_max / (double)nbz};
    const double org[3] = {-x_max, -y_max, -z_max};
    const int64_t nb[3] = {nbx, nby, nbz};
    const double r2_in = r_max * r_max * (1.0 - rel_band);
    const double r2_lim = r_max * r_max * (1.0 + rel_band);
    const int64_t nbins = nbx * nby * nbz;
    memset(lo, 0, sizeof(uint64_t) * nbins);
    memset(hi, 0, sizeof(uint64_t) * nbins);
    uint64_t amb_total = 0;
#pragma omp parallel
    {
        uint64_t* tlo = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
        uint64_t* thi = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
        uint64_t tamb = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < nq; ++i) {
            /* rotation matrix of the normalised quaternion (w, x, y, z) */
            double qw = q_quat[4 * i], qx = q_quat[4 * i + 1], qy = q_quat[4 * i + 2],
                   qz = q_quat[4 * i + 3];
            const double nrm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
            qw /= nrm; qx /= nrm; qy /= nrm; qz /= nrm;
            const double R[3][3] = {
                {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy)},
                {2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx)},
                {2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)}};
            double d[3];
            for (int64_t j = 0; j < n; ++j) {
                if (exclude_ii && i == j) continue;
                const double r2 = pair_r2(b, pts + 3 * j, q + 3 * i, d);
                if (r2 >= r2_lim) continue;
                int64_t b0[3], b1[3];
                for (int k = 0; k < 3; ++k) {
                    /* row k of R^T is column k of R */
                    const double v = R[0][k] * d[0] + R[1][k] * d[1] + R[2][k] * d[2];
                    b0[k] = (int64_t)floor((v - abs_band - org[k]) / w[k]);
                    b1[k] = (int64_t)floor((v + abs_band - org[k]) / w[k]);
                }
                bins3_add(tlo, thi, &tamb, r2 < r2_in, b0, b1, nb, 0);
            }
        }
#pragma omp critical
        {
            for (int64_t t = 0; t < nbins; ++t) { lo[t] += tlo[t]; hi[t] += thi[t]; }
            amb_total += tamb;
        }
        free(tlo);
        free(thi);
    }
    *n_amb = amb_total;
    return 0;
}

/* ------------------------------------------------------------------------
 * Gaussian-smoothed RDF (an extension beyond the paper: a differentiable
 * form of the RDF histogram).  With phi(u) = exp(-u^2/(2 s^2)) /
 * (s sqrt(2 pi)), bin centers c_b = (b + 1/2) dr on [0, r_max), and a window
 * |c_b - r| <= 8 s:
 *     h_b = dr * sum over ordered pairs i != j with r_ij < r_max + 8 s of
 *           phi(c_b - r_ij).
 * smooth_pair_terms adds one pair's contribution to h (scale = dr * weight).
 * Pinned by the sum rule (a single interior pair contributes total mass 1
 * up to an exponentially small aliasing error) and brute-force numpy on tiny
 * inputs.
 * ---------------------------------------------------------------------- */
static void smooth_pair_terms(double r, int64_t bins, double dr, double sigma, double scale,
                              double* h)
{
    const double norm = 1.0 / (sigma * sqrt(2.0 * M_PI));
    for (int64_t bb = 0; bb < bins; ++bb) {
        double u = ((double)bb + 0.5) * dr - r;
        if (fabs(u) > 8.0 * sigma) continue;
        h[bb] += scale * norm * exp(-u * u / (2.0 * sigma * sigma));
    }
}

int orc_smooth_rdf(const orc_box* b, const float* pts, int64_t n, int64_t bins, double r_max,
                   double sigma, double* h)
{
    const double dr = r_max / (double)bins;
    const double rs = r_max + 8.0 * sigma;
    memset(h, 0, sizeof(double) * bins);
#pragma omp parallel
    {
        double* th = (double*)calloc((size_t)bins, sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            double d[3];
            for (int64_t j = 0; j < n; ++j) {
                if (i == j) continue;
                double r = sqrt(pair_r2(b, pts + 3 * j, pts + 3 * i, d));
                if (r < rs) smooth_pair_terms(r, bins, dr, sigma, dr, th);
            }
        }
#pragma omp critical
        for (int64_t k = 0; k < bins; ++k) h[k] += th[k];
        free(th);
    }
    return 0;
}

/* Contribution of the two ordered pairs (k, j) and (j, k), for all j != k,
 * to h, with particle k moved to position pk (three doubles).  Used to
 * evaluate the forward under a perturbation of one particle in O(N) for
 * finite differences: h(p') = h(p) - row(k, p_k) + row(k, p'_k). */
int orc_smooth_rdf_row(const orc_box* b, const float* pts, int64_t n, int64_t k, const double* pk,
                       int64_t bins, double r_max, double sigma, double* h_row)
{
    const double dr = r_max / (double)bins;
    const double rs = r_max + 8.0 * sigma;
    memset(h_row, 0, sizeof(double) * bins);
    for (int64_t j = 0; j < n; ++j) {
        if (j == k) continue;
        double d[3] = {(double)pts[3 * j] - pk[0], (double)pts[3 * j + 1] - pk[1],
                       b->dim == 3 ? (double)pts[3 * j + 2] - pk[2] : 0.0};
        minimum_image(b, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r < rs) smooth_pair_terms(r, bins, dr, sigma, 2.0 * dr, h_row);
    }
    return 0;
}

/* Gradient of a scalar loss through h.  Given gh_b = dL/dh_b:
 *     dL/dp_k = sum_{j != k} 2 A(r_kj) (p_k - p_j)_mi / r_kj,
 *     A(r) = sum_b gh_b dr (c_b - r)/s^2 phi(c_b - r)   (windowed),
 * the factor 2 collecting the ordered pairs (k, j) and (j, k); a pair at
 * r = 0 contributes 0.  Computed for the rows listed in `rows` (nr of
 * them; all rows when rows == NULL), out is nr x 3. */
int orc_smooth_rdf_grad(const orc_box* b, const float* pts, int64_t n, int64_t bins, double r_max,
                        double sigma, const double* gh, const int64_t* rows, int64_t nr,
                        double* out)
{
    const double dr = r_max / (double)bins;
    const double rs = r_max + 8.0 * sigma;
    const double norm = 1.0 / (sigma * sqrt(2.0 * M_PI));
    const int64_t count = rows ? nr : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t) {
        const int64_t k = rows ? rows[t] : t;
        double g[3] = {0.0, 0.0, 0.0};
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            double r = sqrt(pair_r2(b, pts + 3 * j, pts + 3 * k, d)); /* d = p_j - p_k */
            if (!(r < rs) || r == 0.0) continue;
            double A = 0.0;
            for (int64_t bb = 0; bb < bins; ++bb) {
                double u = ((double)bb + 0.5) * dr - r;
                if (fabs(u) > 8.0 * sigma) continue;
                A += gh[bb] * dr * (u / (sigma * sigma)) * norm * exp(-u * u / (2.0 * sigma * sigma));
            }
            /* (p_k - p_j) = -d */
            g[0] += 2.0 * A * (-d[0]) / r;
            g[1] += 2.0 * A * (-d[1]) / r;
            g[2] += 2.0 * A * (-d[2]) / r;
        }
        out[3 * t] = g[0];
        out[3 * t + 1] = g[1];
        out[3 * t + 2] = g[2];
    }
    return 0;
}
