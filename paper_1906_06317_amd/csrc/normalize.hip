// Normalisation of accumulated pair histograms (float64, on the device).
//
// The paper turns the RDF into a potential of mean force through
// g(r) = exp(-beta F(r)) and defines the PMFT as minus the logarithm of the
// histogram of neighbour positions in each particle's own frame (section
// "PMFT"); the RDF and the PMFT accumulate over frames ("Implementation":
// reset=False) and are then averaged.  The histogram of one bin is divided
// by what an ideal gas of the same density would put there:
//
//   RDF:  g_b   = h_b / (D * dV_b),   D = sum_f N_q,f N_p,f / V_f,
//         dV_b  = 4/3 pi (e_{b+1}^3 - e_b^3) in 3D, pi (e_{b+1}^2 - e_b^2) in 2D,
//         e_b   = r_min + b (r_max - r_min) / bins;
//   PMFT: pcf_k = h_k / (D * w),      w = the volume of one bin (for the
//         relative orientation of the XYT PMFT, its share of a full turn);
//   PMF and PMFT (units of kT): -ln g or -ln pcf, +inf where a bin is empty.
//
// The sum D over frames (and the box volumes) is formed on the host in
// float64; one kernel per call divides every bin.  The correlation function
// of per-particle values is finished the same way: C_b = S_b / N_b.
#include <math.h>

#include "internal.hpp"

namespace ppa {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// One thread per bin.  den_per_bin: the bin's ideal-gas count is
// D * shell(b) for the RDF (shell volume from the edges) or D * w for the
// uniform bins of a PMFT (shell == false).
template <typename T>
__global__ void __launch_bounds__(256) normalize_kernel(const T* __restrict__ counts, int64_t nbins,
                                                        double D, bool shell, int dim, double r_min,
                                                        double dr, double w,
                                                        double* __restrict__ ratio,
                                                        double* __restrict__ neglog,
                                                        double* __restrict__ scale)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    double vol = w;
    if (shell) {
        const double e0 = r_min + (double)b * dr;
        const double e1 = r_min + (double)(b + 1) * dr;
        vol = dim == 3 ? (4.0 / 3.0) * kPi * (e1 * e1 * e1 - e0 * e0 * e0)
                       : kPi * (e1 * e1 - e0 * e0);
    }
    const double inv = 1.0 / (D * vol);
    if (scale) scale[b] = inv;
    if (!counts) return;
    const double g = (double)counts[b] * inv;
    if (ratio) ratio[b] = g;
    if (neglog) neglog[b] = g > 0.0 ? -log(g) : (double)INFINITY;
}

__global__ void __launch_bounds__(256) corr_finalize_kernel(const double* __restrict__ sums,
                                                            const uint64_t* __restrict__ counts,
                                                            int bins, double* __restrict__ corr)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bins) return;
    const uint64_t c = counts[b];
    const double re = c ? sums[2 * b] / (double)c : 0.0;
    const double im = c ? sums[2 * b + 1] / (double)c : 0.0;
    corr[2 * b] = re;
    corr[2 * b + 1] = im;
}

// D = sum over frames of N_q N_p / V (area in 2D) for boxes of dimension
// `dim`; checks every frame.
int ideal_density(int32_t n_frames, const ppa_box* boxes, const int64_t* n_points,
                  const int64_t* n_query, int dim, double* D)
{
    if (n_frames < 1) return set_error(PPA_EINVAL, "n_frames must be >= 1");
    if (!boxes || !n_points || !n_query)
        return set_error(PPA_EINVAL, "boxes, n_points and n_query are required");
    double s = 0.0;
    for (int f = 0; f < n_frames; ++f) {
        BoxPrep bp;
        const int rc = prepare_box(&boxes[f], &bp);
        if (rc) return rc;
        if (bp.dim != dim)
            return set_error(PPA_EINVAL, "frame %d: this normalisation needs a %dD box", f, dim);
        if (n_points[f] < 0 || n_query[f] < 0)
            return set_error(PPA_EINVAL, "frame %d: negative point count", f);
        const double V = dim == 3 ? boxes[f].L[0] * boxes[f].L[1] * boxes[f].L[2]
                                  : boxes[f].L[0] * boxes[f].L[1];
        s += (double)n_query[f] * ((double)n_points[f] / V);
    }
    if (!(s > 0.0)) return set_error(PPA_EINVAL, "no query or no point in any frame");
    *D = s;
    return PPA_OK;
}

template <typename T>
int launch_normalize(const T* counts, int64_t nbins, double D, bool shell, int dim, double r_min,
                     double dr, double w, double* ratio, double* neglog, double* scale,
                     hipStream_t s)
{
    const int blocks = (int)((nbins + 255) / 256);
    hipLaunchKernelGGL(normalize_kernel<T>, dim3(blocks), dim3(256), 0, s, counts, nbins, D, shell,
                       dim, r_min, dr, w, ratio, neglog, scale);
    return hip_check(hipGetLastError(), "normalize kernel launch");
}

int check_range(double lo, double hi)
{
    if (!(isfinite(lo) && isfinite(hi) && lo >= 0.0 && hi > lo))
        return set_error(PPA_EINVAL, "need 0 <= r_min < r_max, both finite");
    return PPA_OK;
}

int check_bins3(const int32_t nb[3], const double range[3], int nd)
{
    int64_t tot = 1;
    for (int k = 0; k < nd; ++k) {
        if (nb[k] < 1) return set_error(PPA_EINVAL, "bin counts must be >= 1");
        tot *= nb[k];
        if (tot > (int64_t)1 << 31) return set_error(PPA_EINVAL, "too many bins");
        if (range[k] >= 0.0 && !(isfinite(range[k]) && range[k] > 0.0))
            return set_error(PPA_EINVAL, "coordinate ranges must be finite and positive");
    }
    return PPA_OK;
}

}  // namespace

}  // namespace ppa

using namespace ppa;

extern "C" {

int ppa_rdf_normalize(const uint64_t* counts, int32_t bins, double r_min, double r_max,
                      int32_t n_frames, const ppa_box* boxes, const int64_t* n_points,
                      const int64_t* n_query, double* g, double* pmf, hipStream_t stream)
{
    if (!counts || !g) return set_error(PPA_EINVAL, "counts and g are required");
    if (bins < 1) return set_error(PPA_EINVAL, "bins must be >= 1");
    int rc = check_range(r_min, r_max);
    if (rc) return rc;
    if (!boxes) return set_error(PPA_EINVAL, "boxes are required");
    const int dim = boxes[0].dim;
    double D = 0.0;
    rc = ideal_density(n_frames, boxes, n_points, n_query, dim, &D);
    if (rc) return rc;
    return launch_normalize(counts, bins, D, true, dim, r_min, (r_max - r_min) / bins, 0.0, g, pmf,
                            (double*)nullptr, stream);
}

int ppa_rdf_bin_scale(int32_t bins, double r_min, double r_max, int32_t n_frames,
                      const ppa_box* boxes, const int64_t* n_points, const int64_t* n_query,
                      double* scale, hipStream_t stream)
{
    if (!scale) return set_error(PPA_EINVAL, "scale is required");
    if (bins < 1) return set_error(PPA_EINVAL, "bins must be >= 1");
    int rc = check_range(r_min, r_max);
    if (rc) return rc;
    if (!boxes) return set_error(PPA_EINVAL, "boxes are required");
    const int dim = boxes[0].dim;
    double D = 0.0;
    rc = ideal_density(n_frames, boxes, n_points, n_query, dim, &D);
    if (rc) return rc;
    return launch_normalize((const double*)nullptr, bins, D, true, dim, r_min,
                            (r_max - r_min) / bins, 0.0, (double*)nullptr, (double*)nullptr, scale,
                            stream);
}

int ppa_pmft2d_normalize(const uint32_t* counts, int32_t nbx, int32_t nby, double x_max,
                         double y_max, int32_t n_frames, const ppa_box* boxes,
                         const int64_t* n_points, const int64_t* n_query, double* pcf,
                         double* pmft, hipStream_t stream)
{
    if (!counts || !pcf) return set_error(PPA_EINVAL, "counts and pcf are required");
    const int32_t nb[3] = {nbx, nby, 1};
    const double rg[3] = {x_max, y_max, 1.0};
    int rc = check_bins3(nb, rg, 2);
    if (rc) return rc;
    double D = 0.0;
    rc = ideal_density(n_frames, boxes, n_points, n_query, 2, &D);
    if (rc) return rc;
    const double w = (2.0 * x_max / nbx) * (2.0 * y_max / nby);
    return launch_normalize(counts, (int64_t)nbx * nby, D, false, 2, 0.0, 0.0, w, pcf, pmft,
                            (double*)nullptr, stream);
}

int ppa_pmft_xyt_normalize(const uint32_t* counts, int32_t nbx, int32_t nby, int32_t nbt,
                           double x_max, double y_max, int32_t n_frames, const ppa_box* boxes,
                           const int64_t* n_points, const int64_t* n_query, double* pcf,
                           double* pmft, hipStream_t stream)
{
    if (!counts || !pcf) return set_error(PPA_EINVAL, "counts and pcf are required");
    const int32_t nb[3] = {nbx, nby, nbt};
    const double rg[3] = {x_max, y_max, -1.0};
    int rc = check_bins3(nb, rg, 3);
    if (rc) return rc;
    double D = 0.0;
    rc = ideal_density(n_frames, boxes, n_points, n_query, 2, &D);
    if (rc) return rc;
    // the angle bin's share of the full turn, so an ideal gas gives pcf = 1
    const double w = (2.0 * x_max / nbx) * (2.0 * y_max / nby) / nbt;
    return launch_normalize(counts, (int64_t)nbx * nby * nbt, D, false, 2, 0.0, 0.0, w, pcf, pmft,
                            (double*)nullptr, stream);
}

int ppa_pmft_xyz_normalize(const uint32_t* counts, int32_t nbx, int32_t nby, int32_t nbz,
                           double x_max, double y_max, double z_max, int32_t n_frames,
                           const ppa_box* boxes, const int64_t* n_points, const int64_t* n_query,
                           double* pcf, double* pmft, hipStream_t stream)
{
    if (!counts || !pcf) return set_error(PPA_EINVAL, "counts and pcf are required");
    const int32_t nb[3] = {nbx, nby, nbz};
    const double rg[3] = {x_max, y_max, z_max};
    int rc = check_bins3(nb, rg, 3);
    if (rc) return rc;
    double D = 0.0;
    rc = ideal_density(n_frames, boxes, n_points, n_query, 3, &D);
    if (rc) return rc;
    const double w = (2.0 * x_max / nbx) * (2.0 * y_max / nby) * (2.0 * z_max / nbz);
    return launch_normalize(counts, (int64_t)nbx * nby * nbz, D, false, 3, 0.0, 0.0, w, pcf, pmft,
                            (double*)nullptr, stream);
}

int ppa_correlation_finalize(const double* sums, const uint64_t* counts, int32_t bins,
                             double* corr, hipStream_t stream)
{
    if (!sums || !counts || !corr) return set_error(PPA_EINVAL, "sums, counts and corr are required");
    if (bins < 1) return set_error(PPA_EINVAL, "bins must be >= 1");
    hipLaunchKernelGGL(corr_finalize_kernel, dim3((bins + 255) / 256), dim3(256), 0, stream, sums,
                       counts, bins, corr);
    return hip_check(hipGetLastError(), "correlation finalize launch");
}

}  // extern "C"
