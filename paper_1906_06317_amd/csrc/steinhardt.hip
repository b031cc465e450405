// Steinhardt bond-orientational order parameters of the rows of a
// NeighborList (the paper's order-parameter features; its Q6 example runs on
// the 12-nearest-neighbour list).  For query i with bonds d_ij = minimum
// image of p_j - q_i over its row (bonds of length 0 are skipped):
//     q_lm(i) = (1 / N_b) sum_j Y_lm(d_ij),
//     Q_l(i)  = sqrt(4 pi / (2l + 1) sum_{m=-l..l} |q_lm|^2),
//     W_l(i)  = sum_{m1+m2+m3=0} (l l l; m1 m2 m3) q_lm1 q_lm2 q_lm3
//               / (sum_m |q_lm|^2)^(3/2)          (normalised W-hat).
// One lane per query row, float64 throughout.  Y_lm = N P_l^m(cos t) e^{i m p}
// comes from the recurrences of the normalised associated Legendre
// functions: the sectoral term times e^{i m p} is c_m ((x + i y) / r)^m,
// advanced from m - 1 by one complex product, and P_l^m / P_m^m follows the
// upward recurrence in l (one square root and one division per bond); with
// q_{l,-m} = (-1)^m conj(q_lm) only m >= 0 is accumulated.  The kernel is
// instantiated per l, so the m loops and the recurrence coefficients are
// compile-time constants and q_lm stays in registers; for W each lane
// stages its q_lm in LDS for the double loop over (m1, m2).  The Wigner 3j
// symbols come from a setup kernel (Racah formula) into the workspace.
#include "internal.hpp"

namespace ppa {

namespace {

constexpr int kStBlock = 256;
constexpr double kInvSqrt4Pi = 0.28209479177387814347;

// (l l l; m1 m2 m3) by the Racah formula (float64 factorials from `f`).
__device__ double racah_lll(int l, int m1, int m2, int m3, const double* f)
{
    const int a[6] = {l + m1, l - m1, l + m2, l - m2, l + m3, l - m3};
    double pre = f[l] * f[l] * f[l] / f[3 * l + 1];
    for (int k = 0; k < 6; ++k) pre *= f[a[k]];
    double sum = 0.0;
    for (int k = 0; k <= 3 * l + 1; ++k) {
        const int b0 = k + m1, b1 = k - m2, b2 = l - k, b3 = l - k - m1, b4 = l - k + m2;
        if (b0 < 0 || b1 < 0 || b2 < 0 || b3 < 0 || b4 < 0) continue;
        const double t = 1.0 / (f[k] * f[b0] * f[b1] * f[b2] * f[b3] * f[b4]);
        sum += (k & 1) ? -t : t;
    }
    const double sign = (m3 & 1) ? -1.0 : 1.0;  // (-1)^(j1 - j2 - m3) with j1 = j2
    return sign * sqrt(pre) * sum;
}

// Clears the status word; with W, writes (l l l; m1 m2 -m1-m2) at
// table[(m1 + l)(2l + 1) + m2 + l].
__global__ void __launch_bounds__(256) steinhardt_setup_kernel(int l, int want_w, double* table,
                                                               unsigned* status)
{
    __shared__ double f[3 * kSteinMaxL + 2];
    for (int i = threadIdx.x; i <= 3 * l + 1; i += blockDim.x) {
        double v = 1.0;
        for (int k = 2; k <= i; ++k) v *= (double)k;
        f[i] = v;
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0u;
    if (!want_w) return;
    const int w = 2 * l + 1;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < w * w; t += gridDim.x * blockDim.x) {
        const int m1 = t / w - l, m2 = t % w - l, m3 = -m1 - m2;
        table[t] = (m3 >= -l && m3 <= l) ? racah_lll(l, m1, m2, m3, f) : 0.0;
    }
}

// q_{l,m} for any m from the stored m >= 0 terms: q_{l,-m} = (-1)^m conj(q_lm).
__device__ __forceinline__ double2 q_of(const double2* q, int m)
{
    if (m >= 0) return q[m];
    const double2 v = q[-m];
    return (m & 1) ? make_double2(-v.x, v.y) : make_double2(v.x, -v.y);
}

// Five wavefronts per SIMD for l <= 6 (96 VGPRs: Q6 with W6 on the k = 12
// list of the 2^20-point FCC 0.217 -> 0.203 ms); larger l keep their
// registers (l = 8 at five wavefronts spills; l = 12 bounded to four
// spilled and took 0.80 ms instead of 0.66).
template <int L>
__global__ void __launch_bounds__(kStBlock, (L <= 6 ? 5 : 1)) steinhardt_kernel(const SteinArgs a)
{
    const long long i = (long long)blockIdx.x * kStBlock + threadIdx.x;
    if (i >= a.nq) return;
    double re[L + 1], im[L + 1];
#pragma unroll
    for (int m = 0; m <= L; ++m) re[m] = im[m] = 0.0;
    long long e0 = a.offsets[i], e1 = a.offsets[i + 1];
    if (e0 < 0 || e1 < e0 || e1 > a.capacity) {
        atomicOr(a.status, kStatusBadList);
        e0 = e1 = 0;
    }
    const float* qp = a.qpts + 3 * i;
    const double qx = qp[0], qy = qp[1], qz = a.dim == 3 ? (double)qp[2] : 0.0;
    int nb = 0;
    for (long long e = e0; e < e1; ++e) {
        const int j = a.idx[e];
        if (j < 0 || (long long)j >= a.n) {
            atomicOr(a.status, kStatusBadList);
            continue;
        }
        const float* pp = a.pts + 3 * (long long)j;
        double d[3] = {(double)pp[0] - qx, (double)pp[1] - qy,
                       a.dim == 3 ? (double)pp[2] - qz : 0.0};
        // minimum image: fractional displacement rounded to the nearest image
        double s[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            s[k] = rint(a.minv[k][0] * d[0] + a.minv[k][1] * d[1] + a.minv[k][2] * d[2]);
        if (a.dim != 3) s[2] = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] -= a.m[k][0] * s[0] + a.m[k][1] * s[1] + a.m[k][2] * s[2];
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!isfinite(r2)) {
            atomicOr(a.status, kStatusNonFinite);
            continue;
        }
        if (r2 == 0.0) continue;
        ++nb;
        const double inv_r = 1.0 / sqrt(r2);
        const double x = d[2] * inv_r;                     // cos(theta)
        const double ur = d[0] * inv_r, ui = d[1] * inv_r; // sin(theta) e^{i phi}
        // sectoral term times e^{i m phi}: c_m (sin(theta) e^{i phi})^m, with the
        // normalised P_m^m = c_m sin^m(theta) (Condon-Shortley phase)
        double cr = kInvSqrt4Pi, ci = 0.0;
#pragma unroll
        for (int m = 0; m <= L; ++m) {
            if (m > 0) {
                const double f = -sqrt((2.0 * m + 1.0) / (2.0 * m));
                const double t = cr * ur - ci * ui;
                ci = f * (cr * ui + ci * ur);
                cr = f * t;
            }
            // P_L^m / P_m^m by the upward recurrence in l (linear in P_m^m)
            double ratio = 1.0;
            if (L > m) {
                double p0 = 1.0;
                double p1 = sqrt(2.0 * m + 3.0) * x;
#pragma unroll
                for (int l = m + 2; l <= L; ++l) {
                    const double al = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
                    const double bl = sqrt(((double)(l - 1) * (l - 1) - (double)m * m) /
                                           (4.0 * (l - 1) * (l - 1) - 1.0));
                    const double p2 = al * (x * p1 - bl * p0);
                    p0 = p1;
                    p1 = p2;
                }
                ratio = p1;
            }
            re[m] += ratio * cr;
            im[m] += ratio * ci;
        }
    }
    double s2 = re[0] * re[0] + im[0] * im[0];
#pragma unroll
    for (int m = 1; m <= L; ++m) s2 += 2.0 * (re[m] * re[m] + im[m] * im[m]);
    a.ql[i] = nb > 0 ? sqrt(4.0 * M_PI / (2.0 * L + 1.0) * s2) / nb : 0.0;
    if (a.wl) {
        // the lane's q_lm (m >= 0) in LDS, then the 3j sum over m1 + m2 + m3 = 0
        extern __shared__ double2 s_q[];
        double2* q = s_q + threadIdx.x * (L + 1);
#pragma unroll
        for (int m = 0; m <= L; ++m) q[m] = make_double2(re[m], im[m]);
        constexpr int W = 2 * L + 1;
        double w = 0.0;
        for (int m1 = -L; m1 <= L; ++m1) {
            const double2 a1 = q_of(q, m1);
            const int lo = m1 < 0 ? -L - m1 : -L, hi = m1 < 0 ? L : L - m1;
            for (int m2 = lo; m2 <= hi; ++m2) {
                const double2 a2 = q_of(q, m2), a3 = q_of(q, -m1 - m2);
                // real part of the triple product
                const double pr = a1.x * a2.x - a1.y * a2.y, pi = a1.x * a2.y + a1.y * a2.x;
                w += a.w3j[(m1 + L) * W + (m2 + L)] * (pr * a3.x - pi * a3.y);
            }
        }
        a.wl[i] = (nb > 0 && s2 > 0.0) ? w / (s2 * sqrt(s2)) : 0.0;
    }
}

template <int L>
void launch_l(const SteinArgs& a, hipStream_t s)
{
    const int blocks = (int)((a.nq + kStBlock - 1) / kStBlock);
    const size_t lds = a.wl ? sizeof(double2) * kStBlock * (L + 1) : 0;
    hipLaunchKernelGGL(steinhardt_kernel<L>, dim3(blocks), dim3(kStBlock), lds, s, a);
}

}  // namespace

void launch_steinhardt_setup(int l, bool want_w, double* table, unsigned* status, hipStream_t s)
{
    const int w = 2 * l + 1;
    const int blocks = want_w ? (w * w + 255) / 256 : 1;
    hipLaunchKernelGGL(steinhardt_setup_kernel, dim3(blocks), dim3(256), 0, s, l, want_w ? 1 : 0,
                       table, status);
}

void launch_steinhardt(const SteinArgs& a, hipStream_t s)
{
    if (a.nq == 0) return;
    switch (a.l) {
#define PPA_L(N) \
    case N: launch_l<N>(a, s); break;
        PPA_L(0) PPA_L(1) PPA_L(2) PPA_L(3) PPA_L(4) PPA_L(5) PPA_L(6)
        PPA_L(7) PPA_L(8) PPA_L(9) PPA_L(10) PPA_L(11) PPA_L(12)
#undef PPA_L
    default: break;
    }
}

}  // namespace ppa
