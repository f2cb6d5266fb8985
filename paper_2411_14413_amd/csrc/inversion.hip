// inversion.hip -- recovering a geometry parameter from a sweep of simulated libraries.
//
// The cathode-tilt study of the Results repeats the simulation over a range of tilts and
// compares every simulated library with the measured one, by the compositional area it covers
// (Figure 8: for a ternary library, the area of the convex hull of its compositions in the
// ternary diagram) and by d_e.  After the transport of the whole sweep in one launch and the
// area gather, three kernels finish the inversion on the device:
//   k_sweep_composition  at.% of each sweep point's library, normalised by its own calibration
//                        value (the mean of its area values), in double;
//   k_hull_area          covered area of each ternary library: the points are sorted in LDS
//                        (bitonic), then one lane walks Andrew's monotone chain;
//   k_sweep_fit          the sweep value that minimises a misfit, or at which a curve reaches a
//                        target.
// Decisions (the hull's turns, the bracket of a fit) are taken in double with contraction off,
// so that they are the plain IEEE operations a reader would write down.
#include <hip/hip_runtime.h>

#include <cmath>

#include "spx_host.hpp"

namespace spx {

constexpr int SWEEP_KMAX = 16;
constexpr int HULL_JMAX = 2048;
constexpr int FIT_TMAX = 256;
constexpr double SQRT3 = 1.7320508075688772;   // sqrt(3) rounded to double

// ---- compositions of a sweep -----------------------------------------------------------
// One workgroup per sweep point t.  fref[k] = (sum_j f[t,k,j]) / J with a fixed reduction
// order (per-lane strided sums, then a tree over lanes and waves), so results are repeatable.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_sweep_composition(const double* __restrict__ f,
                                                               const double* __restrict__ a,
                                                               const double* __restrict__ bb,
                                                               const double* __restrict__ P,
                                                               const double* __restrict__ M,
                                                               const double* __restrict__ rho,
                                                               float* __restrict__ c, int J, int K)
{
    __shared__ double red[THREADS];
    __shared__ double w[SWEEP_KMAX];
    const int t = blockIdx.x, tid = threadIdx.x;
    const double* ft = f + (size_t)t * K * J;
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int j = tid; j < J; j += THREADS) s += ft[(size_t)k * J + j];
        red[tid] = s;
        __syncthreads();
        for (int h = THREADS / 2; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        if (tid == 0) {
            const double fref = red[0] / (double)J;
            w[k] = (a[k] * P[k] + bb[k]) * rho[k] / (M[k] * fref);
        }
        __syncthreads();
    }
    for (int j = tid; j < J; j += THREADS) {
        double y[SWEEP_KMAX];
        double S = 0.0;
#pragma unroll
        for (int k = 0; k < SWEEP_KMAX; ++k)
            if (k < K) {
                y[k] = w[k] * ft[(size_t)k * J + j];
                S += y[k];
            }
        float* out = c + ((size_t)t * J + j) * K;
#pragma unroll
        for (int k = 0; k < SWEEP_KMAX; ++k)
            if (k < K) out[k] = (float)(100.0 * y[k] / S);
    }
}

// ---- covered area of a ternary library ---------------------------------------------------
#pragma clang fp contract(off)
__device__ __forceinline__ double turn(double ox, double oy, double ax, double ay, double bx, double by)
{
    return (ax - ox) * (by - oy) - (ay - oy) * (bx - ox);
}

__device__ __forceinline__ bool key_less(double x0, double y0, double x1, double y1)
{
    return x0 < x1 || (x0 == x1 && y0 < y1);
}

// One workgroup per library.  Points go to LDS in ternary-diagram coordinates, padded to a
// power of two with +inf, and are sorted by (x, y) with a bitonic network; lane 0 then builds
// the lower and the upper chain (index stacks in LDS) and sums the shoelace over the hull in
// the order lower chain, then upper chain.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_hull_area(const float* __restrict__ c, int J, float* __restrict__ area)
{
    __shared__ double px[HULL_JMAX], py[HULL_JMAX];
    __shared__ int16_t lo[HULL_JMAX], up[HULL_JMAX];
    const int b = blockIdx.x, tid = threadIdx.x;
    int n = 1;
    while (n < J) n <<= 1;
    const float* cb = c + (size_t)b * J * 3;
    for (int j = tid; j < n; j += THREADS) {
        if (j < J) {
            const double c1 = (double)cb[3 * j + 1], c2 = (double)cb[3 * j + 2];
            px[j] = c1 + 0.5 * c2;
            py[j] = c2 * (SQRT3 / 2.0);
        } else {
            px[j] = INFINITY;
            py[j] = INFINITY;
        }
    }
    __syncthreads();
    for (int size = 2; size <= n; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < n / 2; i += THREADS) {
                const int lo_i = 2 * i - (i & (stride - 1));          // first of the pair
                const int hi_i = lo_i + stride;
                const bool up_dir = (lo_i & size) == 0;
                const double x0 = px[lo_i], y0 = py[lo_i], x1 = px[hi_i], y1 = py[hi_i];
                const bool swap = up_dir ? key_less(x1, y1, x0, y0) : key_less(x0, y0, x1, y1);
                if (swap) {
                    px[lo_i] = x1;
                    py[lo_i] = y1;
                    px[hi_i] = x0;
                    py[hi_i] = y0;
                }
            }
            __syncthreads();
        }
    if (tid != 0) return;
    if (J < 3) {
        area[b] = 0.f;
        return;
    }
    int nl = 0, nu = 0;
    for (int i = 0; i < J; ++i) {
        while (nl >= 2 && turn(px[lo[nl - 2]], py[lo[nl - 2]], px[lo[nl - 1]], py[lo[nl - 1]], px[i], py[i]) <= 0.0)
            --nl;
        lo[nl++] = (int16_t)i;
    }
    for (int i = J - 1; i >= 0; --i) {
        while (nu >= 2 && turn(px[up[nu - 2]], py[up[nu - 2]], px[up[nu - 1]], py[up[nu - 1]], px[i], py[i]) <= 0.0)
            --nu;
        up[nu++] = (int16_t)i;
    }
    // hull = lower chain without its last point, then upper chain without its last point
    const int nh = (nl - 1) + (nu - 1);
    double s = 0.0;
    for (int h = 0; h < nh; ++h) {
        const int i0 = h < nl - 1 ? lo[h] : up[h - (nl - 1)];
        const int h1 = h + 1 == nh ? 0 : h + 1;
        const int i1 = h1 < nl - 1 ? lo[h1] : up[h1 - (nl - 1)];
        s += px[i0] * py[i1] - px[i1] * py[i0];
    }
    area[b] = (float)(0.5 * s / (SQRT3 / 4.0 * 100.0 * 100.0));
}

// ---- fit over a sweep ----------------------------------------------------------------------
struct SweepX {
    double x[FIT_TMAX];
};

// Sweep values as u = (x - mean) / half-range in [-1, 1]; curves are centred on their mean, so a
// flat curve fits exactly zero.  Sums run over t in ascending order.
__device__ void sweep_coords(const SweepX& X, int T, double& xm, double& h)
{
    double sx = 0.0;
    for (int t = 0; t < T; ++t) sx += X.x[t];
    xm = sx / (double)T;
    h = 0.5 * (X.x[T - 1] - X.x[0]);
}

__device__ double mean_of(const float* y, int T)
{
    double s = 0.0;
    for (int t = 0; t < T; ++t) s += (double)y[t];
    return s / (double)T;
}

// Least-squares parabola y - mean(y) ~ p0 + p1 u + p2 u^2 (normal equations, Cramer's rule);
// its vertex if it opens upwards, kept inside the sweep, else the smallest sample.
__device__ double fit_min(const SweepX& X, const float* y, int T)
{
    int i = 0;
    for (int t = 1; t < T; ++t)
        if ((double)y[t] < (double)y[i]) i = t;
    if (T < 3) return X.x[i];
    double xm, h;
    sweep_coords(X, T, xm, h);
    const double ym = mean_of(y, T);
    double S[5] = {0, 0, 0, 0, 0}, Y[3] = {0, 0, 0};
    for (int t = 0; t < T; ++t) {
        const double u = (X.x[t] - xm) / h, yc = (double)y[t] - ym;
        double uk = 1.0;
        for (int k = 0; k < 5; ++k) {
            S[k] += uk;
            if (k < 3) Y[k] += yc * uk;
            uk *= u;
        }
    }
    // | S0 S1 S2 |       | Y0 |
    // | S1 S2 S3 | p  =  | Y1 |
    // | S2 S3 S4 |       | Y2 |
    const double c00 = S[2] * S[4] - S[3] * S[3], c01 = S[1] * S[4] - S[3] * S[2], c02 = S[1] * S[3] - S[2] * S[2];
    const double det = S[0] * c00 - S[1] * c01 + S[2] * c02;
    const double d1 = S[0] * (Y[1] * S[4] - S[3] * Y[2]) - Y[0] * c01 + S[2] * (S[1] * Y[2] - Y[1] * S[2]);
    const double d2 = S[0] * (S[2] * Y[2] - Y[1] * S[3]) - S[1] * (S[1] * Y[2] - Y[1] * S[2]) + Y[0] * c02;
    const double p1 = d1 / det, p2 = d2 / det;
    if (!(p2 > 0.0)) return X.x[i];
    const double v = xm - h * p1 / (2.0 * p2);
    return fmin(fmax(v, X.x[0]), X.x[T - 1]);
}

// Least-squares line through the samples; where it reaches the target, NaN outside the sweep
// or for a flat line.
__device__ double fit_match(const SweepX& X, const float* y, int T, double target)
{
    if (T < 2) return NAN;
    double xm, h;
    sweep_coords(X, T, xm, h);
    const double ym = mean_of(y, T);
    double su = 0.0;
    for (int t = 0; t < T; ++t) su += (X.x[t] - xm) / h;
    const double um = su / (double)T;
    double sxy = 0.0, sxx = 0.0;
    for (int t = 0; t < T; ++t) {
        const double uc = (X.x[t] - xm) / h - um;
        sxy += uc * ((double)y[t] - ym);
        sxx += uc * uc;
    }
    const double q1 = sxy / sxx;
    if (q1 == 0.0) return NAN;
    const double v = xm + h * (um + (target - ym) / q1);
    return (v >= X.x[0] && v <= X.x[T - 1]) ? v : NAN;
}

__global__ __launch_bounds__(64) void k_sweep_fit(SweepX X, const float* __restrict__ y, int B, int T, int mode,
                                                  const float* __restrict__ target, double* __restrict__ out)
{
    for (int b = threadIdx.x; b < B; b += 64)
        out[b] = mode == SPX_FIT_MIN ? fit_min(X, y + (size_t)b * T, T)
                                     : fit_match(X, y + (size_t)b * T, T, (double)target[b]);
}
#pragma clang fp contract(on)

}  // namespace spx

using namespace spx;

extern "C" int spx_sweep_composition(const double* d_f, const double* d_a, const double* d_b, const double* d_P,
                                     const double* d_M, const double* d_rho, float* d_c, int32_t T, int32_t J,
                                     int32_t K, void* stream)
{
    if (T <= 0 || J <= 0 || K <= 0 || K > SWEEP_KMAX) {
        set_error("spx_sweep_composition: need T, J > 0 and 0 < K <= 16");
        return SPX_EINVAL;
    }
    if (!d_f || !d_a || !d_b || !d_P || !d_M || !d_rho || !d_c) {
        set_error("spx_sweep_composition: null pointer");
        return SPX_EINVAL;
    }
    hipLaunchKernelGGL(k_sweep_composition<256>, dim3(T), dim3(256), 0, (hipStream_t)stream, d_f, d_a, d_b, d_P, d_M,
                       d_rho, d_c, J, K);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

extern "C" int spx_hull_area(const float* d_c, int32_t B, int32_t J, float* d_area, void* stream)
{
    if (B <= 0 || J <= 0 || J > HULL_JMAX || !d_c || !d_area) {
        set_error("spx_hull_area: need B > 0, 0 < J <= 2048 and non-null pointers");
        return SPX_EINVAL;
    }
    hipLaunchKernelGGL(k_hull_area<256>, dim3(B), dim3(256), 0, (hipStream_t)stream, d_c, J, d_area);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

extern "C" int spx_sweep_fit(const double* h_x, const float* d_y, int32_t B, int32_t T, int32_t mode,
                             const float* d_target, double* d_xfit, void* stream)
{
    if (B <= 0 || T <= 0 || T > FIT_TMAX || !h_x || !d_y || !d_xfit) {
        set_error("spx_sweep_fit: need B > 0, 0 < T <= 256 and non-null pointers");
        return SPX_EINVAL;
    }
    if (mode != SPX_FIT_MIN && mode != SPX_FIT_MATCH) {
        set_error("spx_sweep_fit: unknown mode");
        return SPX_EINVAL;
    }
    if (mode == SPX_FIT_MATCH && !d_target) {
        set_error("spx_sweep_fit: SPX_FIT_MATCH needs targets");
        return SPX_EINVAL;
    }
    SweepX X{};
    for (int t = 0; t < T; ++t) {
        if (!std::isfinite(h_x[t]) || (t > 0 && !(h_x[t] > h_x[t - 1]))) {
            set_error("spx_sweep_fit: sweep values must be finite and strictly increasing");
            return SPX_EINVAL;
        }
        X.x[t] = h_x[t];
    }
    hipLaunchKernelGGL(k_sweep_fit, dim3(1), dim3(64), 0, (hipStream_t)stream, X, d_y, B, T, mode, d_target, d_xfit);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}
