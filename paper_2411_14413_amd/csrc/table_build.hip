// table_build.hip -- FP64 scattering-angle and cross-section tables on the GPU.
//
// The paper names a screened-Coulomb interaction with Moliere screening for the
// collisions of sputtered atoms with the gas (closing calculation paragraph of
// Methods).  In reduced units x = r/a, beta = b/a, eps = a E_r/(Z1 Z2 e^2) the
// classical centre-of-mass deflection is
//     theta = pi - 2 (beta/x0) Int_0^1 du / sqrt(h(u)),
//     h(u) = 1 - u Phi(x0/u)/(x0 eps) - beta^2 u^2/x0^2,
// with x0 the distance of closest approach (h(1) = 0).  Substituting u = cos(psi)
// turns the integral into Int_0^{pi/2} sqrt(sin^2 psi / h(cos psi)) d psi, whose
// integrand is smooth with vanishing odd derivatives at both ends for a screened
// potential, so the midpoint rule in psi converges faster than any power of 1/N.
// The table depends only on (eps, b/b_max): one table serves every species pair.
#include <hip/hip_runtime.h>
#include <math.h>

#include "spx_host.hpp"

namespace spx {

__device__ __forceinline__ double moliere(double x)
{
    return 0.35 * exp(-0.3 * x) + 0.55 * exp(-1.2 * x) + 0.10 * exp(-6.0 * x);
}

// h(1) as a function of x: 1 - Phi(x)/(x eps) - beta^2/x^2 (increasing in x).
__device__ __forceinline__ double f_root(double x, double eps, double beta)
{
    return 1.0 - moliere(x) / (x * eps) - beta * beta / (x * x);
}

__device__ double closest_approach(double eps, double beta)
{
    double lo = beta, hi = beta > 1.0 ? beta : 1.0;
    for (int k = 0; k < 2100 && f_root(hi, eps, beta) <= 0.0; ++k) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (f_root(mid, eps, beta) > 0.0) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

__device__ double theta_cm(double eps, double beta, int nq)
{
    if (beta <= 0.0) return M_PI;
    const double x0 = closest_approach(eps, beta);
    const double ib = beta / x0;
    const double dpsi = 0.5 * M_PI / nq;
    double sum = 0.0;
    for (int k = 0; k < nq; ++k) {
        double sp, cp;
        sincos((k + 0.5) * dpsi, &sp, &cp);
        const double u = cp;
        double h = 1.0 - u * moliere(x0 / u) / (x0 * eps) - ib * ib * u * u;
        h = h > 1e-300 ? h : 1e-300;
        sum += sqrt(sp * sp / h);
    }
    return M_PI - 2.0 * ib * sum * dpsi;
}

__global__ void k_betamax(int ne, double lo, double hi, double theta_min, int nq, double* betamax)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const double eps = pow(10.0, lo + (hi - lo) * (double)i / (double)(ne - 1));
    double blo = 0.0, bhi = 1.0;
    for (int k = 0; k < 64 && theta_cm(eps, bhi, nq) > theta_min; ++k) {
        blo = bhi;
        bhi *= 2.0;
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (blo + bhi);
        if (mid <= blo || mid >= bhi) break;
        if (theta_cm(eps, mid, nq) > theta_min) blo = mid; else bhi = mid;
    }
    betamax[i] = 0.5 * (blo + bhi);
}

__global__ void k_theta(int ne, int ns, double lo, double hi, int nq, const double* betamax, double* theta)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * ns) return;
    const int i = idx / ns, j = idx - i * ns;
    const double eps = pow(10.0, lo + (hi - lo) * (double)i / (double)(ne - 1));
    const double s = (double)j / (double)(ns - 1);
    theta[idx] = (j == 0) ? M_PI : theta_cm(eps, s * betamax[i], nq);
}

__global__ void k_narrow(const double* src, float* dst, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

int build_tables(Plan* P)
{
    const int ne = P->params.table_ne, ns = P->params.table_ns;
    const double lo = P->params.log_eps_lo, hi = P->params.log_eps_hi;
    const int nq = 512;
    hipStream_t st = P->work_stream;
    hipLaunchKernelGGL(k_betamax, dim3((ne + 63) / 64), dim3(64), 0, st, ne, lo, hi, P->params.theta_min, nq,
                       P->d_betamax64);
    SPX_HIP(hipGetLastError());
    const int n = ne * ns;
    hipLaunchKernelGGL(k_theta, dim3((n + 127) / 128), dim3(128), 0, st, ne, ns, lo, hi, nq, P->d_betamax64,
                       P->d_theta64);
    SPX_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_narrow, dim3((n + 255) / 256), dim3(256), 0, st, P->d_theta64, P->d_theta32, n);
    hipLaunchKernelGGL(k_narrow, dim3((ne + 255) / 256), dim3(256), 0, st, P->d_betamax64, P->d_betamax32, ne);
    SPX_HIP(hipGetLastError());
    P->h_betamax.resize(ne);
    SPX_HIP(hipMemcpyAsync(P->h_betamax.data(), P->d_betamax64, sizeof(double) * ne, hipMemcpyDeviceToHost, st));
    SPX_HIP(hipStreamSynchronize(st));
    return SPX_OK;
}

}  // namespace spx
