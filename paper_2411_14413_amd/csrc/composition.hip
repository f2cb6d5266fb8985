// composition.hip -- from deposition profiles to at.% and back.
//
// The paper converts the simulated arrival fraction of each element into a
// composition by weighting it with the element's sputter rate, which is linear in
// the cathode power, and then with its nominal bulk density over atomic mass
// (Introduction, and the calculation paragraph closing Methods).  The accuracy
// measure is the Euclidean distance d_e of compositions (Results).  With
//   w[b,k] = (a_k P[b,k] + bb_k) rho_k / (M_k fref_k),  y = w[b,k] f[k,j],
//   c[b,j,k] = 100 y[b,j,k] / S[b,j],  S = sum_k y[b,j,k],
// the backward pass is
//   gy[b,j,m] = (100 gc[b,j,m] - sum_k gc[b,j,k] c[b,j,k]) / S[b,j]
//   gw[b,m]   = sum_j gy[b,j,m] f[m,j]          gf[m,j] = sum_b gy[b,j,m] w[b,m]
//   gP = gw a rho/(M fref); ga = sum_b gw P rho/(M fref); gb = sum_b gw rho/(M fref);
//   grho = sum_b gw w/rho; gM = -sum_b gw w/M; gfref = -sum_b gw w/fref.
// Every reduction is a fixed-order tree in LDS: results are deterministic.
#include <hip/hip_runtime.h>

#include "spx_host.hpp"

namespace spx {

constexpr int KMAX = 16;

__device__ __forceinline__ float weight(const float* a, const float* bb, const float* P, const float* M,
                                        const float* rho, const float* fref, int b, int k, int K)
{
    return (a[k] * P[(size_t)b * K + k] + bb[k]) * rho[k] / (M[k] * fref[k]);
}

__global__ void k_comp_forward(const float* __restrict__ f, const float* __restrict__ a, const float* __restrict__ bb,
                               const float* __restrict__ P, const float* __restrict__ M,
                               const float* __restrict__ rho, const float* __restrict__ fref, float* __restrict__ c,
                               int B, int J, int K)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * J) return;
    const int b = (int)(idx / J), j = (int)(idx - (int64_t)b * J);
    float y[KMAX];
    float S = 0.f;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K) {
            y[k] = weight(a, bb, P, M, rho, fref, b, k, K) * f[(size_t)k * J + j];
            S += y[k];
        }
    }
    const float inv = 100.f / S;
    float* out = c + (size_t)idx * K;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < K) out[k] = y[k] * inv;
}

// gy for one (b, j): returns S and fills gy[k]
__device__ __forceinline__ void comp_gy(const float* f, const float* a, const float* bb, const float* P,
                                        const float* M, const float* rho, const float* fref, const float* gc, int b,
                                        int j, int J, int K, float* w, float* gy)
{
    float y[KMAX];
    float S = 0.f;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K) {
            w[k] = weight(a, bb, P, M, rho, fref, b, k, K);
            y[k] = w[k] * f[(size_t)k * J + j];
            S += y[k];
        }
    }
    const float* g = gc + ((size_t)b * J + j) * K;
    float dotgc = 0.f;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < K) dotgc += g[k] * (100.f * y[k] / S);
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < K) gy[k] = (100.f * g[k] - dotgc) / S;
}

template <int NT> __device__ __forceinline__ float block_sum(float v, float* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

// One block per batch row b: gw[b, m] = sum_j gy[b,j,m] f[m,j], written to gP (scratch).
template <int NT>
__global__ void __launch_bounds__(NT) k_comp_bw_w(const float* f, const float* a, const float* bb, const float* P,
                                                  const float* M, const float* rho, const float* fref,
                                                  const float* gc, float* gw_out, int B, int J, int K)
{
    __shared__ float sh[NT];
    const int b = blockIdx.x;
    float part[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) part[k] = 0.f;
    for (int j = threadIdx.x; j < J; j += NT) {
        float w[KMAX], gy[KMAX];
        comp_gy(f, a, bb, P, M, rho, fref, gc, b, j, J, K, w, gy);
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < K) part[k] += gy[k] * f[(size_t)k * J + j];
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K) {   // uniform across the block
            const float s = block_sum<NT>(part[k], sh);
            if (threadIdx.x == 0) gw_out[(size_t)b * K + k] = s;
        }
    }
}

// One block per area j: gf[m, j] = sum_b gy[b,j,m] w[b,m].
template <int NT>
__global__ void __launch_bounds__(NT) k_comp_bw_f(const float* f, const float* a, const float* bb, const float* P,
                                                  const float* M, const float* rho, const float* fref,
                                                  const float* gc, float* gf, int B, int J, int K)
{
    __shared__ float sh[NT];
    const int j = blockIdx.x;
    float part[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) part[k] = 0.f;
    for (int b = threadIdx.x; b < B; b += NT) {
        float w[KMAX], gy[KMAX];
        comp_gy(f, a, bb, P, M, rho, fref, gc, b, j, J, K, w, gy);
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < K) part[k] += gy[k] * w[k];
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K) {   // uniform across the block
            const float s = block_sum<NT>(part[k], sh);
            if (threadIdx.x == 0) gf[(size_t)k * J + j] = s;
        }
    }
}

// One block per element m: reductions over b of gw (held in gP), then gP in place.
template <int NT>
__global__ void __launch_bounds__(NT) k_comp_bw_params(const float* a, const float* bb, const float* P,
                                                       const float* M, const float* rho, const float* fref,
                                                       float* gP, float* ga, float* gb, float* gM, float* grho,
                                                       float* gfref, int B, int K)
{
    __shared__ float sh[NT];
    const int m = blockIdx.x;
    const float q = rho[m] / (M[m] * fref[m]);
    float sa = 0.f, sb = 0.f, sw = 0.f;
    for (int b = threadIdx.x; b < B; b += NT) {
        const float gw = gP[(size_t)b * K + m];
        const float Pm = P[(size_t)b * K + m];
        const float w = (a[m] * Pm + bb[m]) * q;
        sa += gw * Pm;
        sb += gw;
        sw += gw * w;
    }
    const float Sa = block_sum<NT>(sa, sh);
    const float Sb = block_sum<NT>(sb, sh);
    const float Sw = block_sum<NT>(sw, sh);
    if (threadIdx.x == 0) {
        ga[m] = Sa * q;
        gb[m] = Sb * q;
        grho[m] = Sw / rho[m];
        gM[m] = -Sw / M[m];
        gfref[m] = -Sw / fref[m];
    }
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += NT) gP[(size_t)b * K + m] *= a[m] * q;
}

template <int NT>
__global__ void __launch_bounds__(NT) k_sqdist(const float* c, const float* ct, int Bt, const float* gloss,
                                               float* loss, float* gc, int J, int K)
{
    __shared__ float sh[NT];
    const int b = blockIdx.x;
    const size_t n = (size_t)J * K;
    const float* cb = c + (size_t)b * n;
    const float* tb = ct + (Bt == 1 ? 0 : (size_t)b * n);
    const float gl = gloss ? gloss[b] : 1.f;
    float s = 0.f;
    for (size_t i = threadIdx.x; i < n; i += NT) {
        const float d = cb[i] - tb[i];
        s += d * d;
        if (gc) gc[(size_t)b * n + i] = 2.f * d * gl;
    }
    const float tot = block_sum<NT>(s, sh);
    if (threadIdx.x == 0 && loss) loss[b] = tot;
}

// Area average: one thread per (profile, area).
__global__ void k_area_gather(const double* __restrict__ prof, int n_prof, int nu, int nv, double half_u,
                              double half_v, const double* __restrict__ cen, int n_areas, double hw,
                              double* __restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_prof * n_areas) return;
    const int p = (int)(idx / n_areas), ai = (int)(idx - (int64_t)p * n_areas);
    const double du = 2.0 * half_u / nu, dv = 2.0 * half_v / nv;
    const double cu = cen[2 * ai], cv = cen[2 * ai + 1];
    int iu0 = (int)floor((cu - hw + half_u) / du), iu1 = (int)floor((cu + hw + half_u) / du);
    int iv0 = (int)floor((cv - hw + half_v) / dv), iv1 = (int)floor((cv + hw + half_v) / dv);
    iu0 = iu0 < 0 ? 0 : iu0;
    iv0 = iv0 < 0 ? 0 : iv0;
    iu1 = iu1 > nu - 1 ? nu - 1 : iu1;
    iv1 = iv1 > nv - 1 ? nv - 1 : iv1;
    const double* pr = prof + (size_t)p * nu * nv;
    double sw = 0.0, s = 0.0;
    for (int iv = iv0; iv <= iv1; ++iv) {
        const double v0 = -half_v + iv * dv;
        const double ov = fmin(v0 + dv, cv + hw) - fmax(v0, cv - hw);
        if (ov <= 0.0) continue;
        for (int iu = iu0; iu <= iu1; ++iu) {
            const double u0 = -half_u + iu * du;
            const double ou = fmin(u0 + du, cu + hw) - fmax(u0, cu - hw);
            if (ou <= 0.0) continue;
            const double w = ou * ov;
            sw += w;
            s += w * pr[(size_t)iv * nu + iu];
        }
    }
    out[idx] = sw > 0.0 ? s / sw : 0.0;
}

}  // namespace spx

using namespace spx;

extern "C" int spx_comp_forward(const float* d_f, const float* d_a, const float* d_b, const float* d_P,
                                const float* d_M, const float* d_rho, const float* d_fref, float* d_c, int32_t B,
                                int32_t J, int32_t K, void* stream)
{
    if (B <= 0 || J <= 0 || K <= 0 || K > KMAX) {
        set_error("spx_comp_forward: need B, J > 0 and 0 < K <= 16");
        return SPX_EINVAL;
    }
    if (!d_f || !d_a || !d_b || !d_P || !d_M || !d_rho || !d_fref || !d_c) {
        set_error("spx_comp_forward: null pointer");
        return SPX_EINVAL;
    }
    const int64_t n = (int64_t)B * J;
    hipLaunchKernelGGL(k_comp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_f,
                       d_a, d_b, d_P, d_M, d_rho, d_fref, d_c, B, J, K);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

extern "C" int spx_comp_backward(const float* d_f, const float* d_a, const float* d_b, const float* d_P,
                                 const float* d_M, const float* d_rho, const float* d_fref, const float* d_gc,
                                 float* d_gf, float* d_ga, float* d_gb, float* d_gP, float* d_gM, float* d_grho,
                                 float* d_gfref, int32_t B, int32_t J, int32_t K, void* stream)
{
    if (B <= 0 || J <= 0 || K <= 0 || K > KMAX) {
        set_error("spx_comp_backward: need B, J > 0 and 0 < K <= 16");
        return SPX_EINVAL;
    }
    if (!d_f || !d_a || !d_b || !d_P || !d_M || !d_rho || !d_fref || !d_gc || !d_gf || !d_ga || !d_gb || !d_gP ||
        !d_gM || !d_grho || !d_gfref) {
        set_error("spx_comp_backward: null pointer");
        return SPX_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_comp_bw_w<256>, dim3(B), dim3(256), 0, st, d_f, d_a, d_b, d_P, d_M, d_rho, d_fref, d_gc,
                       d_gP, B, J, K);
    hipLaunchKernelGGL(k_comp_bw_f<256>, dim3(J), dim3(256), 0, st, d_f, d_a, d_b, d_P, d_M, d_rho, d_fref, d_gc,
                       d_gf, B, J, K);
    hipLaunchKernelGGL(k_comp_bw_params<256>, dim3(K), dim3(256), 0, st, d_a, d_b, d_P, d_M, d_rho, d_fref, d_gP,
                       d_ga, d_gb, d_gM, d_grho, d_gfref, B, K);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

extern "C" int spx_comp_sqdist(const float* d_c, const float* d_ct, int32_t B_t, const float* d_gloss, float* d_loss,
                               float* d_gc, int32_t B, int32_t J, int32_t K, void* stream)
{
    if (B <= 0 || J <= 0 || K <= 0 || (B_t != 1 && B_t != B) || !d_c || !d_ct || (!d_loss && !d_gc)) {
        set_error("spx_comp_sqdist: invalid arguments");
        return SPX_EINVAL;
    }
    hipLaunchKernelGGL(k_sqdist<256>, dim3(B), dim3(256), 0, (hipStream_t)stream, d_c, d_ct, B_t, d_gloss, d_loss,
                       d_gc, J, K);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

extern "C" int spx_area_gather(const double* d_profiles, int32_t n_prof, int32_t nu, int32_t nv, double half_u,
                               double half_v, const double* d_centres, int32_t n_areas, double half_width,
                               double* d_out, void* stream)
{
    if (!d_profiles || !d_centres || !d_out || n_prof <= 0 || nu <= 0 || nv <= 0 || n_areas <= 0 ||
        !(half_u > 0) || !(half_v > 0) || !(half_width > 0)) {
        set_error("spx_area_gather: invalid arguments");
        return SPX_EINVAL;
    }
    const int64_t n = (int64_t)n_prof * n_areas;
    hipLaunchKernelGGL(k_area_gather, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, (hipStream_t)stream,
                       d_profiles, n_prof, nu, nv, half_u, half_v, d_centres, n_areas, half_width, d_out);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}
