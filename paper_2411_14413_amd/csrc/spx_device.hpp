// spx_device.hpp -- device-side data layout and the per-event physics of the
// sputtered-atom transport, written once for R = float (batched transport) and
// R = double (plain comparator).
//
// Method (Thelen et al., arXiv 2411.14413, Methods, "The SIMTRA model" and the
// calculation paragraph that closes Methods): launch from the racetrack with a
// Thompson energy cut off at E_max and a cosine emission law; free path
// -lambda_m ln RN_1; nearest surface hit; otherwise an elastic collision with a gas
// atom (thermal partner velocity, Moliere-screened Coulomb deflection from a
// table, binary-collision kinematics); below the thermalisation threshold the atom
// takes isotropic exponential diffusive steps until it hits a surface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spx {

enum : int { ST_DEAD = 0, ST_BALLISTIC = 1, ST_DIFFUSIVE = 2 };
enum : int { HIT_NONE = 0, HIT_DEPOSITED = 1, HIT_WALL = 2, HIT_ESCAPED = 3 };
// C_TESTED: diffusive steps tested against the surfaces (a work counter: the batched walk tests
// only the steps that leave their clearance balls, the plain comparator every step)
enum : int { C_LAUNCHED = 0, C_DEPOSITED, C_WALL, C_ESCAPED, C_COLLISIONS, C_DIFFUSIVE, C_THERMALIZED, C_TESTED, N_COUNTERS };

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11); the key words are uniform
// across the launch, so their schedule lives in scalar registers.
// --------------------------------------------------------------------------
// Three-input XOR in one VALU instruction (gfx950 v_bitop3, truth table 0x96 = a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1, xor3((uint32_t)(p0 >> 32), c.w, k1),
                       (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// RN in ]0,1]: ((x >> 8) + 1) * 2^-24, exact in float and double.
template <typename R> __device__ __forceinline__ R u01(uint32_t x);
template <> __device__ __forceinline__ float u01<float>(uint32_t x)
{
    // (k + 1) 2^-24 with k < 2^24: exact, one fused multiply-add
    return __builtin_fmaf((float)(x >> 8), 0x1p-24f, 0x1p-24f);
}
template <> __device__ __forceinline__ double u01<double>(uint32_t x)
{
    return (double)((x >> 8) + 1u) * 0x1p-24;
}

// RN in ]0,1] from a 21-bit code k: (k + 1) * 2^-21, exact in float and double.
template <typename R> __device__ __forceinline__ R u21(uint32_t k);
template <> __device__ __forceinline__ float u21<float>(uint32_t k)
{
    return __builtin_fmaf((float)k, 0x1p-21f, 0x1p-21f);
}
template <> __device__ __forceinline__ double u21<double>(uint32_t k)
{
    return (double)(k + 1u) * 0x1p-21;
}
// 2 u21(k) - 1 = (k + 1 - 2^20) 2^-20 in [-1, 1), formed in one exact multiply-add (both the
// constant 2^-20 - 1 and the result fit the significand).
template <typename R> __device__ __forceinline__ R sym21(uint32_t k)
{
    return fma((R)k, (R)0x1p-20, (R)0x1p-20 - (R)1);
}

// A diffusive step needs three RN, so steps 2m and 2m+1 share the Philox block
// (pid, 2m, cfgcat, 2): the even step takes the top 21 bits of words x, y, z; the odd step
// the low 11 bits of word i followed by bits [10 i, 10 i + 10) of word w.
__device__ __forceinline__ uint4 diffusive_block(uint32_t pid, uint32_t e, uint32_t cfgcat, uint32_t k0, uint32_t k1)
{
    return philox4x32_10(make_uint4(pid, e & ~1u, cfgcat, 2u), k0, k1);
}
__device__ __forceinline__ void diffusive_codes(uint4 w, bool odd, uint32_t* k)
{
    if (odd) {
        k[0] = ((w.x & 0x7FFu) << 10) | (w.w & 0x3FFu);
        k[1] = ((w.y & 0x7FFu) << 10) | ((w.w >> 10) & 0x3FFu);
        k[2] = ((w.z & 0x7FFu) << 10) | ((w.w >> 20) & 0x3FFu);
    } else {
        k[0] = w.x >> 11;
        k[1] = w.y >> 11;
        k[2] = w.z >> 11;
    }
}

// --------------------------------------------------------------------------
// Math overloads for R.
// --------------------------------------------------------------------------
// FP32 uses the native VALU transcendentals (v_sqrt, v_log: log2, v_exp: exp2, v_sin and
// v_cos taking revolutions, v_rcp), each within a few ulp on the ranges used here; FP64 uses
// the correctly rounded library functions.
__device__ __forceinline__ float m_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double m_log2(double x) { return log2(x); }
__device__ __forceinline__ float m_log(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994530942f; }
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896340736f); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double m_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float m_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double m_div(double a, double b) { return a / b; }
__device__ __forceinline__ float m_ninv(float p) { return normcdfinvf(p); }
__device__ __forceinline__ double m_ninv(double p) { return normcdfinv(p); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ bool m_finite(float x) { return isfinite(x); }
__device__ __forceinline__ bool m_finite(double x) { return isfinite(x); }
// sin and cos of 2 pi u for u in ]0, 1]
__device__ __forceinline__ void m_sincos2pi(float u, float* s, float* c)
{
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
}
__device__ __forceinline__ void m_sincos2pi(double u, double* s, double* c) { sincospi(2.0 * u, s, c); }
// sin and cos of an angle in [0, pi] (radians)
__device__ __forceinline__ void m_sincos(float x, float* s, float* c)
{
    const float r = x * 0.15915494309189533577f;
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void m_sincos(double x, double* s, double* c) { sincos(x, s, c); }
template <typename R> __device__ __forceinline__ R m_inf();
template <> __device__ __forceinline__ float m_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double m_inf<double>() { return __builtin_huge_val(); }

// --------------------------------------------------------------------------
// Per-segment constants, derived on the host in double precision.
// Positions are in the chamber-centred frame: z' = z - z_mid.
// --------------------------------------------------------------------------
// One node interval of a measured racetrack: start radius r, normalised cumulative weight C
// at r, and the cubic H(t) = ((p3 t + p2) t + p1) t giving the weight of [r, r + t] for
// t <= dr (depth linear on the interval, density depth(r) r).  The last node has C = 1.
template <typename R> struct RtNode {
    R r, C, p1, p2, p3, dr;
};

// An absorbing object of a segment (chamber frame).  Planar (disc, rectangle): centre c,
// normal n, axes u, v with nc = n.c, uc = u.c, vc = v.c, half sizes hu, hv (discs: r2 = hu^2).
// Tube: axis through c along n, r2 = radius^2, length len.
template <typename R> struct ObjDev {
    int32_t kind, pad;
    R c[3], n[3], u[3], v[3];
    R nc, uc, vc;
    R hu, hv, r2, len;
};

template <typename R> struct SegDev {
    R cat_c[3], cat_n[3], cat_u[3], cat_v[3];
    R cat_R2;
    R cat_nc, cat_uc, cat_vc;             // n.c, u.c, v.c of the target
    R sub_c[3], sub_n[3], sub_u[3], sub_v[3];
    R sub_nc, sub_uc, sub_vc;             // n.c, u.c, v.c of the substrate
    R half_u, half_v, inv_du, inv_dv, sub_R2;
    R ch_R2, zlo, zhi;
    R rt_mu, rt_sig, PhiA, QB, dPhi;      // racetrack truncated normal
    const RtNode<R>* rt;                  // measured racetrack (rt_n nodes), else nullptr
    const ObjDev<R>* obj;                 // absorbing objects (n_obj), else nullptr
    R cosk[6];                            // emission law: G(mu) = sum cosk_i mu^(i+1) rises from 0 to 1
    R Us, smax;                           // Thompson inverse CDF
    R two_over_Ms, half_Ms;               // v = sqrt(2E/Ms), E = Ms v^2 / 2
    R Ms_frac, Mg_frac;                   // Ms/(Ms+Mg), Mg/(Ms+Mg)
    R half_mu_red;                        // E_r = mu |g|^2 / 2
    R xo_coll;                            // table index offset for eps = eps_per_eV * E_r
    R xo_stat;                            // ... for eps of a gas atom at rest: E_r = E Mg/(Ms+Mg)
    R n_pia2;                             // n pi a^2: n sigma = n_pia2 * beta_max^2
    R vth, inv_vg, vg;                    // Maxwellian component sd; mean-speed scale
    R E_th, lam_th;
    R lam_l2;                             // lam_th ln 2: a diffusive step is -lam_l2 log2(RN)
    R z_mid;                              // chamber-frame origin along z (world z = z' + z_mid)
    int32_t shape, nu, nv, gas_motion;
    int32_t vacuum, rt_n;
    int32_t cos_pure, n_obj;              // cos_pure: the cosine law, cos(theta) = sqrt(RN)
    uint32_t cfgcat;                      // (config << 8) | cathode: third Philox counter word
    uint32_t pad1;
    uint64_t bin_off;                     // first bin of this segment in the tally
    uint64_t first_rec;                   // first record of this segment
    uint64_t N;                           // particles
};

template <typename R> struct TabDev {
    const R* theta;    // [ne][ns]
    const R* betamax;  // [ne]
    R xs;              // index per log2(eps): (ne-1) / ((hi - lo) log2(10))
    int32_t ne, ns;
};

// Linear interpolation of beta_max at table coordinate x (clamped).
template <typename R> __device__ __forceinline__ R tab_betamax(const TabDev<R>& tb, R x)
{
    const R xmax = (R)(tb.ne - 1);
    x = (x > (R)0) ? x : (R)0;            // also maps NaN to 0
    x = (x < xmax) ? x : xmax;
    int i = (int)m_floor(x);
    i = (i < tb.ne - 2) ? i : tb.ne - 2;
    const R f = x - (R)i;
    return tb.betamax[i] * ((R)1 - f) + tb.betamax[i + 1] * f;
}

// Bilinear theta_cm at table coordinates (x along log10 eps, s = b/b_max).
template <typename R> __device__ __forceinline__ R tab_theta(const TabDev<R>& tb, R x, R s)
{
    const R xmax = (R)(tb.ne - 1), ymax = (R)(tb.ns - 1);
    x = (x > (R)0) ? x : (R)0;
    x = (x < xmax) ? x : xmax;
    int i = (int)m_floor(x);
    i = (i < tb.ne - 2) ? i : tb.ne - 2;
    const R fx = x - (R)i;
    R y = s * ymax;
    y = (y > (R)0) ? y : (R)0;
    y = (y < ymax) ? y : ymax;
    int j = (int)m_floor(y);
    j = (j < tb.ns - 2) ? j : tb.ns - 2;
    const R fy = y - (R)j;
    const R* T = tb.theta + (size_t)i * tb.ns + j;
    const R t00 = T[0], t01 = T[1], t10 = T[tb.ns], t11 = T[tb.ns + 1];
    return ((R)1 - fx) * ((R)1 - fy) * t00 + fx * ((R)1 - fy) * t10 + ((R)1 - fx) * fy * t01 + fx * fy * t11;
}

template <typename R> __device__ __forceinline__ R dot3(const R* a, const R* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Bisection steps that shrink an interval to the precision of R.
template <typename R> struct Bisect;
template <> struct Bisect<float> { static constexpr int steps = 26; };
template <> struct Bisect<double> { static constexpr int steps = 60; };

// Start radius on a measured racetrack: r = F^-1(RN) with F the normalised weight of
// [0, r]: the node interval with C_i < RN <= C_{i+1} (binary search), then bisection on the
// interval's cubic.
template <typename R> __device__ __forceinline__ R racetrack_radius(const SegDev<R>& s, R u)
{
    const RtNode<R>* T = s.rt;
    int lo = 0, hi = s.rt_n - 1;          // C[lo] < u <= C[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (T[mid].C < u) lo = mid; else hi = mid;
    }
    const RtNode<R> n = T[lo];
    const R want = u - n.C;
    R a = (R)0, b = n.dr;
    for (int it = 0; it < Bisect<R>::steps; ++it) {
        const R mid = (R)0.5 * (a + b);
        const R h = ((n.p3 * mid + n.p2) * mid + n.p1) * mid;
        if (h < want) a = mid; else b = mid;
    }
    return n.r + (R)0.5 * (a + b);
}

// cos(theta) of a general emission law: G(mu) = RN on [0, 1] by bisection.
template <typename R> __device__ __forceinline__ R emission_mu(const SegDev<R>& s, R u)
{
    R a = (R)0, b = (R)1;
    for (int it = 0; it < Bisect<R>::steps; ++it) {
        const R m = (R)0.5 * (a + b);
        const R g =
            m * (s.cosk[0] + m * (s.cosk[1] + m * (s.cosk[2] + m * (s.cosk[3] + m * (s.cosk[4] + m * s.cosk[5])))));
        if (g < u) a = m; else b = m;
    }
    return (R)0.5 * (a + b);
}

// --------------------------------------------------------------------------
// Launch (event 0): sub-block 0 -> u0..u3, sub-block 1 -> u4.
// --------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void launch(const SegDev<R>& s, uint4 r0, uint4 r1, R* x, R* d, R& E)
{
    const R u0 = u01<R>(r0.x), u1 = u01<R>(r0.y), u2 = u01<R>(r0.z), u3 = u01<R>(r0.w);
    const R u4 = u01<R>(r1.x);
    R rr;
    if (s.rt_n > 0) {
        rr = racetrack_radius(s, u0);
    } else {
        // racetrack radius: inverse CDF of the truncated normal; the upper half takes the
        // complement so that no precision is lost near 1.  One inverse-normal call on the
        // chosen argument (lanes of a wave fall on both sides; two calls in the two arms of a
        // branch would each run for the whole wave).
        const R P = s.PhiA + u0 * s.dPhi;
        const bool lower = P <= (R)0.5;
        const R Q = s.QB + ((R)1 - u0) * s.dPhi;
        const R zz = m_ninv(lower ? P : Q);
        const R z = lower ? zz : -zz;
        rr = s.rt_mu + s.rt_sig * z;
    }
    R sp, cp;
    m_sincos2pi(u1, &sp, &cp);
#pragma unroll
    for (int i = 0; i < 3; ++i) x[i] = s.cat_c[i] + rr * (cp * s.cat_u[i] + sp * s.cat_v[i]);
    // Thompson energy: [E/(E+U_s)]^2 proportional to RN up to the cut-off
    const R se = m_sqrt(u2) * s.smax;
    E = m_div(s.Us * se, (R)1 - se);
    // emission law: the cosine law inverts in closed form, cos(theta) = sqrt(RN)
    R mu, st;
    if (s.cos_pure) {
        mu = m_sqrt(u3);
        st = m_sqrt((R)1 - u3);
    } else {
        mu = emission_mu(s, u3);
        st = m_sqrt(((R)1 - mu) * ((R)1 + mu));
    }
    R sf, cf;
    m_sincos2pi(u4, &sf, &cf);
#pragma unroll
    for (int i = 0; i < 3; ++i) d[i] = mu * s.cat_n[i] + st * (cf * s.cat_u[i] + sf * s.cat_v[i]);
}

// erf(x) for x >= 0, given e = exp(-x^2).  FP32: the rational approximation of Abramowitz and
// Stegun (Handbook of Mathematical Functions, 7.1.26), erf x = 1 - t (a1 + t (a2 + ... a5 t)) e
// with t = 1 / (1 + p x), absolute error below 1.5e-7 (a few FP32 ulp near 1), which reuses the
// exponential the mean relative speed needs anyway.  FP64: the library erf.
__device__ __forceinline__ float erf_given_exp(float x, float e)
{
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, x, 1.f));
    float q = __builtin_fmaf(t, 1.061405429f, -1.453152027f);
    q = __builtin_fmaf(t, q, 1.421413741f);
    q = __builtin_fmaf(t, q, -0.284496736f);
    q = __builtin_fmaf(t, q, 0.254829592f);
    return __builtin_fmaf(-(t * q), e, 1.f);
}
__device__ __forceinline__ double erf_given_exp(double x, double) { return erf(x); }

// Mean free path at energy E.
template <typename R>
__device__ __forceinline__ R lambda_m(const SegDev<R>& s, const TabDev<R>& tb, R E)
{
    const R bm = tab_betamax(tb, m_log2(E) * tb.xs + s.xo_stat);
    const R nsig = s.n_pia2 * bm * bm;
    if (!s.gas_motion) return m_rcp(nsig);
    // moving gas: the collision rate uses the Maxwellian mean relative speed <g>(v)
    const R v = m_sqrt(E * s.two_over_Ms);
    const R xx = v * s.inv_vg;
    const R ex = m_exp(-xx * xx);
    const R g = s.vg * ((xx + m_div((R)0.5, xx)) * erf_given_exp(xx, ex) + ex * (R)0.56418958354775628695);
    return m_div(v, nsig * g);
}

struct HitF {
    int state;     // HIT_NONE / HIT_DEPOSITED / HIT_WALL
};

// Nearest surface with 0 < t <= ell; exact ties keep substrate, then cathode, then the
// absorbing objects in order, then chamber.  Planes use the precomputed n.c, u.c, v.c:
// t = (n.c - n.x)/(n.d), q.u = u.x + t u.d - u.c.  The fixed surfaces are written without
// branches (every candidate computed, then selected) so that they form one basic block: a
// wave runs them once whatever its lanes need, and the loads of the surface constants can be
// scheduled early; the objects follow in a loop uniform over the segment.  A direction
// parallel to a plane gives a reciprocal of zero, hence t = inf or NaN, which fails t > 0 as
// intended.
template <typename R>
__device__ __forceinline__ HitF hit_test(const SegDev<R>& s, const R* x, const R* d, R ell, R& t_hit, R& qu_hit,
                                         R& qv_hit, bool first)
{
    const R inf = m_inf<R>();
    // substrate plate: the front face (moving against its normal) deposits
    const R dn = dot3(d, s.sub_n);
    const R ts = (s.sub_nc - dot3(x, s.sub_n)) * m_rcp(dn);
    const R qu = dot3(x, s.sub_u) + ts * dot3(d, s.sub_u) - s.sub_uc;
    const R qv = dot3(x, s.sub_v) + ts * dot3(d, s.sub_v) - s.sub_vc;
    const bool in_s = (s.shape == 0) ? (fabs(qu) <= s.half_u && fabs(qv) <= s.half_v) : (qu * qu + qv * qv <= s.sub_R2);
    const bool hit_s = (ts > (R)0) && in_s;
    R best = hit_s ? ts : inf;
    int state = hit_s ? (dn < (R)0 ? HIT_DEPOSITED : HIT_WALL) : HIT_NONE;
    qu_hit = qu;
    qv_hit = qv;
    // emitting cathode disc (both faces absorb).  The first flight starts on the target
    // plane and a line meets a plane once, so on that flight the target is not tested.
    const R dc = dot3(d, s.cat_n);
    const R tcat = (s.cat_nc - dot3(x, s.cat_n)) * m_rcp(dc);
    const R cu = dot3(x, s.cat_u) + tcat * dot3(d, s.cat_u) - s.cat_uc;
    const R cv = dot3(x, s.cat_v) + tcat * dot3(d, s.cat_v) - s.cat_vc;
    const bool hit_c = !first && (tcat > (R)0) && (tcat < best) && (cu * cu + cv * cv <= s.cat_R2);
    best = hit_c ? tcat : best;
    state = hit_c ? HIT_WALL : state;
    // absorbing objects (both faces): a plane crossing inside the disc or rectangle; for a tube
    // the smaller positive root of |w_perp + t d_perp| = radius whose axial coordinate lies
    // in [0, len]
    for (int k = 0; k < s.n_obj; ++k) {
        const ObjDev<R>& o = s.obj[k];
        R to = inf;
        if (o.kind != 2) {
            const R dn_o = dot3(d, o.n);
            const R tp = (o.nc - dot3(x, o.n)) * m_rcp(dn_o);
            const R ou = dot3(x, o.u) + tp * dot3(d, o.u) - o.uc;
            const R ov = dot3(x, o.v) + tp * dot3(d, o.v) - o.vc;
            const bool in = (o.kind == 0) ? (ou * ou + ov * ov <= o.r2) : (fabs(ou) <= o.hu && fabs(ov) <= o.hv);
            to = (tp > (R)0 && in) ? tp : inf;
        } else {
            const R w[3] = {x[0] - o.c[0], x[1] - o.c[1], x[2] - o.c[2]};
            const R wa = dot3(w, o.n), da = dot3(d, o.n);
            const R wp[3] = {w[0] - wa * o.n[0], w[1] - wa * o.n[1], w[2] - wa * o.n[2]};
            const R dp[3] = {d[0] - da * o.n[0], d[1] - da * o.n[1], d[2] - da * o.n[2]};
            const R A = dot3(dp, dp), B = dot3(wp, dp), C = dot3(wp, wp) - o.r2;
            const R D = B * B - A * C;
            if (A > (R)0 && D >= (R)0) {
                const R sq = m_sqrt(D), ia = m_rcp(A);
                const R t1 = (-B - sq) * ia, t2 = (-B + sq) * ia;
                const R z1 = wa + t1 * da, z2 = wa + t2 * da;
                if (t1 > (R)0 && z1 >= (R)0 && z1 <= o.len) to = t1;
                else if (t2 > (R)0 && z2 >= (R)0 && z2 <= o.len) to = t2;
            }
        }
        const bool hit_o = to < best;
        best = hit_o ? to : best;
        state = hit_o ? HIT_WALL : state;
    }
    // chamber: cylinder side (stable root of |x + t d|^2 = R^2 in the xy-plane) and caps
    const R a = d[0] * d[0] + d[1] * d[1];
    const R b = x[0] * d[0] + x[1] * d[1];
    const R c = x[0] * x[0] + x[1] * x[1] - s.ch_R2;
    R disc = b * b - a * c;
    disc = disc > (R)0 ? disc : (R)0;
    const R sq = m_sqrt(disc);
    R tside = (b <= (R)0) ? (sq - b) * m_rcp(a) : -c * m_rcp(b + sq);
    tside = (a > (R)0) ? (tside > (R)0 ? tside : (R)0) : inf;
    R tcap = ((d[2] > (R)0 ? s.zhi : s.zlo) - x[2]) * m_rcp(d[2]);
    tcap = (d[2] != (R)0) ? (tcap > (R)0 ? tcap : (R)0) : inf;
    const R tch = tcap < tside ? tcap : tside;
    const bool hit_w = tch < best;
    best = hit_w ? tch : best;
    state = hit_w ? HIT_WALL : state;
    if (!(best <= ell)) state = HIT_NONE;
    t_hit = best;
    return HitF{state};
}

// Distance from x to the nearest absorbing surface the surface test knows (never more than
// the true distance): the substrate plate, the target disc and the planar objects as
// point-to-region distances, tubes as point-to-open-cylinder distances, the chamber side and
// caps.  A path that stays closer to x than this cannot
// meet any surface.
template <typename R> __device__ __forceinline__ R clearance(const SegDev<R>& s, const R* x)
{
    const R h = dot3(x, s.sub_n) - s.sub_nc;
    const R qu = dot3(x, s.sub_u) - s.sub_uc, qv = dot3(x, s.sub_v) - s.sub_vc;
    R e2;
    if (s.shape == 0) {
        const R eu = fmax(fabs(qu) - s.half_u, (R)0), ev = fmax(fabs(qv) - s.half_v, (R)0);
        e2 = eu * eu + ev * ev;
    } else {
        const R er = fmax(m_sqrt(qu * qu + qv * qv) - m_sqrt(s.sub_R2), (R)0);
        e2 = er * er;
    }
    const R d_sub2 = h * h + e2;
    const R hc = dot3(x, s.cat_n) - s.cat_nc;
    const R cu = dot3(x, s.cat_u) - s.cat_uc, cv = dot3(x, s.cat_v) - s.cat_vc;
    const R ec = fmax(m_sqrt(cu * cu + cv * cv) - m_sqrt(s.cat_R2), (R)0);
    const R d_cat2 = hc * hc + ec * ec;
    R dmin2 = fmin(d_sub2, d_cat2);
    for (int k = 0; k < s.n_obj; ++k) {
        const ObjDev<R>& o = s.obj[k];
        R d2;
        if (o.kind != 2) {
            const R ho = dot3(x, o.n) - o.nc;
            const R ou = dot3(x, o.u) - o.uc, ov = dot3(x, o.v) - o.vc;
            R e2;
            if (o.kind == 0) {
                const R er = fmax(m_sqrt(ou * ou + ov * ov) - o.hu, (R)0);
                e2 = er * er;
            } else {
                const R eu = fmax(fabs(ou) - o.hu, (R)0), ev = fmax(fabs(ov) - o.hv, (R)0);
                e2 = eu * eu + ev * ev;
            }
            d2 = ho * ho + e2;
        } else {
            // open cylinder: radial distance to the wall, plus the axial overhang past a rim
            const R w[3] = {x[0] - o.c[0], x[1] - o.c[1], x[2] - o.c[2]};
            const R wa = dot3(w, o.n);
            const R rp = m_sqrt(fmax(dot3(w, w) - wa * wa, (R)0));
            const R dr = rp - o.hu;
            const R off = fmax(fmax(-wa, wa - o.len), (R)0);
            d2 = dr * dr + off * off;
        }
        dmin2 = fmin(dmin2, d2);
    }
    const R side = m_sqrt(s.ch_R2) - m_sqrt(x[0] * x[0] + x[1] * x[1]);
    const R caps = fmin(x[2] - s.zlo, s.zhi - x[2]);
    return fmin(m_sqrt(dmin2), fmin(side, caps));
}

// Tally bin of a deposit at in-plane coordinates (qu, qv) of the substrate (clamped).
template <typename R> __device__ __forceinline__ int tally_bin(const SegDev<R>& s, R qu, R qv)
{
    int iu = (int)m_floor((qu + s.half_u) * s.inv_du);
    int iv = (int)m_floor((qv + s.half_v) * s.inv_dv);
    iu = iu < 0 ? 0 : (iu > s.nu - 1 ? s.nu - 1 : iu);
    iv = iv < 0 ? 0 : (iv > s.nv - 1 ? s.nv - 1 : iv);
    return iv * s.nu + iu;
}

// Maxwellian partner velocity from one Philox block (Box-Muller).
template <typename R> __device__ __forceinline__ void gas_velocity(const SegDev<R>& s, uint4 r, R* V)
{
    const R w0 = u01<R>(r.x), w1 = u01<R>(r.y), w2 = u01<R>(r.z), w3 = u01<R>(r.w);
    const R r0 = s.vth * m_sqrt((R)-2 * m_log(w0)), r1 = s.vth * m_sqrt((R)-2 * m_log(w2));
    R s1, c1, s3, c3;
    m_sincos2pi(w1, &s1, &c1);
    m_sincos2pi(w3, &s3, &c3);
    V[0] = r0 * c1;
    V[1] = r0 * s1;
    V[2] = r1 * c3;
}

// Elastic binary collision with a gas atom of velocity V: new direction and energy.
template <typename R>
__device__ __forceinline__ void collide(const SegDev<R>& s, const TabDev<R>& tb, R& E, R* d, const R* V, R u_b,
                                        R u_phi)
{
    const R v = m_sqrt(E * s.two_over_Ms);
    const R vv[3] = {v * d[0], v * d[1], v * d[2]};
    const R g[3] = {vv[0] - V[0], vv[1] - V[1], vv[2] - V[2]};
    const R gm2 = dot3(g, g);
    if (!(gm2 > (R)0)) return;                // no relative motion: nothing happens
    const R gm = m_sqrt(gm2);
    const R Er = s.half_mu_red * gm2;
    const R th = tab_theta(tb, m_log2(Er) * tb.xs + s.xo_coll, m_sqrt(u_b));
    R st, ct, sp, cp;
    m_sincos(th, &st, &ct);
    m_sincos2pi(u_phi, &sp, &cp);
    const R inv = m_rcp(gm);
    const R gu = g[0] * inv, gv = g[1] * inv, gw = g[2] * inv;
    R n0, n1, n2;
    if (fabs(gw) < (R)0.99999) {
        const R rho = m_sqrt(((R)1 - gw) * ((R)1 + gw));
        const R ir = m_rcp(rho);
        n0 = gu * ct + st * (gu * gw * cp - gv * sp) * ir;
        n1 = gv * ct + st * (gv * gw * cp + gu * sp) * ir;
        n2 = gw * ct - rho * st * cp;
    } else {
        n0 = st * cp;
        n1 = st * sp;
        n2 = (gw > (R)0 ? ct : -ct);
    }
    const R k = s.Mg_frac * gm;
    const R vp[3] = {s.Ms_frac * vv[0] + s.Mg_frac * V[0] + k * n0, s.Ms_frac * vv[1] + s.Mg_frac * V[1] + k * n1,
                     s.Ms_frac * vv[2] + s.Mg_frac * V[2] + k * n2};
    const R vp2 = dot3(vp, vp);
    E = s.half_Ms * vp2;
    if (vp2 > (R)0) {
        const R iv = m_rcp(m_sqrt(vp2));
        d[0] = vp[0] * iv;
        d[1] = vp[1] * iv;
        d[2] = vp[2] * iv;
    }
}

// Isotropic direction and exponential step (mean lam_th, the segment's thermal mean free path)
// of a thermalised atom from its three 21-bit codes (length, direction cosine, azimuth).  The
// step -lam_th ln(RN) is formed as -(lam_th ln 2) log2(RN) with lam_l2 = lam_th ln 2, and
// sin^2 = 1 - mu^2 with one fused multiply-add (exact product, one rounding).
template <typename R>
__device__ __forceinline__ R diffusive_draw(R lam_l2, const uint32_t* k, R* d)
{
    const R u0 = u21<R>(k[0]), u2 = u21<R>(k[2]);
    const R mu = sym21<R>(k[1]);       // 2 u1 - 1
    const R st = m_sqrt(fma(-mu, mu, (R)1));
    R sp, cp;
    m_sincos2pi(u2, &sp, &cp);
    d[0] = st * cp;
    d[1] = st * sp;
    d[2] = mu;
    return -lam_l2 * m_log2(u0);
}

// Compensated (Kahan) accumulation: the position is s - c with c the rounding lost so far,
// so thousands of diffusive steps do not accumulate FP32 rounding of the position.
template <typename R> __device__ __forceinline__ void kahan_add(R& s, R& c, R v)
{
    const R y = v - c;
    const R t = s + y;
    c = (t - s) - y;
    s = t;
}

// Per-particle dynamic state.
template <typename R> struct Particle {
    R x[3], xc[3], d[3], E;   // position = x - xc (compensated)
    R r2;              // batched FP32 diffusive mode: squared clearance-ball radius (centre x)
    uint32_t e;        // flights taken
    uint32_t ndiff;    // diffusive steps ended in the gas
    uint32_t ncoll;    // ballistic collisions
    int st;            // ST_BALLISTIC / ST_DIFFUSIVE / ST_DEAD
};

struct Term {
    int state;         // HIT_DEPOSITED / HIT_WALL / HIT_ESCAPED, HIT_NONE while alive
    int bin;
    float cos_in;      // deposits: cosine of the incidence angle (-d . substrate normal); else 0
};

// Terminal outcome of a surface hit along direction d.
template <typename R>
__device__ __forceinline__ Term hit_term(const SegDev<R>& s, int state, R qu, R qv, const R* d)
{
    if (state != HIT_DEPOSITED) return Term{state, -1, 0.f};
    return Term{state, tally_bin(s, qu, qv), (float)(-dot3(d, s.sub_n))};
}

// One flight of a live particle in state MODE (ST_BALLISTIC or ST_DIFFUSIVE): event
// number p.e + 1.  Returns the terminal outcome (HIT_NONE if still in the gas).
template <typename R, int MODE>
__device__ __forceinline__ Term step_mode(const SegDev<R>& s, const TabDev<R>& tb, uint32_t k0, uint32_t k1,
                                          uint32_t pid, uint32_t cap, Particle<R>& p)
{
    if (p.e >= cap) return Term{HIT_ESCAPED, -1, 0.f};
    const uint32_t e = p.e + 1;
    p.e = e;
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    R ell;
    if (MODE == ST_BALLISTIC) {
        r = philox4x32_10(make_uint4(pid, e, s.cfgcat, 0u), k0, k1);
        ell = s.vacuum ? m_inf<R>() : -lambda_m(s, tb, p.E) * m_log(u01<R>(r.x));
    } else {
        uint32_t k[3];
        diffusive_codes(diffusive_block(pid, e, s.cfgcat, k0, k1), (e & 1u) != 0, k);
        ell = diffusive_draw(s.lam_l2, k, p.d);   // diffusive only after a gas collision: never in vacuum
    }
    R t, qu = (R)0, qv = (R)0;
    const HitF h = hit_test(s, p.x, p.d, ell, t, qu, qv, e == 1u);
    // one compensated move: to the surface hit, else the whole flight (a wave whose lanes
    // differ runs the move once)
    const bool hit = h.state != HIT_NONE, finite = ell < m_inf<R>();
    if (hit || finite) {
        const R mv = hit ? t : ell;
#pragma unroll
        for (int i = 0; i < 3; ++i) kahan_add(p.x[i], p.xc[i], mv * p.d[i]);
    }
    if (hit) return hit_term(s, h.state, qu, qv, p.d);
    if (!finite) return Term{HIT_ESCAPED, -1, 0.f};
    if (MODE == ST_BALLISTIC) {
        R V[3] = {(R)0, (R)0, (R)0};
        if (s.gas_motion) gas_velocity(s, philox4x32_10(make_uint4(pid, e, s.cfgcat, 1u), k0, k1), V);
        collide(s, tb, p.E, p.d, V, u01<R>(r.y), u01<R>(r.z));
        ++p.ncoll;
        if (p.E <= s.E_th) {
            p.st = ST_DIFFUSIVE;
            p.r2 = (R)-1;      // no clearance ball yet: the first diffusive step is tested
        }
        if (!(m_finite(p.x[0]) && m_finite(p.x[1]) && m_finite(p.x[2]) && m_finite(p.E)))
            return Term{HIT_ESCAPED, -1, 0.f};
    } else {
        // an isotropic unit direction and a finite step keep the position finite
        ++p.ndiff;
    }
    return Term{HIT_NONE, -1, 0.f};
}

// Position of a thermalised atom in the batched FP32 walk.  The particle keeps its position
// as the unevaluated difference x - xc of two floats (as the compensated sum does).  Between
// two surface tests the walk leaves x alone, so x is the centre of the clearance ball, and
// adds every step to xc alone: xc <- xc - ell d, one fused multiply-add per coordinate.  Then
// -xc is the offset from the centre, the ball test is |xc|^2 < r^2 with no subtraction, and
// the rounding of a step is relative to the offset (at most the ball radius), not to the
// position.  Before a step is tested, the pair is renormalised exactly (x the rounded
// position, xc what that rounding lost), which restores the form the compensated sum and
// the surface test work on.
//
// The same operations serve the step-by-step walk and the wave-cooperative walk, so both
// produce identical positions.
__device__ __forceinline__ void offset_try(const float* xc, float ell, const float* dir, float* t)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) t[i] = __builtin_fmaf(-ell, dir[i], xc[i]);
}
// offset t strictly inside the ball of squared radius r2 (false for NaN and infinities)
__device__ __forceinline__ bool offset_holds(const float* t, float r2)
{
    return __builtin_fmaf(t[2], t[2], __builtin_fmaf(t[1], t[1], t[0] * t[0])) < r2;
}
// (x, xc) -> (rounded x - xc, the rounding error), exactly (Knuth's two-sum)
__device__ __forceinline__ void renormalise(float* x, float* xc)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float a = x[i], b = -xc[i];
        const float s = a + b;
        const float bb = s - a;
        const float err = (a - (s - bb)) + (b - bb);
        x[i] = s;
        xc[i] = -err;
    }
}
// v = ell d, then the compensated add of v (the tested step of diffusive_resolve)
__device__ __forceinline__ void compensated_step(float* x, float* xc, float ell, const float* dir)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float v = ell * dir[i];
        const float y = v - xc[i];
        const float t = x[i] + y;
        xc[i] = (t - x[i]) - y;
        x[i] = t;
    }
}

// Slack between the clearance and the ball radius [mm]: far above the FP32 rounding of the
// position and of the surface test at chamber sizes up to metres.
constexpr float CLEAR_MARGIN = 0.02f;

// A diffusive step of the batched FP32 path (event p.e + 1).  p.r2 is the squared radius of
// a clearance ball around p.x: the clearance of p.x less CLEAR_MARGIN.  A step that ends
// strictly inside the ball (a convex set, entered at its start) stays more than CLEAR_MARGIN
// away from every surface, so the surface test would find nothing and is skipped: the step
// is added to the offset.  Otherwise the step is tested as usual and, if it ends in the gas,
// the ball is rebuilt around its end.  Outcome and arithmetic are those of the tested step.
//
// Such a step is taken in two halves, so that a wave can defer its surface tests.
// diffusive_advance takes the next steps while they stay in the clearance ball: both steps
// of the current Philox block (one if the next event is odd).  A step that leaves the ball
// is held (direction in p.d, length in p.r2: the ball is rebuilt after the test anyway) and
// sets held.  diffusive_resolve tests a held step and finishes it.  The advance needs only
// two numbers of the particle's segment (its thermal mean free path and the Philox counter
// word), passed per lane, so lanes of different segments advance together; the test needs
// the segment's geometry.
//
// One diffusive sub-step from block w (the odd or the even half) for a lane where `active`:
// every lane draws and forms the move; the commit and the hold are written under the lanes'
// masks, so inactive lanes keep their state.
__device__ __forceinline__ void diffusive_substep(float lam_l2, uint4 w, bool odd, bool active, Particle<float>& p,
                                                  bool& held)
{
    uint32_t k[3];
    diffusive_codes(w, odd, k);
    float dir[3];
    const float ell = diffusive_draw(lam_l2, k, dir);   // diffusive only after a gas collision
    float t[3];
    offset_try(p.xc, ell, dir, t);
    const bool ok = offset_holds(t, p.r2);
    const bool commit = active && ok, hold = active && !ok;
    // the writes under the lanes' masks (cheaper than selecting between old and new values)
    if (commit) {
#pragma unroll
        for (int i = 0; i < 3; ++i) p.xc[i] = t[i];
        ++p.ndiff;
        ++p.e;
    }
    if (hold) {
#pragma unroll
        for (int i = 0; i < 3; ++i) p.d[i] = dir[i];
        p.r2 = ell;
        ++p.e;
    }
    held = held || hold;
}

__device__ __forceinline__ Term diffusive_advance(float lam_l2, uint32_t cfgcat, uint32_t k0, uint32_t k1,
                                                  uint32_t pid, uint32_t cap, Particle<float>& p, bool& held)
{
    if (p.e >= cap) return Term{HIT_ESCAPED, -1, 0.f};
    const uint4 w = diffusive_block(pid, p.e + 1, cfgcat, k0, k1);
    // the even step of the block (if the next event is even), then its odd step unless the
    // even one is held or the cap is reached (a capped history escapes at its next step)
    diffusive_substep(lam_l2, w, false, ((p.e + 1) & 1u) == 0, p, held);
    diffusive_substep(lam_l2, w, true, !held && p.e < cap, p, held);
    return Term{HIT_NONE, -1, 0.f};
}

__device__ __forceinline__ Term diffusive_resolve(const SegDev<float>& s, Particle<float>& p)
{
    const float dir[3] = {p.d[0], p.d[1], p.d[2]};
    const float ell = p.r2;
    renormalise(p.x, p.xc);
    float th, qu = 0.f, qv = 0.f;
    const HitF h = hit_test(s, p.x, dir, ell, th, qu, qv, false);
    if (h.state != HIT_NONE) {
#pragma unroll
        for (int i = 0; i < 3; ++i) kahan_add(p.x[i], p.xc[i], th * dir[i]);
        return hit_term(s, h.state, qu, qv, dir);
    }
    if (!(ell < m_inf<float>())) return Term{HIT_ESCAPED, -1, 0.f};
    compensated_step(p.x, p.xc, ell, dir);
    ++p.ndiff;
    const float c = clearance(s, p.x) - CLEAR_MARGIN;
    p.r2 = c > 0.f ? c * c : -1.f;
    return Term{HIT_NONE, -1, 0.f};
}

// One lane along each 16-lane row (DPP row_shr:1): lane j of a row takes src of lane j - 1; the
// first lane of a row has no source there and keeps old.
__device__ __forceinline__ float row_shift1(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), 0x111, 0xF, 0xF, false));
}

// Diffusive steps of up to four thermalised particles of a wave (its lanes in G) taken with the
// whole wave.  Each particle gets a span of 64, 32 or 16 lanes (one, two, or three and four
// particles); lane j of a span draws step e + 1 + j of its particle (Philox block, direction and
// length).  The offsets the steps reach, T_j = fma(-ell_j, d_j, T_{j-1}) from T_{-1} = xc, are
// formed along the spans by shifting the chain one lane per round: within 16-lane rows (DPP), one
// row of every span per phase, the last offset of a row seeding the first lane of the next.  That
// is the order of diffusive_substep, one step after the other, so each T_j is the value the
// step-by-step walk computes, and the committed position, event and step counts are equal.  A
// particle takes its steps up to the first one that leaves the clearance ball or passes the event
// cap (a phase ends the chain early once every particle has such a step); the step that leaves
// the ball is held for the surface test, as diffusive_substep holds it, and a step past the cap
// is not taken (the history, at the cap, escapes).  Every call therefore takes a step, holds one,
// or leaves each particle at the cap.  Called by the whole wave with G uniform, 1 to 4 lanes.
__device__ __forceinline__ void coop_walk(uint32_t k0, uint32_t k1, uint32_t cap, uint64_t G, float lam_l2,
                                          uint32_t cfgcat, uint32_t pid, Particle<float>& p, bool& held, int lane)
{
    const int g = __popcll(G);
    const int sh = g == 1 ? 6 : g == 2 ? 5 : 4;      // log2 of the span
    const int span = 1 << sh;
    const int slot = lane >> sh, j = lane & (span - 1);
    int home[4];                                      // the particles' lanes, in lane order
    {
        uint64_t m = G;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            home[q] = m ? __ffsll((unsigned long long)m) - 1 : 0;
            m &= m - 1;
        }
    }
    const int src = slot == 0 ? home[0] : slot == 1 ? home[1] : slot == 2 ? home[2] : home[3];
    const uint32_t pidw = (uint32_t)__shfl((int)pid, src);
    const uint32_t e0 = (uint32_t)__shfl((int)p.e, src);
    const float r2 = __shfl(p.r2, src);
    const float lam = __shfl(lam_l2, src);
    const uint32_t cc = (uint32_t)__shfl((int)cfgcat, src);
    float xc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) xc[i] = __shfl(p.xc[i], src);
    const uint32_t ej = e0 + 1u + (uint32_t)j;
    uint32_t kc[3];
    diffusive_codes(diffusive_block(pidw, ej, cc, k0, k1), (ej & 1u) != 0, kc);
    float dir[3];
    const float ell = diffusive_draw(lam, kc, dir);
    const bool allowed = ej <= cap && slot < g;        // steps within the event cap
    const float nell = -ell;
    // t: the lane's offset T_j; u: its input T_{j-1} (at the first lane of a row, the row's seed,
    // which the shift leaves in place)
    float t[3], u[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) t[i] = u[i] = xc[i];
    uint64_t ok = 0;
    const int rows = span >> 4;
    for (int r = 0; r < rows; ++r) {
#pragma unroll
        for (int it = 0; it < 16; ++it) {
#pragma unroll
            for (int i = 0; i < 3; ++i) u[i] = row_shift1(u[i], t[i]);
#pragma unroll
            for (int i = 0; i < 3; ++i) t[i] = __builtin_fmaf(nell, dir[i], u[i]);
        }
        // rows 0..r of every span are final: done once each particle has a step it cannot take
        ok = __ballot(allowed && offset_holds(t, r2));
        const uint64_t done_rows = r == 3 ? ~0ull : (1ull << (16 * (r + 1))) - 1;
        bool all = true;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < g) all = all && (~ok & (done_rows << (q << sh))) != 0;
        if (all || r == rows - 1) break;
        float c[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) c[i] = __shfl(t[i], lane - 1);
#pragma unroll
        for (int i = 0; i < 3; ++i) u[i] = j == 16 * (r + 1) ? c[i] : u[i];
    }
    const uint64_t in_cap = __ballot(allowed);
    const uint64_t span_mask = span == 64 ? ~0ull : (1ull << span) - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= g) break;
        const int b = q << sh;
        const uint64_t bad = (~ok >> b) & span_mask;
        const int f = bad ? __ffsll((unsigned long long)bad) - 1 : span;   // steps taken
        const bool hold = f < span && ((in_cap >> (b + f)) & 1ull);
        float nx[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            nx[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f > 0 ? t[i] : xc[i]), f > 0 ? b + f - 1 : b));
        float hd[3] = {0.f, 0.f, 0.f}, hl = 0.f;
        if (hold) {
            hl = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ell), b + f));
#pragma unroll
            for (int i = 0; i < 3; ++i) hd[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dir[i]), b + f));
        }
        if (lane == home[q]) {      // a particle's lane may lie in another particle's span
#pragma unroll
            for (int i = 0; i < 3; ++i) p.xc[i] = nx[i];
            p.e += (uint32_t)f;
            p.ndiff += (uint32_t)f;
            if (hold) {
#pragma unroll
                for (int i = 0; i < 3; ++i) p.d[i] = hd[i];
                p.r2 = hl;
                p.e += 1u;
                held = true;
            }
        }
    }
}

template <typename R>
__device__ __forceinline__ Term step(const SegDev<R>& s, const TabDev<R>& tb, uint32_t k0, uint32_t k1, uint32_t pid,
                                     uint32_t cap, Particle<R>& p)
{
    return p.st == ST_BALLISTIC ? step_mode<R, ST_BALLISTIC>(s, tb, k0, k1, pid, cap, p)
                                : step_mode<R, ST_DIFFUSIVE>(s, tb, k0, k1, pid, cap, p);
}

template <typename R>
__device__ __forceinline__ void start(const SegDev<R>& s, uint32_t k0, uint32_t k1, uint32_t pid, Particle<R>& p)
{
    const uint4 r0 = philox4x32_10(make_uint4(pid, 0u, s.cfgcat, 0u), k0, k1);
    const uint4 r1 = philox4x32_10(make_uint4(pid, 0u, s.cfgcat, 1u), k0, k1);
    launch(s, r0, r1, p.x, p.d, p.E);
    p.xc[0] = p.xc[1] = p.xc[2] = (R)0;
    p.r2 = (R)-1;
    p.e = 0;
    p.ndiff = 0;
    p.ncoll = 0;
    p.st = ST_BALLISTIC;
}

// Arrival tallies of deposits.  Energy bin = #{k in 1..59 : E >= e_k} with e_k = 10^(-3+k/10)
// eV; angle bin = #{k in 1..89 : cos_in <= cos(k deg)}: comparisons with tabulated edges, so
// a bin is decided exactly as a host-side histogram of the records with the same edges would.
template <typename R> __device__ __forceinline__ int energy_bin(const R* e, R E)
{
    int lo = 0, hi = 59;                 // largest j with j == 0 or e[j] <= E
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (e[mid] <= E) lo = mid; else hi = mid - 1;
    }
    return lo;
}
template <typename R> __device__ __forceinline__ int angle_bin(const R* c, R cos_in)
{
    int lo = 0, hi = 89;                 // largest j with j == 0 or cos_in <= c[j]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cos_in <= c[mid]) lo = mid; else hi = mid - 1;
    }
    return lo;
}
// Energy in integer units of 2^-24 eV (exact sums in any order).
__device__ __forceinline__ unsigned long long energy_units(double E) { return (unsigned long long)rint(E * 0x1p24); }

}  // namespace spx
