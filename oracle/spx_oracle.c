/*
 * spx_oracle.c -- plain FP64 CPU oracle of the sputtered-atom Monte Carlo transport.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  The product path (HIP kernels behind
 * the spx_* C-ABI) never calls, links or includes anything here, and this file
 * includes nothing from the product.  It is deliberately slow and literal: every
 * step follows the method in the paper's order, in double precision, with no
 * blocking or reordering, so that it can be checked against the paper by eye.
 *
 * Paper: Thelen, Zehl, Buergel, Depla, Ludwig, "A Python-Based Approach to Sputter
 * Deposition Simulations in Combinatorial Materials Science" (arXiv 2411.14413).
 * The Monte Carlo model is the one of its Methods section, "The SIMTRA model":
 *   - start point sampled from the racetrack profile,
 *   - Thompson energy distribution E/(E+U_s)^3 cut off at E_max = k*Lambda*E_i - U_s,
 *     Lambda = 4 M_i M_t / (M_i + M_t)^2,
 *   - cosine-law emission (c_1 = 1, other c_i = 0),
 *   - free path lambda = -lambda_m ln RN_1 with RN_1 uniform on ]0,1],
 *     lambda_m chosen from the velocities of sputtered and gas atoms,
 *   - trajectory/surface intersection, deposition on a collecting ("dummy") surface,
 *   - otherwise an elastic collision with an Ar atom: scattering angle, new velocity;
 * and, from the calculation paragraph that closes the Methods section, gas motion,
 * diffusion of thermalised atoms and a screened-Coulomb potential with Moliere
 * screening.  Constants and rules the paper does not print are stated where used;
 * each is a documented reading of the paper, not something the paper fixes.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter
 * (particle, event, (config << 8) | cathode, sub-block), key (seed_lo, seed_hi);
 * a 32-bit word x maps to u = ((x >> 8) + 1) * 2^-24, i.e. the paper's ]0,1].
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared (see oracle/build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_PI 3.14159265358979323846

/* Physical constants (CODATA 2018). */
#define KB_EV 8.617333262e-5        /* Boltzmann constant, eV/K */
#define KB_J 1.380649e-23           /* Boltzmann constant, J/K */
#define E2_EV_ANG 14.3996454784     /* e^2/(4 pi eps0), eV * Angstrom */
#define BOHR_ANG 0.529177210903     /* Bohr radius, Angstrom */
#define ANG_TO_MM 1.0e-7

/* Terminal states. */
enum { OR_ALIVE = 0, OR_DEPOSITED = 1, OR_WALL = 2, OR_ESCAPED = 3 };
/* Counters per (config, cathode). */
enum { OC_LAUNCHED = 0, OC_DEPOSITED, OC_WALL, OC_ESCAPED, OC_COLLISIONS, OC_DIFFSTEPS, OC_THERMALIZED, OC_N };

/* ------------------------------------------------------------------------- */
/* Philox4x32-10                                                              */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {                 /* Weyl key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Many blocks at once: out[4i..4i+3] = philox(ctr[4i..4i+3], key). */
void or_philox_batch(const uint32_t* ctr, int64_t n, const uint32_t key[2], uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i) or_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* RN on ]0,1]: 24 random bits, shifted up by one ulp of 2^-24 so 0 is excluded and 1 is reachable. */
double or_u01(uint32_t x) { return (double)((x >> 8) + 1u) * (1.0 / 16777216.0); }

static void draw4(uint64_t seed, uint32_t pid, uint32_t event, uint32_t cfgcat, uint32_t sub, double u[4])
{
    uint32_t ctr[4] = {pid, event, cfgcat, sub};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    or_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = or_u01(x[i]);
}

/* The three RN of diffusive step `event` (direction cosine, azimuth, length).  A diffusive
 * step needs 3 RN, so two steps share one Philox block: steps 2m and 2m+1 use block
 * (pid, 2m, cfgcat, 2).  The even step takes the top 21 bits of words 0, 1, 2; the odd step
 * takes the low 11 bits of word i followed by bits [10 i, 10 i + 10) of word 3, i = 0, 1, 2.
 * RN = (k + 1) 2^-21 on ]0,1] for a 21-bit k. */
void or_diffusive_uniforms(uint64_t seed, uint32_t pid, uint32_t event, uint32_t cfgcat, double u[3])
{
    uint32_t ctr[4] = {pid, event & ~1u, cfgcat, 2u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    or_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 3; ++i) {
        uint32_t k;
        if (event & 1u)
            k = ((x[i] & 0x7FFu) << 10) | ((x[3] >> (10 * i)) & 0x3FFu);
        else
            k = x[i] >> 11;
        u[i] = (double)(k + 1u) * (1.0 / 2097152.0);
    }
}

/* ------------------------------------------------------------------------- */
/* Normal distribution: CDF via erfc, inverse CDF via Wichura's AS241 (PPND16). */
/* ------------------------------------------------------------------------- */
double or_norm_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

double or_norm_inv(double p)
{
    /* Wichura, M. J. (1988) Algorithm AS 241, Appl. Statist. 37, 477-484: PPND16. */
    const double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        const double r = 0.180625 - q * q;
        return q * (((((((2509.0809287301226727 * r + 33430.575583588128105) * r +
                         67265.770927008700853) * r + 45921.953931549871457) * r +
                       13731.693765509461125) * r + 1971.5909503065514427) * r +
                     133.14166789178437745) * r + 3.387132872796366608) /
               (((((((5226.495278852545925 * r + 28729.085735721942674) * r +
                     39307.89580009271061) * r + 21213.794301586595867) * r +
                   5394.1960214247511077) * r + 687.1870074920579083) * r +
                 42.313330701600911252) * r + 1.0);
    }
    double r = (q < 0.0) ? p : 1.0 - p;
    if (r <= 0.0) return (q < 0.0) ? -INFINITY : INFINITY;
    r = sqrt(-log(r));
    double val;
    if (r <= 5.0) {
        r -= 1.6;
        val = (((((((7.7454501427834140764e-4 * r + 0.0227238449892691845833) * r +
                    0.24178072517745061177) * r + 1.27045825245236838258) * r +
                  3.64784832476320460504) * r + 5.7694972214606914055) * r +
                4.6303378461565452959) * r + 1.42343711074968357734) /
              (((((((1.05075007164441684324e-9 * r + 5.475938084995344946e-4) * r +
                    0.0151986665636164571966) * r + 0.14810397642748007459) * r +
                  0.68976733498510000455) * r + 1.6763848301838038494) * r +
                2.05319162663775882187) * r + 1.0);
    } else {
        r -= 5.0;
        val = (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
                    0.0012426609473880784386) * r + 0.026532189526576123093) * r +
                  0.29656057182850489123) * r + 1.7848265399172913358) * r +
                5.4637849111641143699) * r + 6.6579046435011037772) /
              (((((((2.04426310338993978564e-15 * r + 1.4215117583164458887e-7) * r +
                    1.8463183175100546818e-5) * r + 7.868691311456132591e-4) * r +
                  0.0148753612908506148525) * r + 0.13692988092273580531) * r +
                0.59983220655588793769) * r + 1.0);
    }
    return (q < 0.0) ? -val : val;
}

/* ------------------------------------------------------------------------- */
/* Classical scattering angle of a screened-Coulomb potential.                */
/*                                                                           */
/* Reduced units: x = r/a, beta = b/a, eps = a E_r / (Z1 Z2 e^2).  With       */
/* w(x) = V(a x)/E_r the centre-of-mass deflection is                         */
/*   theta = pi - 2 (beta/x0) Int_0^1 du / sqrt(h(u)),                        */
/*   h(u) = 1 - w(x0/u) - beta^2 u^2 / x0^2,                                  */
/* where u = r0/r and x0 = r0/a solves h(1) = 0 (distance of closest approach). */
/* The substitution u = 1 - t^2 removes the inverse-square-root end point, and */
/* the t-integral is done by Gauss-Legendre.                                  */
/*                                                                           */
/* kind 0: Moliere screening Phi(x) = 0.35 e^-0.3x + 0.55 e^-1.2x + 0.10 e^-6x, */
/*         w = Phi(x)/(x eps)  (the potential the paper names);               */
/* kind 1: bare Coulomb, w = 1/(x eps) (Rutherford closed form, for checks);  */
/* kind 2: inverse square, w = eps/x^2 (closed form, for checks).             */
/* ------------------------------------------------------------------------- */
double or_moliere(double x) { return 0.35 * exp(-0.3 * x) + 0.55 * exp(-1.2 * x) + 0.10 * exp(-6.0 * x); }

static double red_potential(int kind, double eps, double x)
{
    switch (kind) {
    case 0: return or_moliere(x) / (x * eps);
    case 1: return 1.0 / (x * eps);
    default: return eps / (x * x);
    }
}

/* Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n (three-term recurrence). */
void or_gauss_legendre01(int n, double* t, double* w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {     /* P_k(z) = ((2k-1) z P_{k-1} - (k-1) P_{k-2}) / k */
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) {
                /* one more evaluation of the derivative at the converged node */
                p0 = 1.0; p1 = 0.0;
                for (int k = 1; k <= n; ++k) {
                    double p2 = p1;
                    p1 = p0;
                    p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
                }
                dp = n * (z * p0 - p1) / (z * z - 1.0);
                break;
            }
        }
        double wz = 2.0 / ((1.0 - z * z) * dp * dp);
        /* map [-1,1] -> [0,1]: nodes come in +-z pairs */
        t[i] = 0.5 * (1.0 - z);
        t[n - 1 - i] = 0.5 * (1.0 + z);
        w[i] = 0.5 * wz;
        w[n - 1 - i] = 0.5 * wz;
    }
}

/* Closest approach x0: root of f(x) = 1 - w(x) - beta^2/x^2, increasing in x. Plain bisection. */
double or_closest_approach(int kind, double eps, double beta)
{
    double lo = (beta > 0.0) ? beta : 1e-300;
    double hi = (beta > 1.0) ? beta : 1.0;
    while (1.0 - red_potential(kind, eps, hi) - beta * beta / (hi * hi) <= 0.0) hi *= 2.0;
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double f = 1.0 - red_potential(kind, eps, mid) - beta * beta / (mid * mid);
        if (f > 0.0) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

static double theta_nodes(int kind, double eps, double beta, int nq, const double* t, const double* w)
{
    if (beta <= 0.0) return OR_PI;              /* head-on: back-scattered */
    const double x0 = or_closest_approach(kind, eps, beta);
    double sum = 0.0;
    for (int k = 0; k < nq; ++k) {
        const double u = 1.0 - t[k] * t[k];
        double h = 1.0 - red_potential(kind, eps, x0 / u) - beta * beta * u * u / (x0 * x0);
        if (h < 1e-300) h = 1e-300;
        sum += w[k] * 2.0 * t[k] / sqrt(h);
    }
    return OR_PI - 2.0 * (beta / x0) * sum;
}

#define OR_NQ 128

double or_theta_cm(int kind, double eps, double beta, int nq)
{
    double* t = (double*)malloc(sizeof(double) * nq);
    double* w = (double*)malloc(sizeof(double) * nq);
    or_gauss_legendre01(nq, t, w);
    double th = theta_nodes(kind, eps, beta, nq, t, w);
    free(t); free(w);
    return th;
}

/* Reduced impact parameter at which the deflection falls to theta_min (cross-section cut-off). */
static double beta_max_nodes(int kind, double eps, double theta_min, int nq, const double* t, const double* w)
{
    double lo = 0.0, hi = 1.0;
    while (theta_nodes(kind, eps, hi, nq, t, w) > theta_min) { lo = hi; hi *= 2.0; }
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (theta_nodes(kind, eps, mid, nq, t, w) > theta_min) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double or_beta_max(int kind, double eps, double theta_min, int nq)
{
    double* t = (double*)malloc(sizeof(double) * nq);
    double* w = (double*)malloc(sizeof(double) * nq);
    or_gauss_legendre01(nq, t, w);
    double b = beta_max_nodes(kind, eps, theta_min, nq, t, w);
    free(t); free(w);
    return b;
}

/*
 * Scattering table: theta[i*ns + j] = theta_cm(eps_i, s_j * beta_max(eps_i)), with
 * log10(eps_i) uniform on [lo, hi] (ne nodes) and s_j = j/(ns-1); betamax[i] = beta_max(eps_i).
 * Sampling b = b_max sqrt(RN) is the same as s = sqrt(RN).
 */
void or_build_table(int kind, double theta_min, int ne, int ns, double lo, double hi,
                    double* theta, double* betamax)
{
    double t[OR_NQ], w[OR_NQ];
    or_gauss_legendre01(OR_NQ, t, w);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < ne; ++i) {
        const double eps = pow(10.0, lo + (hi - lo) * (double)i / (double)(ne - 1));
        const double bm = beta_max_nodes(kind, eps, theta_min, OR_NQ, t, w);
        betamax[i] = bm;
        for (int j = 0; j < ns; ++j) {
            const double s = (double)j / (double)(ns - 1);
            theta[(size_t)i * ns + j] = theta_nodes(kind, eps, s * bm, OR_NQ, t, w);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Per-(config, cathode) segment: raw inputs and derived constants.          */
/* ------------------------------------------------------------------------- */
/* Flat raw layout (doubles), written by oracle/__init__.py:                  */
enum {
    S_CFG = 0, S_CATH, S_CH_R, S_CH_ZLO, S_CH_ZHI, S_P, S_T, S_MG, S_ZG, S_GASMOTION,
    S_SUB_C = 10, S_SUB_N = 13, S_SUB_U = 16, S_HALF_U = 19, S_HALF_V, S_SHAPE, S_NU, S_NV,
    S_CAT_C = 24, S_CAT_N = 27, S_CAT_U = 30, S_CAT_R = 33, S_RT_MU, S_RT_SIG, S_RT_LO, S_RT_HI,
    S_US = 38, S_EI, S_KCUT, S_MS, S_ZS, S_N, S_BINOFF,
    S_RT_N = 45,               /* 0: truncated-normal racetrack; else nodes of a measured profile */
    S_COS = 46,                /* c_0 .. c_5 of the emission law */
    S_RT = 52,                 /* (r_i, depth_i), i < RT_MAX */
    RT_MAX = 256,
    S_OBJ_N = S_RT + 2 * RT_MAX,   /* absorbing objects of the segment */
    S_OBJ = S_OBJ_N + 1,           /* OBJ_LEN doubles each: kind, c[3], n[3], u[3], half_u, half_v, length */
    OBJ_LEN = 16, OBJ_MAX = 32,
    S_LEN = S_OBJ + OBJ_LEN * OBJ_MAX
};
enum { OBJ_DISC = 0, OBJ_RECT = 1, OBJ_TUBE = 2 };
/* Flat parameter layout. */
enum { P_THETA_MIN = 0, P_ETH_KT, P_EVENT_CAP, P_NE, P_NS, P_LOGLO, P_LOGHI, P_LEN = 8 };

/* An absorbing object ("dummy" object: mask, shutter, chimney, another target).  Planar
 * disc (radius hu) or rectangle (half sizes hu, hv) with centre c, normal n, axes u, v; or an
 * open tube: axis through c along n, radius hu, from c to c + len n.  Both faces absorb. */
typedef struct {
    int kind;
    double c[3], n[3], u[3], v[3];
    double hu, hv, len;
} obj_t;

typedef struct {
    uint32_t cfgcat;
    double chR, zlo, zhi;
    double sub_c[3], sub_n[3], sub_u[3], sub_v[3], half_u, half_v, du, dv;
    int shape, nu, nv;
    double cat_c[3], cat_n[3], cat_u[3], cat_v[3], cat_R;
    double rt_mu, rt_sig, PhiA, QB, dPhi;
    int rt_n;                             /* measured racetrack: nodes (0 = truncated normal) */
    double rt_r[RT_MAX], rt_d[RT_MAX];    /* radius, erosion depth */
    double rt_F[RT_MAX];                  /* integral_0^{r_i} depth(s) s ds */
    double cosc[6], cos_norm;             /* emission law sum c_i mu^i; norm = sum c_i / (i + 1) */
    int cos_pure;                         /* the cosine law c = (0, 1, 0, 0, 0, 0) */
    double Us, Emax, smax, Lambda;
    double Ms, Mg, mu_red, eps_per_eV, a_mm;
    double n_mm3, kT, vth, vg;           /* vth = sqrt(kT/Mg) per Cartesian component; vg = sqrt(2kT/Mg) */
    double E_th, lam_th;
    int gas_motion;
    int n_obj;
    obj_t obj[OBJ_MAX];
    uint64_t N, bin_off;
} seg_t;

typedef struct {
    const double* theta;
    const double* betamax;
    int ne, ns;
    double lo, hi;
    uint32_t event_cap;
} tab_t;

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* beta_max(eps): linear in log10(eps) between table nodes, eps clamped to the table range. */
static double tab_betamax(const tab_t* tb, double eps)
{
    double x = (log10(eps) - tb->lo) / (tb->hi - tb->lo) * (tb->ne - 1);
    if (!(x > 0.0)) x = 0.0;
    if (x > tb->ne - 1) x = tb->ne - 1;
    int i = (int)floor(x);
    if (i > tb->ne - 2) i = tb->ne - 2;
    double f = x - i;
    return tb->betamax[i] * (1.0 - f) + tb->betamax[i + 1] * f;
}

/* theta_cm(eps, s): bilinear in (log10 eps, s) on the table grid. */
static double tab_theta(const tab_t* tb, double eps, double s)
{
    double x = (log10(eps) - tb->lo) / (tb->hi - tb->lo) * (tb->ne - 1);
    if (!(x > 0.0)) x = 0.0;
    if (x > tb->ne - 1) x = tb->ne - 1;
    int i = (int)floor(x);
    if (i > tb->ne - 2) i = tb->ne - 2;
    double fx = x - i;
    double y = s * (tb->ns - 1);
    if (!(y > 0.0)) y = 0.0;
    if (y > tb->ns - 1) y = tb->ns - 1;
    int j = (int)floor(y);
    if (j > tb->ns - 2) j = tb->ns - 2;
    double fy = y - j;
    const double* T = tb->theta;
    const size_t ns = (size_t)tb->ns;
    return (1.0 - fx) * (1.0 - fy) * T[i * ns + j] + fx * (1.0 - fy) * T[(i + 1) * ns + j] +
           (1.0 - fx) * fy * T[i * ns + j + 1] + fx * fy * T[(i + 1) * ns + j + 1];
}

/* sigma(eps) = pi (a beta_max)^2 in mm^2. */
static double seg_sigma(const seg_t* s, const tab_t* tb, double eps)
{
    double b = s->a_mm * tab_betamax(tb, eps);
    return OR_PI * b * b;
}

/* integral over s in [r_i, r_i + t] of depth(s) s, depth linear on the node interval i */
static double rt_piece(const seg_t* s, int i, double t)
{
    const double dr = s->rt_r[i + 1] - s->rt_r[i];
    const double m = (s->rt_d[i + 1] - s->rt_d[i]) / dr;
    const double d0 = s->rt_d[i], r0 = s->rt_r[i];
    return d0 * r0 * t + (d0 + m * r0) * t * t / 2.0 + m * t * t * t / 3.0;
}

static void seg_init(const double* r, const double* prm, const tab_t* tb, seg_t* s)
{
    memset(s, 0, sizeof(*s));
    s->cfgcat = ((uint32_t)r[S_CFG] << 8) | (uint32_t)r[S_CATH];
    s->chR = r[S_CH_R]; s->zlo = r[S_CH_ZLO]; s->zhi = r[S_CH_ZHI];
    for (int i = 0; i < 3; ++i) {
        s->sub_c[i] = r[S_SUB_C + i]; s->sub_n[i] = r[S_SUB_N + i]; s->sub_u[i] = r[S_SUB_U + i];
        s->cat_c[i] = r[S_CAT_C + i]; s->cat_n[i] = r[S_CAT_N + i]; s->cat_u[i] = r[S_CAT_U + i];
    }
    cross(s->sub_n, s->sub_u, s->sub_v);
    cross(s->cat_n, s->cat_u, s->cat_v);
    s->half_u = r[S_HALF_U]; s->half_v = r[S_HALF_V];
    s->shape = (int)r[S_SHAPE]; s->nu = (int)r[S_NU]; s->nv = (int)r[S_NV];
    s->du = 2.0 * s->half_u / s->nu; s->dv = 2.0 * s->half_v / s->nv;
    s->cat_R = r[S_CAT_R];

    /* Racetrack start radius: normal(mu, sigma) truncated to [lo, hi]. */
    s->rt_mu = r[S_RT_MU]; s->rt_sig = r[S_RT_SIG];
    const double al = (r[S_RT_LO] - s->rt_mu) / s->rt_sig, be = (r[S_RT_HI] - s->rt_mu) / s->rt_sig;
    s->PhiA = or_norm_cdf(al);
    s->QB = or_norm_cdf(-be);                       /* 1 - Phi(beta), without cancellation */
    s->dPhi = or_norm_cdf(be) - s->PhiA;

    /* Measured racetrack: erosion depth linear between the nodes; the start radius has a
     * density proportional to depth(r) r (area element of an axisymmetric target). */
    s->rt_n = (int)r[S_RT_N];
    for (int i = 0; i < s->rt_n; ++i) {
        s->rt_r[i] = r[S_RT + 2 * i];
        s->rt_d[i] = r[S_RT + 2 * i + 1];
    }
    if (s->rt_n > 0) s->rt_F[0] = 0.0;
    for (int i = 0; i + 1 < s->rt_n; ++i)
        s->rt_F[i + 1] = s->rt_F[i] + rt_piece(s, i, s->rt_r[i + 1] - s->rt_r[i]);

    /* Emission law: density of mu = cos(theta) on [0, 1] proportional to sum c_i mu^i. */
    s->cos_norm = 0.0;
    s->cos_pure = 1;
    for (int i = 0; i < 6; ++i) {
        s->cosc[i] = r[S_COS + i];
        s->cos_norm += s->cosc[i] / (i + 1);
        if (s->cosc[i] != (i == 1 ? 1.0 : 0.0)) s->cos_pure = 0;
    }

    /* Thompson energy with cut-off: the ion is the working-gas ion (Ar+), M_i = gas mass. */
    s->Ms = r[S_MS]; s->Mg = r[S_MG];
    s->Us = r[S_US];
    s->Lambda = 4.0 * s->Mg * s->Ms / ((s->Mg + s->Ms) * (s->Mg + s->Ms));
    s->Emax = r[S_KCUT] * s->Lambda * r[S_EI] - s->Us;
    s->smax = s->Emax / (s->Emax + s->Us);

    /* Interaction: Firsov screening length, reduced energy per eV of CM energy. */
    const double Zs = r[S_ZS], Zg = r[S_ZG];
    const double a_ang = 0.8853 * BOHR_ANG * pow(sqrt(Zs) + sqrt(Zg), -2.0 / 3.0);
    s->a_mm = a_ang * ANG_TO_MM;
    s->eps_per_eV = a_ang / (Zs * Zg * E2_EV_ANG);
    s->mu_red = s->Ms * s->Mg / (s->Ms + s->Mg);

    /* Gas: ideal-gas number density, thermal speeds in sqrt(eV/u). */
    const double T = r[S_T];
    s->n_mm3 = r[S_P] / (KB_J * T) * 1e-9;
    s->kT = KB_EV * T;
    s->vth = sqrt(s->kT / s->Mg);
    s->vg = sqrt(2.0 * s->kT / s->Mg);
    s->gas_motion = (int)r[S_GASMOTION];

    /* Thermalisation: threshold E_th = c kT; diffusive mean free path from the
     * cross-section at the thermal CM energy 1.5 kT and the mean relative speed. */
    s->E_th = prm[P_ETH_KT] * s->kT;
    if (s->n_mm3 > 0.0) {
        const double sig_th = seg_sigma(s, tb, s->eps_per_eV * 1.5 * s->kT);
        s->lam_th = 1.0 / (s->n_mm3 * sig_th * sqrt(1.0 + s->Ms / s->Mg));
    } else {
        s->lam_th = INFINITY;
    }
    s->n_obj = (int)r[S_OBJ_N];
    for (int k = 0; k < s->n_obj; ++k) {
        const double* o = r + S_OBJ + OBJ_LEN * k;
        obj_t* b = &s->obj[k];
        b->kind = (int)o[0];
        for (int i = 0; i < 3; ++i) { b->c[i] = o[1 + i]; b->n[i] = o[4 + i]; b->u[i] = o[7 + i]; }
        cross(b->n, b->u, b->v);
        b->hu = o[10]; b->hv = o[11]; b->len = o[12];
    }
    s->N = (uint64_t)r[S_N];
    s->bin_off = (uint64_t)r[S_BINOFF];
}

/* Mean free path of a sputtered atom of energy E (mm). */
static double lambda_m(const seg_t* s, const tab_t* tb, double E)
{
    if (!(s->n_mm3 > 0.0)) return INFINITY;
    /* cross-section at the CM energy of a collision with a gas atom at rest */
    const double eps = s->eps_per_eV * E * s->Mg / (s->Ms + s->Mg);
    const double sig = seg_sigma(s, tb, eps);
    if (!s->gas_motion) return 1.0 / (s->n_mm3 * sig);
    /* moving gas: collision rate n sigma <|v - V|>, <g> the Maxwellian mean relative speed */
    const double v = sqrt(2.0 * E / s->Ms);
    const double x = v / s->vg;
    const double g = s->vg * ((x + 0.5 / x) * erf(x) + exp(-x * x) / sqrt(OR_PI));
    return v / (s->n_mm3 * sig * g);
}

/* Free path lambda = -lambda_m ln RN_1 (infinite in vacuum). */
static double flight_length(const seg_t* s, const tab_t* tb, double E, double rn1)
{
    return (s->n_mm3 > 0.0) ? -lambda_m(s, tb, E) * log(rn1) : INFINITY;
}

/* ------------------------------------------------------------------------- */
/* Launch: racetrack start point, Thompson energy, cosine direction.         */
/* ------------------------------------------------------------------------- */
/* Start radius of a measured racetrack: r = F^{-1}(RN F(R)) with F(r) the integral of
 * depth(s) s from 0 to r.  The node interval holding the target is the first whose end
 * value reaches it (RN > 0, so it carries positive weight); inside it F is a cubic, inverted
 * by bisection to the resolution of the doubles. */
static double racetrack_radius(const seg_t* s, double rn)
{
    const double target = rn * s->rt_F[s->rt_n - 1];
    int i = 0;
    while (i < s->rt_n - 2 && s->rt_F[i + 1] < target) ++i;
    const double want = target - s->rt_F[i];
    double lo = 0.0, hi = s->rt_r[i + 1] - s->rt_r[i];
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (rt_piece(s, i, mid) < want) lo = mid; else hi = mid;
    }
    return s->rt_r[i] + 0.5 * (lo + hi);
}

/* cos(theta) of the emission law: G(mu) = sum c_i mu^(i+1)/(i+1) = RN G(1), by bisection on [0, 1]. */
static double emission_mu(const seg_t* s, double rn)
{
    const double want = rn * s->cos_norm;
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double g = 0.0, p = mid;
        for (int i = 0; i < 6; ++i) {
            g += s->cosc[i] * p / (i + 1);
            p *= mid;
        }
        if (g < want) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static void launch(const seg_t* s, uint64_t seed, uint32_t pid, double x[3], double d[3], double* E)
{
    double u[4], u4[4];
    draw4(seed, pid, 0, s->cfgcat, 0, u);
    draw4(seed, pid, 0, s->cfgcat, 1, u4);
    double rr;
    if (s->rt_n > 0) {
        rr = racetrack_radius(s, u[0]);
    } else {
        /* start radius by inverse CDF of the truncated normal; the upper half uses the complement */
        double z;
        const double P = s->PhiA + u[0] * s->dPhi;
        if (P <= 0.5) {
            z = or_norm_inv(P);
        } else {
            const double Q = s->QB + (1.0 - u[0]) * s->dPhi;
            z = -or_norm_inv(Q);
        }
        rr = s->rt_mu + s->rt_sig * z;
    }
    const double psi = 2.0 * OR_PI * u[1];
    for (int i = 0; i < 3; ++i) x[i] = s->cat_c[i] + rr * (cos(psi) * s->cat_u[i] + sin(psi) * s->cat_v[i]);
    /* Thompson: F(E) = [E/(E+U_s)]^2 / [E_max/(E_max+U_s)]^2 inverted */
    const double sE = sqrt(u[2]) * s->smax;
    *E = s->Us * sE / (1.0 - sE);
    /* polar angle from the emission law (cosine law: cos(theta) = sqrt(RN)), azimuth uniform */
    double mu, st;
    if (s->cos_pure) {
        mu = sqrt(u[3]);
        st = sqrt(1.0 - u[3]);
    } else {
        mu = emission_mu(s, u[3]);
        st = sqrt((1.0 - mu) * (1.0 + mu));
    }
    const double phi = 2.0 * OR_PI * u4[0];
    for (int i = 0; i < 3; ++i)
        d[i] = mu * s->cat_n[i] + st * (cos(phi) * s->cat_u[i] + sin(phi) * s->cat_v[i]);
}

/* ------------------------------------------------------------------------- */
/* Surface intersection.  Returns nearest hit with 0 < t <= ell; ties keep the */
/* first in the order substrate, cathode, objects, chamber.                   */
/* ------------------------------------------------------------------------- */
typedef struct { double t; int state; int bin; } hit_t;

static hit_t hit_test(const seg_t* s, const double x[3], const double d[3], double ell, int first_flight)
{
    hit_t best = {INFINITY, OR_ALIVE, -1};
    /* substrate plate */
    {
        const double dn = dot(d, s->sub_n);
        if (dn != 0.0) {
            double w[3] = {s->sub_c[0] - x[0], s->sub_c[1] - x[1], s->sub_c[2] - x[2]};
            const double t = dot(w, s->sub_n) / dn;
            if (t > 0.0) {
                double q[3];
                for (int i = 0; i < 3; ++i) q[i] = x[i] + t * d[i] - s->sub_c[i];
                const double qu = dot(q, s->sub_u), qv = dot(q, s->sub_v);
                int inside = (s->shape == 0) ? (fabs(qu) <= s->half_u && fabs(qv) <= s->half_v)
                                             : (qu * qu + qv * qv <= s->half_u * s->half_u);
                if (inside && t < best.t) {
                    best.t = t;
                    if (dn < 0.0) {           /* front face: the normal faces the cathodes */
                        int iu = (int)floor((qu + s->half_u) / s->du);
                        int iv = (int)floor((qv + s->half_v) / s->dv);
                        if (iu < 0) iu = 0;
                        if (iu > s->nu - 1) iu = s->nu - 1;
                        if (iv < 0) iv = 0;
                        if (iv > s->nv - 1) iv = s->nv - 1;
                        best.state = OR_DEPOSITED;
                        best.bin = iv * s->nu + iu;
                    } else {
                        best.state = OR_WALL;
                        best.bin = -1;
                    }
                }
            }
        }
    }
    /* emitting cathode disc, absorbing on both faces.  The first flight starts on the
     * target plane (the atom leaves the surface into the gas), and a straight line meets
     * a plane once, so the target cannot be hit at t > 0 on that flight: it is not tested,
     * rather than left to the rounding of a distance that is zero. */
    if (!first_flight) {
        const double dn = dot(d, s->cat_n);
        if (dn != 0.0) {
            double w[3] = {s->cat_c[0] - x[0], s->cat_c[1] - x[1], s->cat_c[2] - x[2]};
            const double t = dot(w, s->cat_n) / dn;
            if (t > 0.0) {
                double q[3];
                for (int i = 0; i < 3; ++i) q[i] = x[i] + t * d[i] - s->cat_c[i];
                const double qu = dot(q, s->cat_u), qv = dot(q, s->cat_v);
                if (qu * qu + qv * qv <= s->cat_R * s->cat_R && t < best.t) {
                    best.t = t; best.state = OR_WALL; best.bin = -1;
                }
            }
        }
    }
    /* absorbing objects: discs and rectangles (a plane crossing inside the region), open
     * tubes (the smaller positive root of the distance to the axis with its axial
     * coordinate inside the tube) */
    for (int k = 0; k < s->n_obj; ++k) {
        const obj_t* b = &s->obj[k];
        double t = INFINITY;
        if (b->kind == OBJ_DISC || b->kind == OBJ_RECT) {
            const double dn = dot(d, b->n);
            if (dn != 0.0) {
                double w[3] = {b->c[0] - x[0], b->c[1] - x[1], b->c[2] - x[2]};
                const double tp = dot(w, b->n) / dn;
                if (tp > 0.0) {
                    double q[3];
                    for (int i = 0; i < 3; ++i) q[i] = x[i] + tp * d[i] - b->c[i];
                    const double qu = dot(q, b->u), qv = dot(q, b->v);
                    const int in = (b->kind == OBJ_DISC) ? (qu * qu + qv * qv <= b->hu * b->hu)
                                                         : (fabs(qu) <= b->hu && fabs(qv) <= b->hv);
                    if (in) t = tp;
                }
            }
        } else {
            double w[3] = {x[0] - b->c[0], x[1] - b->c[1], x[2] - b->c[2]};
            const double wa = dot(w, b->n), da = dot(d, b->n);
            double wp[3], dp[3];
            for (int i = 0; i < 3; ++i) { wp[i] = w[i] - wa * b->n[i]; dp[i] = d[i] - da * b->n[i]; }
            const double A = dot(dp, dp), B = dot(wp, dp), C = dot(wp, wp) - b->hu * b->hu;
            const double D = B * B - A * C;
            if (A > 0.0 && D >= 0.0) {
                const double sq = sqrt(D);
                const double roots[2] = {(-B - sq) / A, (-B + sq) / A};
                for (int j = 0; j < 2; ++j) {
                    const double tr = roots[j];
                    const double za = wa + tr * da;
                    if (tr > 0.0 && za >= 0.0 && za <= b->len) { t = tr; break; }
                }
            }
        }
        if (t < best.t) { best.t = t; best.state = OR_WALL; best.bin = -1; }
    }
    /* chamber: cylinder side and the two caps (closed: some t >= 0 always exists) */
    {
        double tc = INFINITY;
        const double a = d[0] * d[0] + d[1] * d[1];
        if (a > 0.0) {
            const double b = x[0] * d[0] + x[1] * d[1];
            const double c = x[0] * x[0] + x[1] * x[1] - s->chR * s->chR;
            double disc = b * b - a * c;
            if (disc < 0.0) disc = 0.0;
            const double sq = sqrt(disc);
            double t = (b <= 0.0) ? (-b + sq) / a : -c / (b + sq);
            if (t < 0.0) t = 0.0;
            tc = t;
        }
        if (d[2] > 0.0) {
            double t = (s->zhi - x[2]) / d[2];
            if (t < 0.0) t = 0.0;
            if (t < tc) tc = t;
        } else if (d[2] < 0.0) {
            double t = (s->zlo - x[2]) / d[2];
            if (t < 0.0) t = 0.0;
            if (t < tc) tc = t;
        }
        if (tc < best.t) { best.t = tc; best.state = OR_WALL; best.bin = -1; }
    }
    if (!(best.t <= ell)) { best.state = OR_ALIVE; best.bin = -1; }
    return best;
}

/* ------------------------------------------------------------------------- */
/* Elastic binary collision with a gas atom of velocity V.                   */
/* ------------------------------------------------------------------------- */
static void collide(const seg_t* s, const tab_t* tb, double* E, double d[3], const double V[3],
                    double u_b, double u_phi)
{
    const double v = sqrt(2.0 * (*E) / s->Ms);
    double vv[3], g[3];
    for (int i = 0; i < 3; ++i) { vv[i] = v * d[i]; g[i] = vv[i] - V[i]; }
    const double gm = sqrt(dot(g, g));
    if (!(gm > 0.0)) return;                         /* no relative motion: nothing happens */
    const double Er = 0.5 * s->mu_red * gm * gm;
    const double th = tab_theta(tb, s->eps_per_eV * Er, sqrt(u_b));
    const double ph = 2.0 * OR_PI * u_phi;
    const double gu = g[0] / gm, gv = g[1] / gm, gw = g[2] / gm;
    const double ct = cos(th), st = sin(th), cp = cos(ph), sp = sin(ph);
    double n0, n1, n2;
    if (fabs(gw) < 0.99999) {
        const double rho = sqrt(1.0 - gw * gw);
        n0 = gu * ct + st * (gu * gw * cp - gv * sp) / rho;
        n1 = gv * ct + st * (gv * gw * cp + gu * sp) / rho;
        n2 = gw * ct - rho * st * cp;
    } else {
        n0 = st * cp;
        n1 = st * sp;
        n2 = (gw > 0.0 ? 1.0 : -1.0) * ct;
    }
    const double M = s->Ms + s->Mg;
    double vp[3];
    const double gn[3] = {n0, n1, n2};
    for (int i = 0; i < 3; ++i) vp[i] = (s->Ms * vv[i] + s->Mg * V[i]) / M + s->Mg / M * gm * gn[i];
    const double vp2 = dot(vp, vp);
    *E = 0.5 * s->Ms * vp2;
    if (vp2 > 0.0) {
        const double inv = 1.0 / sqrt(vp2);
        for (int i = 0; i < 3; ++i) d[i] = vp[i] * inv;
    }
}

/* Maxwellian velocity of the gas partner from one Philox block (Box-Muller). */
static void gas_velocity(const seg_t* s, const double w[4], double V[3])
{
    const double r0 = sqrt(-2.0 * log(w[0])), r1 = sqrt(-2.0 * log(w[2]));
    V[0] = s->vth * r0 * cos(2.0 * OR_PI * w[1]);
    V[1] = s->vth * r0 * sin(2.0 * OR_PI * w[1]);
    V[2] = s->vth * r1 * cos(2.0 * OR_PI * w[3]);
}

/* Isotropic direction and exponential step of a thermalised atom from its three RN. */
static void diffusive_draw(const seg_t* s, const double u[3], double d[3], double* ell)
{
    const double mu = 2.0 * u[1] - 1.0;
    const double st = sqrt(1.0 - mu * mu);
    const double ph = 2.0 * OR_PI * u[2];
    d[0] = st * cos(ph); d[1] = st * sin(ph); d[2] = mu;
    *ell = (s->lam_th < INFINITY) ? -s->lam_th * log(u[0]) : INFINITY;
}

/* ------------------------------------------------------------------------- */
/* One particle history.                                                     */
/* ------------------------------------------------------------------------- */
typedef struct {
    double x[3], E;
    double cos_in;          /* deposits: cosine of the incidence angle (-d . substrate normal); else 0 */
    int state, bin;
    uint32_t events, ndiff, ncoll;
    int thermalized;
} result_t;

static int finite3(const double x[3]) { return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]); }

static void trace(const seg_t* s, const tab_t* tb, uint64_t seed, uint32_t pid, result_t* res)
{
    double x[3], d[3], E;
    launch(s, seed, pid, x, d, &E);
    int diffusive = 0;
    uint32_t ndiff = 0, ncoll = 0;
    uint32_t e = 1;
    res->state = OR_ESCAPED;
    res->bin = -1;
    res->cos_in = 0.0;
    for (;; ++e) {
        if (e > tb->event_cap) { res->state = OR_ESCAPED; e = tb->event_cap; break; }
        double u[4];
        double ell;
        if (!diffusive) {
            draw4(seed, pid, e, s->cfgcat, 0, u);
            ell = flight_length(s, tb, E, u[0]);
        } else {
            or_diffusive_uniforms(seed, pid, e, s->cfgcat, u);
            diffusive_draw(s, u, d, &ell);
        }
        hit_t h = hit_test(s, x, d, ell, e == 1);
        if (h.state != OR_ALIVE) {
            for (int i = 0; i < 3; ++i) x[i] += h.t * d[i];
            res->state = h.state;
            res->bin = h.bin;
            if (h.state == OR_DEPOSITED) res->cos_in = -dot(d, s->sub_n);
            break;
        }
        if (!(ell < INFINITY)) { res->state = OR_ESCAPED; break; }   /* open line of sight: cannot happen in a closed chamber */
        for (int i = 0; i < 3; ++i) x[i] += ell * d[i];
        if (!diffusive) {
            double V[3] = {0.0, 0.0, 0.0};
            if (s->gas_motion) {
                double w[4];
                draw4(seed, pid, e, s->cfgcat, 1, w);
                gas_velocity(s, w, V);
            }
            collide(s, tb, &E, d, V, u[1], u[2]);
            ++ncoll;
            if (E <= s->E_th) diffusive = 1;
        } else {
            ++ndiff;
        }
        if (!finite3(x) || !isfinite(E)) { res->state = OR_ESCAPED; break; }
    }
    for (int i = 0; i < 3; ++i) res->x[i] = x[i];
    res->E = E;
    res->events = e;
    res->ndiff = ndiff;
    res->ncoll = ncoll;
    res->thermalized = diffusive;
}

static void make_tab(const double* prm, const double* theta, const double* betamax, tab_t* tb)
{
    tb->theta = theta;
    tb->betamax = betamax;
    tb->ne = (int)prm[P_NE];
    tb->ns = (int)prm[P_NS];
    tb->lo = prm[P_LOGLO];
    tb->hi = prm[P_LOGHI];
    tb->event_cap = (uint32_t)prm[P_EVENT_CAP];
}

/* ------------------------------------------------------------------------- */
/* Public driver entry points.                                               */
/* ------------------------------------------------------------------------- */
#define OR_REC 9   /* record: x, y, z, state, bin, events, diffusive steps, final E, incidence cosine */

static void write_record(double* rec, const result_t* r)
{
    rec[0] = r->x[0]; rec[1] = r->x[1]; rec[2] = r->x[2];
    rec[3] = r->state; rec[4] = r->bin; rec[5] = r->events; rec[6] = r->ndiff; rec[7] = r->E;
    rec[8] = r->cos_in;
}

/*
 * Run particles [pid_begin, min(pid_end, N)) of every segment.  counts (u64) is
 * indexed by seg.bin_off + bin; counters is [n_seg][7]; records (nullable) holds
 * OR_REC doubles per particle in segment-major order over the simulated range.
 * Returns the number of OpenMP threads used.
 */
int or_run(const double* segs, int n_seg, const double* prm, const double* theta, const double* betamax,
           uint64_t seed, uint64_t pid_begin, uint64_t pid_end, int n_threads,
           uint64_t* counts, uint64_t* counters, double* records)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t* S = (seg_t*)malloc(sizeof(seg_t) * (size_t)n_seg);
    uint64_t* first = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n_seg + 1));
    first[0] = 0;
    for (int k = 0; k < n_seg; ++k) {
        seg_init(segs + (size_t)k * S_LEN, prm, &tb, &S[k]);
        uint64_t hi = S[k].N < pid_end ? S[k].N : pid_end;
        uint64_t n = hi > pid_begin ? hi - pid_begin : 0;
        first[k + 1] = first[k] + n;
    }
    const int64_t total = (int64_t)first[n_seg];
    if (n_threads <= 0) n_threads = omp_get_max_threads();
    int used = 1;
#pragma omp parallel num_threads(n_threads)
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 64)
        for (int64_t g = 0; g < total; ++g) {
            int k = 0;
            while (first[k + 1] <= (uint64_t)g) ++k;
            const uint32_t pid = (uint32_t)(pid_begin + ((uint64_t)g - first[k]));
            result_t r;
            trace(&S[k], &tb, seed, pid, &r);
            uint64_t* C = counters + (size_t)k * OC_N;
            __atomic_fetch_add(&C[OC_LAUNCHED], 1, __ATOMIC_RELAXED);
            __atomic_fetch_add(&C[r.state == OR_DEPOSITED ? OC_DEPOSITED : r.state == OR_WALL ? OC_WALL : OC_ESCAPED],
                               1, __ATOMIC_RELAXED);
            __atomic_fetch_add(&C[OC_COLLISIONS], r.ncoll, __ATOMIC_RELAXED);
            __atomic_fetch_add(&C[OC_DIFFSTEPS], r.ndiff, __ATOMIC_RELAXED);
            __atomic_fetch_add(&C[OC_THERMALIZED], (uint64_t)r.thermalized, __ATOMIC_RELAXED);
            if (r.state == OR_DEPOSITED) __atomic_fetch_add(&counts[S[k].bin_off + (uint64_t)r.bin], 1, __ATOMIC_RELAXED);
            if (records) write_record(records + (size_t)g * OR_REC, &r);
        }
    }
    free(S);
    free(first);
    return used;
}

/* Trace an explicit list of (segment, particle) pairs; records only. */
void or_run_list(const double* segs, int n_seg, const double* prm, const double* theta, const double* betamax,
                 uint64_t seed, const uint32_t* seg_ids, const uint32_t* pids, int64_t n, int n_threads,
                 double* records)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t* S = (seg_t*)malloc(sizeof(seg_t) * (size_t)n_seg);
    for (int k = 0; k < n_seg; ++k) seg_init(segs + (size_t)k * S_LEN, prm, &tb, &S[k]);
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for num_threads(n_threads) schedule(dynamic, 16)
    for (int64_t g = 0; g < n; ++g) {
        result_t r;
        trace(&S[seg_ids[g]], &tb, seed, pids[g], &r);
        write_record(records + (size_t)g * OR_REC, &r);
    }
    free(S);
}

/* ------------------------------------------------------------------------- */
/* Hooks exposing single steps, for the pins in the test-suite.              */
/* ------------------------------------------------------------------------- */
/* Derived segment constants: Lambda, E_max, s_max, a_mm, eps_per_eV, n_mm3, kT,
 * E_th, lam_th, PhiA, QB, dPhi, mu_red, vth, vg. */
void or_seg_info(const double* seg, const double* prm, const double* theta, const double* betamax, double* out)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    const double v[15] = {s.Lambda, s.Emax, s.smax, s.a_mm, s.eps_per_eV, s.n_mm3, s.kT, s.E_th,
                          s.lam_th, s.PhiA, s.QB, s.dPhi, s.mu_red, s.vth, s.vg};
    memcpy(out, v, sizeof(v));
}

/* Launch sample of particle pid: out = x[3], d[3], E. */
void or_launch(const double* seg, const double* prm, const double* theta, const double* betamax,
               uint64_t seed, uint32_t pid, double* out)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    launch(&s, seed, pid, out, out + 3, out + 6);
}

/* Launch samples of particles pid0 .. pid0+n-1: out[7*i ..] = x[3], d[3], E. */
void or_launch_batch(const double* seg, const double* prm, const double* theta, const double* betamax,
                     uint64_t seed, uint32_t pid0, int64_t n, double* out)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    for (int64_t i = 0; i < n; ++i) {
        double* o = out + 7 * i;
        launch(&s, seed, pid0 + (uint32_t)i, o, o + 3, o + 6);
    }
}

/* First-flight lengths at energy E for particles pid0 .. pid0+n-1 (the RN_1 of event 1). */
void or_flights(const double* seg, const double* prm, const double* theta, const double* betamax,
                uint64_t seed, uint32_t pid0, int64_t n, double E, double* out)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    for (int64_t i = 0; i < n; ++i) {
        double u[4];
        draw4(seed, pid0 + (uint32_t)i, 1, s.cfgcat, 0, u);
        out[i] = flight_length(&s, &tb, E, u[0]);
    }
}

double or_lambda_m(const double* seg, const double* prm, const double* theta, const double* betamax, double E)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    return lambda_m(&s, &tb, E);
}

double or_table_theta(const double* prm, const double* theta, const double* betamax, double eps, double s)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    return tab_theta(&tb, eps, s);
}

/* Collision with a given gas velocity V: io = {E, d[3]} updated in place. */
void or_collide(const double* seg, const double* prm, const double* theta, const double* betamax,
                const double* V, double u_b, double u_phi, double* io)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    collide(&s, &tb, &io[0], &io[1], V, u_b, u_phi);
}

void or_gas_velocity(const double* seg, const double* prm, const double* theta, const double* betamax,
                     const double* w, double* V)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    gas_velocity(&s, w, V);
}

/* Hit test: out = {t, state, bin}. */
void or_hit(const double* seg, const double* prm, const double* theta, const double* betamax,
            const double* x, const double* d, double ell, int first_flight, double* out)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    hit_t h = hit_test(&s, x, d, ell, first_flight);
    out[0] = h.t; out[1] = h.state; out[2] = h.bin;
}

/* Unbounded diffusive walk of n_steps from the origin with the step sampler of the
 * transport (same Philox keying as the diffusive events 1..n_steps of particle pid). */
void or_walk(const double* seg, const double* prm, const double* theta, const double* betamax,
             uint64_t seed, uint32_t pid, uint32_t n_steps, double* out)
{
    tab_t tb;
    make_tab(prm, theta, betamax, &tb);
    seg_t s;
    seg_init(seg, prm, &tb, &s);
    double x[3] = {0.0, 0.0, 0.0};
    for (uint32_t e = 1; e <= n_steps; ++e) {
        double u[3], d[3], ell;
        or_diffusive_uniforms(seed, pid, e, s.cfgcat, u);
        diffusive_draw(&s, u, d, &ell);
        for (int i = 0; i < 3; ++i) x[i] += ell * d[i];
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2];
}

int or_max_threads(void) { return omp_get_max_threads(); }
