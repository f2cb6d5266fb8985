// api.hip -- host runtime of libspx: validation, per-segment constants, plan
// memory, the FP32 graph replay, the autotuner and the C-ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "spx_host.hpp"

namespace spx {

namespace {
thread_local std::string g_error;

constexpr double KB_EV = 8.617333262e-5;     // eV/K
constexpr double KB_J = 1.380649e-23;        // J/K
constexpr double E2 = 14.3996454784;         // e^2/(4 pi eps0), eV Angstrom
constexpr double A0 = 0.529177210903;        // Bohr radius, Angstrom
constexpr double PI = 3.14159265358979323846;

double norm_cdf(double z) { return 0.5 * std::erfc(-z / std::sqrt(2.0)); }
void cross(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
bool unit(const double* a) { return std::fabs(std::sqrt(dot(a, a)) - 1.0) < 1e-9; }
// A unit vector perpendicular to the unit vector n.
void perp_axis(const double* n, double* u)
{
    const double a[3] = {std::fabs(n[0]) < 0.9 ? 1.0 : 0.0, std::fabs(n[0]) < 0.9 ? 0.0 : 1.0, 0.0};
    double c[3];
    c[0] = n[1] * a[2] - n[2] * a[1];
    c[1] = n[2] * a[0] - n[0] * a[2];
    c[2] = n[0] * a[1] - n[1] * a[0];
    const double l = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int i = 0; i < 3; ++i) u[i] = c[i] / l;
}
bool inside_chamber(const spx_chamber& ch, const double* p)
{
    return std::hypot(p[0], p[1]) <= ch.radius * (1.0 + 1e-12) && p[2] >= ch.z_lo && p[2] <= ch.z_hi;
}
// Every boundary point of a disc (centre c, axes u, v, radius R) inside the chamber.
bool disc_inside(const spx_chamber& ch, const double* c, const double* u, const double* v, double R)
{
    for (int k = 0; k < 720; ++k) {
        const double a = 2.0 * PI * k / 720.0;
        double p[3];
        for (int i = 0; i < 3; ++i) p[i] = c[i] + R * (std::cos(a) * u[i] + std::sin(a) * v[i]);
        if (!inside_chamber(ch, p)) return false;
    }
    return inside_chamber(ch, c);
}
}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

static int fail(const std::string& msg)
{
    set_error(msg);
    return SPX_EINVAL;
}

static int validate(const spx_config* cfgs, int n_cfgs, const spx_params* p)
{
    if (!cfgs || !p) return fail("null configuration or parameter pointer");
    if (n_cfgs < 1 || n_cfgs >= (1 << 24)) return fail("n_cfgs must be in [1, 2^24)");
    if (!(p->theta_min > 0.0 && p->theta_min < PI)) return fail("theta_min must be in (0, pi)");
    if (!(p->E_th_kT > 0.0)) return fail("E_th_kT must be > 0");
    if (p->event_cap < 1) return fail("event_cap must be >= 1");
    if (p->table_ne < 2 || p->table_ns < 2 || (int64_t)p->table_ne * p->table_ns > (1 << 22))
        return fail("table sizes must be >= 2 and ne*ns <= 2^22");
    if (!(p->log_eps_lo < p->log_eps_hi)) return fail("log_eps_lo must be < log_eps_hi");
    if (p->precision != 32 && p->precision != 64) return fail("precision must be 32 or 64");
    uint64_t total = 0;
    for (int c = 0; c < n_cfgs; ++c) {
        const spx_config& C = cfgs[c];
        const std::string w = "config " + std::to_string(c) + ": ";
        const spx_chamber& ch = C.chamber;
        if (!(ch.radius > 0.0) || !(ch.z_hi > ch.z_lo)) return fail(w + "chamber needs radius > 0 and z_hi > z_lo");
        if (!(ch.pressure >= 0.0)) return fail(w + "pressure must be >= 0");
        if (!(ch.T > 0.0)) return fail(w + "temperature must be > 0");
        if (!(ch.gas_mass > 0.0) || ch.gas_Z < 1) return fail(w + "gas mass and Z must be positive");
        const spx_grid& g = C.grid;
        if (!unit(g.normal) || !unit(g.u_axis) || std::fabs(dot(g.normal, g.u_axis)) > 1e-9)
            return fail(w + "substrate normal and u_axis must be orthonormal");
        if (!(g.half_u > 0.0) || !(g.half_v > 0.0)) return fail(w + "substrate half sizes must be > 0");
        if (g.shape != 0 && g.shape != 1) return fail(w + "substrate shape must be 0 or 1");
        if (g.shape == 1 && g.half_v != g.half_u) return fail(w + "disc substrate needs half_v == half_u");
        if (g.nu < 1 || g.nv < 1 || (int64_t)g.nu * g.nv > (1 << 24)) return fail(w + "need 1 <= nu*nv <= 2^24");
        {
            double gv[3];
            cross(g.normal, g.u_axis, gv);
            if (g.shape == 0) {
                for (int sx = -1; sx <= 1; sx += 2)
                    for (int sy = -1; sy <= 1; sy += 2) {
                        double q[3];
                        for (int i = 0; i < 3; ++i) q[i] = g.center[i] + sx * g.half_u * g.u_axis[i] + sy * g.half_v * gv[i];
                        if (!inside_chamber(ch, q)) return fail(w + "substrate outside the chamber");
                    }
            } else if (!disc_inside(ch, g.center, g.u_axis, gv, g.half_u)) {
                return fail(w + "substrate outside the chamber");
            }
        }
        if (C.n_cathodes < 1 || C.n_cathodes > 255 || !C.cathodes) return fail(w + "need 1..255 cathodes");
        for (int k = 0; k < C.n_cathodes; ++k) {
            const spx_cathode& K = C.cathodes[k];
            const std::string wk = w + "cathode " + std::to_string(k) + ": ";
            if (!unit(K.normal) || !unit(K.u_axis) || std::fabs(dot(K.normal, K.u_axis)) > 1e-9)
                return fail(wk + "normal and u_axis must be orthonormal");
            if (!(K.radius > 0.0)) return fail(wk + "radius must be > 0");
            double kv[3];
            cross(K.normal, K.u_axis, kv);
            if (!disc_inside(ch, K.center, K.u_axis, kv, K.radius)) return fail(wk + "target disc outside the chamber");
            if (K.rt_n == 0) {
                if (!(K.rt_sigma > 0.0) || !(K.rt_lo < K.rt_hi) || K.rt_lo < 0.0 || K.rt_hi > K.radius)
                    return fail(wk + "racetrack needs sigma > 0 and 0 <= rt_lo < rt_hi <= radius");
            } else {
                if (K.rt_n < 2 || K.rt_n > RT_MAX_NODES || !K.rt_profile)
                    return fail(wk + "racetrack profile needs 2.." + std::to_string(RT_MAX_NODES) + " nodes");
                double wsum = 0.0;
                for (int i = 0; i < K.rt_n; ++i) {
                    const double r = K.rt_profile[2 * i], d = K.rt_profile[2 * i + 1];
                    if (!std::isfinite(r) || !std::isfinite(d) || d < 0.0 || r < 0.0 || r > K.radius ||
                        (i > 0 && !(r > K.rt_profile[2 * i - 2])))
                        return fail(wk + "racetrack profile: radii must increase within [0, radius], depths >= 0");
                    if (i > 0) wsum += (d + K.rt_profile[2 * i - 1]) * (r - K.rt_profile[2 * i - 2]);
                }
                if (!(wsum > 0.0)) return fail(wk + "racetrack profile has no erosion");
            }
            if (!(K.U_s > 0.0) || !(K.E_i > 0.0) || !(K.k_cut > 0.0)) return fail(wk + "U_s, E_i, k_cut must be > 0");
            if (!(K.mass > 0.0) || K.Z < 1) return fail(wk + "mass and Z must be positive");
            const double lam = 4.0 * K.mass * ch.gas_mass / ((K.mass + ch.gas_mass) * (K.mass + ch.gas_mass));
            if (!(K.k_cut * lam * K.E_i - K.U_s > 0.0)) return fail(wk + "E_max = k Lambda E_i - U_s must be > 0");
            {
                double norm = 0.0;
                for (int i = 0; i < 6; ++i) {
                    if (!std::isfinite(K.cos_coeff[i])) return fail(wk + "emission coefficients must be finite");
                    norm += K.cos_coeff[i] / (i + 1);
                }
                bool neg = false;
                for (int j = 0; j <= 4096; ++j) {
                    const double mu = j / 4096.0;
                    double f = 0.0, pw = 1.0;
                    for (int i = 0; i < 6; ++i) {
                        f += K.cos_coeff[i] * pw;
                        pw *= mu;
                    }
                    neg = neg || f < 0.0;
                }
                if (neg || !(norm > 0.0))
                    return fail(wk + "emission law sum c_i cos^i must be >= 0 on [0, 90 deg] with a positive integral");
            }
            if (K.n_particles >= (1ull << 32)) return fail(wk + "n_particles must be < 2^32");
            total += K.n_particles;
        }
        if (C.n_objects < 0 || (C.n_objects > 0 && !C.objects)) return fail(w + "bad object list");
        if (C.n_objects + (C.cross_absorb ? C.n_cathodes - 1 : 0) > OBJ_MAX_SEG)
            return fail(w + "more than " + std::to_string(OBJ_MAX_SEG) + " absorbing objects in one run");
        for (int j = 0; j < C.n_objects; ++j) {
            const spx_object& O = C.objects[j];
            const std::string wo = w + "object " + std::to_string(j) + ": ";
            if (O.kind < SPX_OBJ_DISC || O.kind > SPX_OBJ_TUBE) return fail(wo + "unknown kind");
            if (!unit(O.normal)) return fail(wo + "normal must be a unit vector");
            if (!(O.half_u > 0.0)) return fail(wo + "half_u must be > 0");
            double ou[3], ov[3];
            if (O.kind == SPX_OBJ_RECT) {
                if (!unit(O.u_axis) || std::fabs(dot(O.normal, O.u_axis)) > 1e-9)
                    return fail(wo + "normal and u_axis must be orthonormal");
                if (!(O.half_v > 0.0)) return fail(wo + "half_v must be > 0");
                for (int i = 0; i < 3; ++i) ou[i] = O.u_axis[i];
            } else {
                perp_axis(O.normal, ou);
            }
            cross(O.normal, ou, ov);
            bool inside = true;
            if (O.kind == SPX_OBJ_DISC) {
                inside = disc_inside(ch, O.center, ou, ov, O.half_u);
            } else if (O.kind == SPX_OBJ_RECT) {
                for (int a = -1; a <= 1; a += 2)
                    for (int b = -1; b <= 1; b += 2) {
                        double q[3];
                        for (int i = 0; i < 3; ++i) q[i] = O.center[i] + a * O.half_u * ou[i] + b * O.half_v * ov[i];
                        inside = inside && inside_chamber(ch, q);
                    }
            } else {
                if (!(O.length > 0.0)) return fail(wo + "tube length must be > 0");
                double top[3];
                for (int i = 0; i < 3; ++i) top[i] = O.center[i] + O.length * O.normal[i];
                inside = disc_inside(ch, O.center, ou, ov, O.half_u) && disc_inside(ch, top, ou, ov, O.half_u);
            }
            if (!inside) return fail(wo + "object outside the chamber");
        }
    }
    if (total == 0) return fail("every cathode has n_particles == 0");
    return SPX_OK;
}

// Derive the FP64 constants of every segment (the table must exist for lam_th).
static void derive(Plan* P, const spx_config* cfgs, int n_cfgs)
{
    const spx_params& pr = P->params;
    for (int c = 0; c < n_cfgs; ++c) {
        const spx_config& C = cfgs[c];
        const spx_chamber& ch = C.chamber;
        const spx_grid& g = C.grid;
        for (int k = 0; k < C.n_cathodes; ++k) {
            const spx_cathode& K = C.cathodes[k];
            SegHost s{};
            s.cfg = c;
            s.cath = k;
            s.z_mid = 0.5 * (ch.z_lo + ch.z_hi);
            for (int i = 0; i < 3; ++i) {
                s.cat_c[i] = K.center[i] - (i == 2 ? s.z_mid : 0.0);
                s.cat_n[i] = K.normal[i];
                s.cat_u[i] = K.u_axis[i];
                s.sub_c[i] = g.center[i] - (i == 2 ? s.z_mid : 0.0);
                s.sub_n[i] = g.normal[i];
                s.sub_u[i] = g.u_axis[i];
            }
            cross(s.cat_n, s.cat_u, s.cat_v);
            cross(s.sub_n, s.sub_u, s.sub_v);
            s.cat_R = K.radius;
            s.half_u = g.half_u;
            s.half_v = g.half_v;
            s.shape = g.shape;
            s.nu = g.nu;
            s.nv = g.nv;
            s.du = 2.0 * g.half_u / g.nu;
            s.dv = 2.0 * g.half_v / g.nv;
            s.ch_R = ch.radius;
            s.zlo = ch.z_lo - s.z_mid;
            s.zhi = ch.z_hi - s.z_mid;
            s.rt_mu = K.rt_mu;
            s.rt_sig = K.rt_sigma;
            // measured racetrack: cumulative weight F_i = integral_0^{r_i} depth(s) s ds at the nodes
            for (int i = 0; i < K.rt_n; ++i) {
                s.rt_r.push_back(K.rt_profile[2 * i]);
                s.rt_d.push_back(K.rt_profile[2 * i + 1]);
            }
            for (int i = 0; i < 6; ++i) s.cosc[i] = K.cos_coeff[i];
            // absorbing objects of this run: the configuration's, then the other targets
            for (int j = 0; j < C.n_objects; ++j) s.objs.push_back(C.objects[j]);
            if (C.cross_absorb)
                for (int j = 0; j < C.n_cathodes; ++j) {
                    if (j == k) continue;
                    spx_object o{};
                    o.kind = SPX_OBJ_DISC;
                    for (int i = 0; i < 3; ++i) {
                        o.center[i] = C.cathodes[j].center[i];
                        o.normal[i] = C.cathodes[j].normal[i];
                    }
                    o.half_u = o.half_v = C.cathodes[j].radius;
                    s.objs.push_back(o);
                }
            for (auto& o : s.objs) {
                o.center[2] -= s.z_mid;
                if (o.kind != SPX_OBJ_RECT) perp_axis(o.normal, o.u_axis);
            }
            const double al = (K.rt_lo - K.rt_mu) / K.rt_sigma, be = (K.rt_hi - K.rt_mu) / K.rt_sigma;
            s.PhiA = norm_cdf(al);
            s.QB = norm_cdf(-be);
            s.dPhi = norm_cdf(be) - s.PhiA;
            s.Ms = K.mass;
            s.Mg = ch.gas_mass;
            s.Us = K.U_s;
            s.Lambda = 4.0 * s.Ms * s.Mg / ((s.Ms + s.Mg) * (s.Ms + s.Mg));
            s.Emax = K.k_cut * s.Lambda * K.E_i - s.Us;
            s.smax = s.Emax / (s.Emax + s.Us);
            const double a_ang = 0.8853 * A0 * std::pow(std::sqrt((double)K.Z) + std::sqrt((double)ch.gas_Z), -2.0 / 3.0);
            s.a_mm = a_ang * 1e-7;
            s.eps_per_eV = a_ang / ((double)K.Z * (double)ch.gas_Z * E2);
            s.mu_red = s.Ms * s.Mg / (s.Ms + s.Mg);
            s.pressure = ch.pressure;
            s.n_mm3 = ch.pressure / (KB_J * ch.T) * 1e-9;
            s.kT = KB_EV * ch.T;
            s.vth = std::sqrt(s.kT / s.Mg);
            s.vg = std::sqrt(2.0 * s.kT / s.Mg);
            s.E_th = pr.E_th_kT * s.kT;
            s.gas_motion = ch.gas_motion ? 1 : 0;
            s.N = K.n_particles;
            P->seg.push_back(s);
        }
    }
}

// beta_max(eps) linear in log10(eps) on the FP64 table (host copy).
static double betamax_host(const Plan* P, double eps)
{
    const spx_params& pr = P->params;
    const int ne = pr.table_ne;
    double x = (std::log10(eps) - pr.log_eps_lo) / (pr.log_eps_hi - pr.log_eps_lo) * (ne - 1);
    x = x > 0.0 ? x : 0.0;
    x = x < ne - 1 ? x : ne - 1;
    int i = (int)std::floor(x);
    i = i < ne - 2 ? i : ne - 2;
    const double f = x - i;
    return P->h_betamax[i] * (1.0 - f) + P->h_betamax[i + 1] * f;
}

template <typename R> static SegDev<R> to_device(const Plan* P, const SegHost& s)
{
    const spx_params& pr = P->params;
    SegDev<R> d{};
    for (int i = 0; i < 3; ++i) {
        d.cat_c[i] = (R)s.cat_c[i];
        d.cat_n[i] = (R)s.cat_n[i];
        d.cat_u[i] = (R)s.cat_u[i];
        d.cat_v[i] = (R)s.cat_v[i];
        d.sub_c[i] = (R)s.sub_c[i];
        d.sub_n[i] = (R)s.sub_n[i];
        d.sub_u[i] = (R)s.sub_u[i];
        d.sub_v[i] = (R)s.sub_v[i];
    }
    d.cat_R2 = (R)(s.cat_R * s.cat_R);
    d.cat_nc = (R)dot(s.cat_n, s.cat_c);
    d.cat_uc = (R)dot(s.cat_u, s.cat_c);
    d.cat_vc = (R)dot(s.cat_v, s.cat_c);
    d.sub_nc = (R)dot(s.sub_n, s.sub_c);
    d.sub_uc = (R)dot(s.sub_u, s.sub_c);
    d.sub_vc = (R)dot(s.sub_v, s.sub_c);
    d.half_u = (R)s.half_u;
    d.half_v = (R)s.half_v;
    d.inv_du = (R)(1.0 / s.du);
    d.inv_dv = (R)(1.0 / s.dv);
    d.sub_R2 = (R)(s.half_u * s.half_u);
    d.ch_R2 = (R)(s.ch_R * s.ch_R);
    d.zlo = (R)s.zlo;
    d.zhi = (R)s.zhi;
    d.rt_mu = (R)s.rt_mu;
    d.rt_sig = (R)s.rt_sig;
    d.PhiA = (R)s.PhiA;
    d.QB = (R)s.QB;
    d.dPhi = (R)s.dPhi;
    d.Us = (R)s.Us;
    d.smax = (R)s.smax;
    d.two_over_Ms = (R)(2.0 / s.Ms);
    d.half_Ms = (R)(0.5 * s.Ms);
    d.Ms_frac = (R)(s.Ms / (s.Ms + s.Mg));
    d.Mg_frac = (R)(s.Mg / (s.Ms + s.Mg));
    d.half_mu_red = (R)(0.5 * s.mu_red);
    const double sc = (pr.table_ne - 1) / (pr.log_eps_hi - pr.log_eps_lo);
    d.xo_coll = (R)((std::log10(s.eps_per_eV) - pr.log_eps_lo) * sc);
    d.xo_stat = (R)((std::log10(s.eps_per_eV * s.Mg / (s.Ms + s.Mg)) - pr.log_eps_lo) * sc);
    d.n_pia2 = (R)(s.n_mm3 * PI * s.a_mm * s.a_mm);
    d.vth = (R)s.vth;
    d.inv_vg = (R)(1.0 / s.vg);
    d.vg = (R)s.vg;
    d.E_th = (R)s.E_th;
    d.lam_th = (R)s.lam_th;
    d.lam_l2 = (R)(s.lam_th * 0.69314718055994530942);
    d.z_mid = (R)s.z_mid;
    d.shape = s.shape;
    d.nu = s.nu;
    d.nv = s.nv;
    d.gas_motion = s.gas_motion;
    d.vacuum = s.n_mm3 > 0.0 ? 0 : 1;
    d.rt = nullptr;                          // set once the racetrack tables are on the device
    d.obj = nullptr;                         // set once the objects are on the device
    d.n_obj = (int32_t)s.objs.size();
    d.rt_n = (int32_t)s.rt_r.size();
    double norm = 0.0;
    bool pure = true;
    for (int i = 0; i < 6; ++i) {
        norm += s.cosc[i] / (i + 1);
        pure = pure && s.cosc[i] == (i == 1 ? 1.0 : 0.0);
    }
    for (int i = 0; i < 6; ++i) d.cosk[i] = (R)(s.cosc[i] / ((i + 1) * norm));
    d.cos_pure = pure ? 1 : 0;
    d.cfgcat = ((uint32_t)s.cfg << 8) | (uint32_t)s.cath;
    d.bin_off = s.bin_off;
    d.first_rec = s.first_rec;
    d.N = s.N;
    return d;
}

template <typename T> static int dalloc(T** p, size_t n)
{
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * n);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
        return SPX_ENOMEM;
    }
    return SPX_OK;
}

static void release(Plan* P)
{
    if (!P) return;
    if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    void* ptrs[] = {P->d_theta64, P->d_betamax64, P->d_theta32, P->d_betamax32, P->d_seg32,   P->d_seg64,
                    P->d_tfirst,  P->d_torder,    P->d_qstate,  P->d_queue,     P->d_bin_off, P->d_seg_norm,
                    P->d_rt32,    P->d_rt64,      P->d_edges32, P->d_edges64, P->d_obj32,   P->d_obj64};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (hipEvent_t e : P->phase_events) (void)hipEventDestroy(e);
    if (P->done_event) (void)hipEventDestroy(P->done_event);
    if (P->work_stream) (void)hipStreamDestroy(P->work_stream);
    delete P;
}

static int create(const spx_config* cfgs, int n_cfgs, const spx_params* prm, Plan** out)
{
    SPX_TRY(validate(cfgs, n_cfgs, prm));
    int ndev = 0;
    SPX_HIP(hipGetDeviceCount(&ndev));
    if (ndev < 1) {
        set_error("no HIP device");
        return SPX_EDEVICE;
    }
    int dev = 0;
    SPX_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SPX_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error(std::string("libspx is built for gfx950; current device is ") + prop.gcnArchName);
        return SPX_EDEVICE;
    }
    Plan* P = new Plan();
    P->device = dev;
    P->params = *prm;
    P->n_cu = prop.multiProcessorCount;
    derive(P, cfgs, n_cfgs);
    P->n_seg = (int)P->seg.size();
    uint64_t boff = 0, first = 0;
    for (auto& s : P->seg) {
        s.bin_off = boff;
        s.first_rec = first;
        P->h_bin_off.push_back(boff);
        P->h_first.push_back(first);
        boff += (uint64_t)s.nu * s.nv;
        first += s.N;
    }
    P->n_bins_total = boff;
    P->n_particles_total = first;

    int rc = SPX_OK;
    auto chk = [&](int r) {
        if (rc == SPX_OK && r != SPX_OK) rc = r;
        return rc == SPX_OK;
    };
    const int ne = prm->table_ne, ns = prm->table_ns, n = P->n_seg;
    if (hipStreamCreateWithFlags(&P->work_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P->done_event, hipEventDisableTiming) != hipSuccess) {
        set_error("hipStreamCreate / hipEventCreate failed");
        release(P);
        return SPX_EDEVICE;
    }
    chk(dalloc(&P->d_theta64, (size_t)ne * ns)) && chk(dalloc(&P->d_betamax64, ne)) &&
        chk(dalloc(&P->d_theta32, (size_t)ne * ns)) && chk(dalloc(&P->d_betamax32, ne)) &&
        chk(dalloc(&P->d_seg32, n)) && chk(dalloc(&P->d_seg64, n)) && chk(dalloc(&P->d_tfirst, n + 1)) &&
        chk(dalloc(&P->d_torder, n)) && chk(dalloc(&P->d_qstate, QSTATE_WORDS)) && chk(dalloc(&P->d_bin_off, n + 1)) &&
        chk(dalloc(&P->d_seg_norm, n));
    if (rc == SPX_OK) rc = build_tables(P);
    if (rc != SPX_OK) {
        release(P);
        return rc;
    }
    // thermal mean free path and normalisation from the FP64 table
    for (auto& s : P->seg) {
        if (s.n_mm3 > 0.0) {
            const double bm = betamax_host(P, s.eps_per_eV * 1.5 * s.kT);
            const double sig = PI * (s.a_mm * bm) * (s.a_mm * bm);
            s.lam_th = 1.0 / (s.n_mm3 * sig * std::sqrt(1.0 + s.Ms / s.Mg));
        } else {
            s.lam_th = INFINITY;
        }
        P->seg_norm.push_back(s.N ? 1.0 / ((double)s.N * s.du * s.dv) : 0.0);
    }
    std::vector<SegDev<float>> s32;
    std::vector<SegDev<double>> s64;
    for (const auto& s : P->seg) {
        s32.push_back(to_device<float>(P, s));
        s64.push_back(to_device<double>(P, s));
    }
    // measured racetracks: per node interval the normalised cumulative weight and the cubic
    // of the weight integral_r^{r+t} depth(s) s ds (depth linear on the interval), FP64 on the host
    std::vector<RtNode<double>> rt64;
    std::vector<size_t> rt_off(n, 0);
    for (int k = 0; k < n; ++k) {
        const auto& sg = P->seg[k];
        const int m = (int)sg.rt_r.size();
        rt_off[k] = rt64.size();
        if (m == 0) continue;
        std::vector<double> F(m, 0.0), p1(m, 0.0), p2(m, 0.0), p3(m, 0.0);
        for (int i = 0; i + 1 < m; ++i) {
            const double dr = sg.rt_r[i + 1] - sg.rt_r[i], sl = (sg.rt_d[i + 1] - sg.rt_d[i]) / dr;
            const double d0 = sg.rt_d[i], r0 = sg.rt_r[i];
            p1[i] = d0 * r0;
            p2[i] = (d0 + sl * r0) / 2.0;
            p3[i] = sl / 3.0;
            F[i + 1] = F[i] + ((p3[i] * dr + p2[i]) * dr + p1[i]) * dr;
        }
        const double Z = F[m - 1];
        for (int i = 0; i < m; ++i) {
            const bool last = i + 1 == m;
            rt64.push_back(RtNode<double>{sg.rt_r[i], last ? 1.0 : F[i] / Z, p1[i] / Z, p2[i] / Z, p3[i] / Z,
                                          last ? 0.0 : sg.rt_r[i + 1] - sg.rt_r[i]});
        }
    }
    {
        // absorbing objects: per segment a run of ObjDev in one array (FP32 and FP64)
        std::vector<ObjDev<double>> ob64;
        std::vector<size_t> ob_off(n, 0);
        for (int k = 0; k < n; ++k) {
            ob_off[k] = ob64.size();
            for (const auto& o : P->seg[k].objs) {
                ObjDev<double> q{};
                q.kind = o.kind;
                double v[3];
                cross(o.normal, o.u_axis, v);
                for (int i = 0; i < 3; ++i) {
                    q.c[i] = o.center[i];
                    q.n[i] = o.normal[i];
                    q.u[i] = o.u_axis[i];
                    q.v[i] = v[i];
                }
                q.nc = dot(o.normal, o.center);
                q.uc = dot(o.u_axis, o.center);
                q.vc = dot(v, o.center);
                q.hu = o.half_u;
                q.hv = o.kind == SPX_OBJ_RECT ? o.half_v : o.half_u;
                q.r2 = o.half_u * o.half_u;
                q.len = o.length;
                ob64.push_back(q);
            }
        }
        if (!ob64.empty()) {
            std::vector<ObjDev<float>> ob32;
            for (const auto& q : ob64) {
                ObjDev<float> f{};
                f.kind = q.kind;
                for (int i = 0; i < 3; ++i) {
                    f.c[i] = (float)q.c[i];
                    f.n[i] = (float)q.n[i];
                    f.u[i] = (float)q.u[i];
                    f.v[i] = (float)q.v[i];
                }
                f.nc = (float)q.nc;
                f.uc = (float)q.uc;
                f.vc = (float)q.vc;
                f.hu = (float)q.hu;
                f.hv = (float)q.hv;
                f.r2 = (float)q.r2;
                f.len = (float)q.len;
                ob32.push_back(f);
            }
            if (dalloc(&P->d_obj32, ob32.size()) != SPX_OK || dalloc(&P->d_obj64, ob64.size()) != SPX_OK ||
                hipMemcpy(P->d_obj32, ob32.data(), sizeof(ObjDev<float>) * ob32.size(), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(P->d_obj64, ob64.data(), sizeof(ObjDev<double>) * ob64.size(), hipMemcpyHostToDevice) != hipSuccess) {
                set_error("copying the absorbing objects to the device failed");
                release(P);
                return SPX_EDEVICE;
            }
            for (int k = 0; k < n; ++k)
                if (!P->seg[k].objs.empty()) {
                    s32[k].obj = P->d_obj32 + ob_off[k];
                    s64[k].obj = P->d_obj64 + ob_off[k];
                }
        }
    }
    {
        double e[SPX_ARRIVAL_E_BINS + 1 + SPX_ARRIVAL_A_BINS + 1];
        arrival_edges(e, e + SPX_ARRIVAL_E_BINS + 1);
        float f[SPX_ARRIVAL_E_BINS + 1 + SPX_ARRIVAL_A_BINS + 1];
        const size_t ne = sizeof(e) / sizeof(e[0]);
        for (size_t i = 0; i < ne; ++i) f[i] = (float)e[i];
        if (dalloc(&P->d_edges32, ne) != SPX_OK || dalloc(&P->d_edges64, ne) != SPX_OK ||
            hipMemcpy(P->d_edges32, f, sizeof(f), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(P->d_edges64, e, sizeof(e), hipMemcpyHostToDevice) != hipSuccess) {
            set_error("copying the arrival bin edges to the device failed");
            release(P);
            return SPX_EDEVICE;
        }
    }
    if (!rt64.empty()) {
        std::vector<RtNode<float>> rt32;
        for (const auto& q : rt64)
            rt32.push_back(RtNode<float>{(float)q.r, (float)q.C, (float)q.p1, (float)q.p2, (float)q.p3, (float)q.dr});
        if (dalloc(&P->d_rt32, rt32.size()) != SPX_OK || dalloc(&P->d_rt64, rt64.size()) != SPX_OK ||
            hipMemcpy(P->d_rt32, rt32.data(), sizeof(RtNode<float>) * rt32.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(P->d_rt64, rt64.data(), sizeof(RtNode<double>) * rt64.size(), hipMemcpyHostToDevice) != hipSuccess) {
            set_error("copying the racetrack tables to the device failed");
            release(P);
            return SPX_EDEVICE;
        }
        for (int k = 0; k < n; ++k)
            if (!P->seg[k].rt_r.empty()) {
                s32[k].rt = P->d_rt32 + rt_off[k];
                s64[k].rt = P->d_rt64 + rt_off[k];
            }
    }
    // ticket order: highest pressure (longest histories) first
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return P->seg[a].pressure > P->seg[b].pressure; });
    std::vector<uint64_t> tfirst(n + 1, 0);
    for (int o = 0; o < n; ++o) tfirst[o + 1] = tfirst[o] + P->seg[order[o]].N;
    P->n_tickets = tfirst[n];
    if (prm->precision == 32) {
        // thermalisation queue of one round of the batched path (48 B per ticket of a round)
        // thermalised atoms of a round, plus the slots a resident wave may leave unused
        const uint64_t r = rounds_of(P->n_tickets);
        const uint64_t waves = std::max<uint64_t>(QUEUE_SLACK_WAVES, (uint64_t)P->n_cu * 32);
        P->queue_cap = (r ? (P->n_tickets + r - 1) / r : 0) + waves * QUEUE_CHUNK;
        if (dalloc(&P->d_queue, P->queue_cap) != SPX_OK) {
            set_error("hipMalloc of the thermalisation queue (" + std::to_string(P->queue_cap * sizeof(ThermRec)) +
                      " bytes) failed");
            release(P);
            return SPX_ENOMEM;
        }
    }
    std::vector<uint64_t> bo(P->h_bin_off);
    bo.push_back(P->n_bins_total);
    hipStream_t st = P->work_stream;
    bool ok = hipMemcpyAsync(P->d_seg32, s32.data(), sizeof(SegDev<float>) * n, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(P->d_seg64, s64.data(), sizeof(SegDev<double>) * n, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(P->d_tfirst, tfirst.data(), sizeof(uint64_t) * (n + 1), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(P->d_torder, order.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(P->d_bin_off, bo.data(), sizeof(uint64_t) * (n + 1), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(P->d_seg_norm, P->seg_norm.data(), sizeof(double) * n, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        set_error("copying plan constants to the device failed");
        release(P);
        return SPX_EDEVICE;
    }
    int bpc = 0, bpc_d = 0;
    if (occupancy_transport32(P, P->threads, &bpc, &bpc_d) != SPX_OK || bpc < 1 || bpc_d < 1) {
        release(P);
        set_error("occupancy query failed for the transport kernels");
        return SPX_EDEVICE;
    }
    P->max_blocks_per_cu = bpc;
    P->blocks = bpc * P->n_cu;
    P->blocks_diff = std::min(P->blocks, bpc_d * P->n_cu);
    *out = P;
    return SPX_OK;
}

// A sink that keeps the launches of a run.
struct ListSink : LaunchSink {
    std::vector<KLaunch> L;
    int put(const KLaunch& k) override
    {
        if (k.n_args < 0 || !k.func) {
            set_error("internal: malformed kernel launch");
            return SPX_ESTATE;
        }
        L.push_back(k);
        return SPX_OK;
    }
};

Shape plan_shape(const Plan* P)
{
    Shape sh;
    sh.blocks = P->blocks;
    sh.blocks_diff = P->blocks_diff;
    sh.threads = P->threads;
    sh.refill_min = P->refill_min;
    sh.refill_ballistic = P->refill_ballistic;
    sh.defer_min = P->defer_min;
    return sh;
}

// The graph of a run: its launches as a chain of kernel nodes, with the phase events of each
// round (recorded before the ballistic kernel, between the kernels and after the diffusive one).
static int build_graph(Plan* P, const std::vector<KLaunch>& L)
{
    const size_t n_rounds = (size_t)rounds_of(P->n_tickets);
    while (P->phase_events.size() < 3 * n_rounds) {
        hipEvent_t e = nullptr;
        SPX_HIP(hipEventCreate(&e));
        P->phase_events.push_back(e);
    }
    if (P->graph_exec) {
        SPX_HIP(hipGraphExecDestroy(P->graph_exec));
        P->graph_exec = nullptr;
    }
    if (P->graph) {
        SPX_HIP(hipGraphDestroy(P->graph));
        P->graph = nullptr;
    }
    P->graph_launches.clear();
    P->graph_nodes.clear();
    hipGraph_t g = nullptr;
    SPX_HIP(hipGraphCreate(&g, 0));
    P->graph = g;
    hipGraphNode_t prev = nullptr;
    size_t round = 0;
    auto chain_event = [&](hipEvent_t e) -> int {
        hipGraphNode_t n = nullptr;
        SPX_HIP(hipGraphAddEventRecordNode(&n, g, prev ? &prev : nullptr, prev ? 1 : 0, e));
        prev = n;
        return SPX_OK;
    };
    for (const KLaunch& k : L) {
        if (k.phase == 1) {
            if (round >= n_rounds) {
                set_error("internal: more rounds in the run than in the plan");
                return SPX_ESTATE;
            }
            SPX_TRY(chain_event(P->phase_events[3 * round]));
        }
        void* args[8];
        k.pointers(args);
        hipKernelNodeParams kp{};
        kp.func = const_cast<void*>(k.func);
        kp.gridDim = k.grid;
        kp.blockDim = k.block;
        kp.sharedMemBytes = k.smem;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t n = nullptr;
        SPX_HIP(hipGraphAddKernelNode(&n, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        prev = n;
        P->graph_launches.push_back(k);
        P->graph_nodes.push_back(n);
        if (k.phase == 1) SPX_TRY(chain_event(P->phase_events[3 * round + 1]));
        if (k.phase == 2) SPX_TRY(chain_event(P->phase_events[3 * round++ + 2]));
    }
    if (round != n_rounds) {
        set_error("internal: unexpected number of rounds in the transport graph");
        return SPX_ESTATE;
    }
    SPX_HIP(hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0));
    ++P->graph_instantiations;
    return SPX_OK;
}

// A run of the batched path replays the plan's graph.  The graph is built once per launch
// geometry and set of outputs; a new seed or new output buffers only replace the arguments of
// the kernel nodes in the instantiated graph.
static int run(Plan* P, uint64_t seed, const Outputs& o, hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SPX_HIP(hipStreamIsCapturing(st, &cs));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    // runs on other streams share the plan's queue and counters: wait for the last one
    if (P->done_recorded && !capturing) SPX_HIP(hipStreamWaitEvent(st, P->done_event, 0));
    if (P->params.precision == 64) {
        SPX_TRY(launch_transport64(P, seed, o, st));
    } else if (capturing) {
        // inside a stream capture the kernels go straight onto the capturing stream, so that
        // they become nodes of the caller's graph (a launch of the plan's own graph would not be
        // recorded); the runs of the plan in that graph share its queue and are ordered by the
        // caller
        QueueMem q;
        q.queue = P->d_queue;
        q.cap = P->queue_cap;
        q.qstate = P->d_qstate;
        StreamSink ss(st, nullptr);
        SPX_TRY(build_transport32(P, seed, o, P->d_tfirst, P->n_tickets, plan_shape(P), q, ss));
    } else {
        QueueMem q;
        q.queue = P->d_queue;
        q.cap = P->queue_cap;
        q.qstate = P->d_qstate;
        ListSink ls;
        SPX_TRY(build_transport32(P, seed, o, P->d_tfirst, P->n_tickets, plan_shape(P), q, ls));
        bool same = P->graph_exec && ls.L.size() == P->graph_launches.size();
        for (size_t i = 0; same && i < ls.L.size(); ++i) same = ls.L[i].same_shape(P->graph_launches[i]);
        if (!same) {
            SPX_TRY(build_graph(P, ls.L));
        } else {
            // an instantiated graph may keep its kernel arguments in device memory: replace them
            // only once the previous launch of the graph has finished
            bool waited = false;
            for (size_t i = 0; i < ls.L.size(); ++i) {
                if (ls.L[i].same_args(P->graph_launches[i])) continue;
                if (!waited && P->done_recorded) SPX_HIP(hipEventSynchronize(P->done_event));
                waited = true;
                const KLaunch& k = ls.L[i];
                void* args[8];
                k.pointers(args);
                hipKernelNodeParams kp{};
                kp.func = const_cast<void*>(k.func);
                kp.gridDim = k.grid;
                kp.blockDim = k.block;
                kp.sharedMemBytes = k.smem;
                kp.kernelParams = args;
                kp.extra = nullptr;
                SPX_HIP(hipGraphExecKernelNodeSetParams(P->graph_exec, P->graph_nodes[i], &kp));
                P->graph_launches[i] = k;
                ++P->graph_updates;
            }
        }
        SPX_HIP(hipGraphLaunch(P->graph_exec, st));
    }
    if (!capturing) {
        SPX_HIP(hipEventRecord(P->done_event, st));
        P->done_recorded = true;
    }
    return SPX_OK;
}

// Time FP32 transport launch shapes on a reduced ticket space (the first n_tune
// particles of every segment) and keep the fastest.  Outputs go to scratch.
static int autotune(Plan* P, hipStream_t st)
{
    const int n = P->n_seg;
    // The tuning sample keeps the plan's mix: the same fraction of every segment, the whole
    // plan up to 4e7 particles, else at least ~48 histories per resident lane: a persistent
    // launch ends in a tail of the longest histories whose share of the time shrinks with the
    // work per lane, and a sample with too little work per lane favours shapes that only
    // shorten that tail.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SPX_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) {
        set_error("spx_autotune cannot run inside a stream capture (it times and synchronises)");
        return SPX_ESTATE;
    }
    if (P->done_recorded) SPX_HIP(hipStreamWaitEvent(st, P->done_event, 0));
    int bpc_max = 0, bpc_dmax = 0;
    SPX_TRY(occupancy_transport32(P, 256, &bpc_max, &bpc_dmax));
    const double lanes = (double)std::max(1, bpc_max) * P->n_cu * 256.0;
    const double frac =
        std::min(1.0, std::max(48.0 * lanes, 4e7) / (double)std::max<uint64_t>(1, P->n_particles_total));
    std::vector<uint64_t> tf(n + 1, 0);
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return P->seg[a].pressure > P->seg[b].pressure; });
    for (int o = 0; o < n; ++o) {
        const uint64_t Nk = P->seg[order[o]].N;
        tf[o + 1] = tf[o] + std::min<uint64_t>(Nk, (uint64_t)std::ceil(frac * (double)Nk));
    }
    if (tf[n] == 0) return SPX_OK;     // no particles: nothing to time, the defaults stay
    uint64_t *d_tf = nullptr, *d_counts = nullptr, *d_ctr = nullptr;
    SPX_TRY(dalloc(&d_tf, n + 1));
    int rc = dalloc(&d_counts, P->n_bins_total);
    if (rc == SPX_OK) rc = dalloc(&d_ctr, (size_t)n * N_COUNTERS);
    // events around the two phases of every round of the sample
    std::vector<hipEvent_t> ev(3 * rounds_of(tf[n]), nullptr);
    for (auto& e : ev)
        if (rc == SPX_OK && hipEventCreate(&e) != hipSuccess) rc = SPX_EDEVICE;
    if (rc == SPX_OK && hipMemcpyAsync(d_tf, tf.data(), sizeof(uint64_t) * (n + 1), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = SPX_EDEVICE;
    // One launch shape on the sample, best of two runs for each phase on its own: the ballistic
    // kernel's time depends on the ballistic refill threshold, the diffusive kernel's on the
    // diffusive refill and deferral thresholds, so each threshold is chosen by the time of its
    // own kernel and not by a step total in which the other kernel's noise can hide it.
    struct PhaseMs {
        float b = 1e30f, d = 1e30f;
    };
    auto time_shape = [&](int blocks, int blocks_d, int t, int rmin, int rbal, int defer) -> PhaseMs {
        PhaseMs best;
        for (int rep = 0; rep < 2 && rc == SPX_OK; ++rep) {
            Outputs to;
            to.counts = d_counts;
            to.counters = d_ctr;
            Shape sh;
            sh.blocks = blocks;
            sh.blocks_diff = blocks_d;
            sh.threads = t;
            sh.refill_min = rmin;
            sh.refill_ballistic = rbal;
            sh.defer_min = defer;
            QueueMem q;
            q.queue = P->d_queue;
            q.cap = P->queue_cap;
            q.qstate = P->d_qstate;
            StreamSink ss(st, ev.data());
            if (rc == SPX_OK) rc = build_transport32(P, 0x5eed, to, d_tf, tf[n], sh, q, ss);
            if (rc == SPX_OK && hipEventSynchronize(ev.back()) != hipSuccess) rc = SPX_EDEVICE;
            float b = 0.f, d = 0.f;
            for (size_t r = 0; r + 2 < ev.size() && rc == SPX_OK; r += 3) {
                float t1 = 0.f, t2 = 0.f;
                if (hipEventElapsedTime(&t1, ev[r], ev[r + 1]) != hipSuccess ||
                    hipEventElapsedTime(&t2, ev[r + 1], ev[r + 2]) != hipSuccess)
                    rc = SPX_EDEVICE;
                b += t1;
                d += t2;
            }
            if (rc == SPX_OK) {
                best.b = std::min(best.b, b);
                best.d = std::min(best.d, d);
            }
        }
        return best;
    };
    float best = 1e30f, best_d = 1e30f;
    int bb = P->blocks, bd = P->blocks_diff, bt = P->threads, br = P->refill_min, bm = P->refill_ballistic;
    int bdef = DEFER_MIN;
    const int thread_opts[] = {256, 512, 1024};
    // (refill_min, refill_ballistic): four runs measure four values of each threshold
    const int mode_opts[][2] = {{2, 12}, {4, 16}, {8, 24}, {16, 8}};
    for (int t : thread_opts) {
        if (rc != SPX_OK) break;
        int bpc = 0, bpc_d = 0;
        if (occupancy_transport32(P, t, &bpc, &bpc_d) != SPX_OK || bpc < 1 || bpc_d < 1) continue;
        const int blocks = bpc * P->n_cu, blocks_d = std::min(blocks, bpc_d * P->n_cu);
        PhaseMs tb;
        int rmin = mode_opts[0][0], rbal = mode_opts[0][1];
        for (const auto& ro : mode_opts) {
            const PhaseMs ms = time_shape(blocks, blocks_d, t, ro[0], ro[1], DEFER_MIN);
            if (rc != SPX_OK) break;
            if (ms.b < tb.b) {
                tb.b = ms.b;
                rbal = ro[1];
            }
            if (ms.d < tb.d) {
                tb.d = ms.d;
                rmin = ro[0];
            }
        }
        if (rc == SPX_OK && tb.b + tb.d < best) {
            best = tb.b + tb.d;
            best_d = tb.d;
            bb = blocks;
            bd = blocks_d;
            bt = t;
            br = rmin;
            bm = rbal;
        }
    }
    // then the deferral threshold for that shape, by the diffusive kernel's time: more held
    // steps per test pass pays off where steps leave their clearance balls often (near
    // surfaces, absorbing objects)
    for (int defer = 2 * DEFER_MIN; defer <= 4 * DEFER_MIN && rc == SPX_OK; defer *= 2) {
        const PhaseMs ms = time_shape(bb, bd, bt, br, bm, defer);
        if (rc != SPX_OK || !(ms.d < best_d)) break;     // doubling again only while it helps
        best_d = ms.d;
        bdef = defer;
    }
    // where doubling did not help, half of it: fewer held steps per test pass pays off where
    // walks are short and a held lane would otherwise idle longer
    if (rc == SPX_OK && bdef == DEFER_MIN) {
        const PhaseMs ms = time_shape(bb, bd, bt, br, bm, DEFER_MIN / 2);
        if (rc == SPX_OK && ms.d < best_d) bdef = DEFER_MIN / 2;
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipFree(d_tf);
    if (d_counts) (void)hipFree(d_counts);
    if (d_ctr) (void)hipFree(d_ctr);
    if (rc != SPX_OK) {
        if (rc == SPX_EDEVICE) set_error("autotune: HIP error while timing launch shapes");
        return rc;
    }
    P->blocks = bb;
    P->blocks_diff = bd;
    P->defer_min = bdef;
    P->threads = bt;
    P->refill_min = br;
    P->refill_ballistic = bm;
    return SPX_OK;
}

}  // namespace spx

using namespace spx;

__global__ void k_philox(const uint32_t* __restrict__ ctr, uint32_t k0, uint32_t k1, uint32_t* __restrict__ out,
                         uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    const uint4 r = philox4x32_10(c, k0, k1);
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

extern "C" {

int spx_plan_create(const spx_config* h_cfgs, int32_t n_cfgs, const spx_params* h_params, spx_plan** out)
{
    if (!out) return fail("null output pointer");
    try {
        return create(h_cfgs, n_cfgs, h_params, out);
    } catch (const std::exception& e) {
        set_error(std::string("spx_plan_create: ") + e.what());
        return SPX_ENOMEM;
    }
}

int spx_plan_query(const spx_plan* P, uint64_t* n_bins_total, uint64_t* n_counters, uint64_t* n_particles_total,
                   int32_t* n_segments)
{
    if (!P) return fail("null plan");
    if (n_bins_total) *n_bins_total = P->n_bins_total;
    if (n_counters) *n_counters = (uint64_t)P->n_seg * N_COUNTERS;
    if (n_particles_total) *n_particles_total = P->n_particles_total;
    if (n_segments) *n_segments = P->n_seg;
    return SPX_OK;
}

int spx_plan_layout(const spx_plan* P, uint64_t* h_bin_off, uint64_t* h_first)
{
    if (!P) return fail("null plan");
    if (h_bin_off) std::memcpy(h_bin_off, P->h_bin_off.data(), sizeof(uint64_t) * P->n_seg);
    if (h_first) std::memcpy(h_first, P->h_first.data(), sizeof(uint64_t) * P->n_seg);
    return SPX_OK;
}

int spx_run(spx_plan* P, uint64_t seed, uint64_t* d_counts, uint64_t* d_counters, double* d_profiles,
            spx_record* d_records, void* stream)
{
    if (!P) return fail("null plan");
    if (!d_counts || !d_counters) return fail("spx_run: d_counts and d_counters are required");
    Outputs o;
    o.counts = d_counts;
    o.counters = d_counters;
    o.profiles = d_profiles;
    o.records = d_records;
    try {
        SPX_HIP(hipSetDevice(P->device));
        return run(P, seed, o, (hipStream_t)stream);
    } catch (const std::exception& e) {
        set_error(std::string("spx_run: ") + e.what());
        return SPX_ENOMEM;
    }
}

int spx_run_ex(spx_plan* P, uint64_t seed, const spx_outputs* out, void* stream)
{
    if (!P || !out) return fail("null argument");
    if (!out->counts || !out->counters) return fail("spx_run_ex: counts and counters are required");
    const int na = (out->arrival_energy != nullptr) + (out->arrival_angle != nullptr) + (out->energy_sum != nullptr);
    if (na != 0 && na != 3) return fail("spx_run_ex: the arrival outputs go together (all three or none)");
    Outputs o;
    o.counts = out->counts;
    o.counters = out->counters;
    o.profiles = out->profiles;
    o.records = out->records;
    o.arr_E = out->arrival_energy;
    o.arr_A = out->arrival_angle;
    o.esum = out->energy_sum;
    try {
        SPX_HIP(hipSetDevice(P->device));
        return run(P, seed, o, (hipStream_t)stream);
    } catch (const std::exception& e) {
        set_error(std::string("spx_run_ex: ") + e.what());
        return SPX_ENOMEM;
    }
}

int spx_arrival_edges(double* e64, double* c64, float* e32, float* c32)
{
    double e[SPX_ARRIVAL_E_BINS + 1], c[SPX_ARRIVAL_A_BINS + 1];
    arrival_edges(e, c);
    for (int k = 0; k <= SPX_ARRIVAL_E_BINS; ++k) {
        if (e64) e64[k] = e[k];
        if (e32) e32[k] = (float)e[k];
    }
    for (int k = 0; k <= SPX_ARRIVAL_A_BINS; ++k) {
        if (c64) c64[k] = c[k];
        if (c32) c32[k] = (float)c[k];
    }
    return SPX_OK;
}

int spx_autotune(spx_plan* P, void* stream)
{
    if (!P) return fail("null plan");
    if (P->params.precision != 32) return SPX_OK;
    SPX_HIP(hipSetDevice(P->device));
    return autotune(P, (hipStream_t)stream);
}

int spx_get_launch(const spx_plan* P, int32_t* blocks, int32_t* threads, int32_t* refill_min,
                   int32_t* refill_ballistic, int32_t* defer_min)
{
    if (!P) return fail("null plan");
    if (blocks) *blocks = P->blocks;
    if (threads) *threads = P->threads;
    if (refill_min) *refill_min = P->refill_min;
    if (refill_ballistic) *refill_ballistic = P->refill_ballistic;
    if (defer_min) *defer_min = P->defer_min;
    return SPX_OK;
}

int spx_set_launch(spx_plan* P, int32_t blocks, int32_t threads, int32_t refill_min, int32_t refill_ballistic,
                   int32_t defer_min)
{
    if (!P) return fail("null plan");
    if (threads < 64 || threads > 1024 || (threads & 63)) return fail("threads must be a multiple of 64 in [64, 1024]");
    if (refill_min < 1 || refill_min > 64) return fail("refill_min must be in [1, 64]");
    if (refill_ballistic < 1 || refill_ballistic > 64) return fail("refill_ballistic must be in [1, 64]");
    if (defer_min < 1 || defer_min > 64) return fail("defer_min must be in [1, 64]");
    int bpc = 0, bpc_d = 0;
    SPX_TRY(occupancy_transport32(P, threads, &bpc, &bpc_d));
    if (bpc < 1 || bpc_d < 1) return fail("transport kernels do not fit with this block size");
    // a persistent grid larger than the resident limit would still be correct, but it is never
    // useful: each kernel runs at most its own resident grid
    const int limit = bpc * P->n_cu;
    P->blocks = (blocks <= 0 || blocks > limit) ? limit : blocks;
    P->blocks_diff = std::min(P->blocks, bpc_d * P->n_cu);
    P->threads = threads;
    P->refill_min = refill_min;
    P->refill_ballistic = refill_ballistic;
    P->defer_min = defer_min;
    return SPX_OK;
}

int spx_get_table(const spx_plan* P, double* h_theta, double* h_betamax)
{
    if (!P || !h_theta || !h_betamax) return fail("null argument");
    const size_t ne = P->params.table_ne, ns = P->params.table_ns;
    SPX_HIP(hipMemcpyAsync(h_theta, P->d_theta64, sizeof(double) * ne * ns, hipMemcpyDeviceToHost, P->work_stream));
    SPX_HIP(hipMemcpyAsync(h_betamax, P->d_betamax64, sizeof(double) * ne, hipMemcpyDeviceToHost, P->work_stream));
    SPX_HIP(hipStreamSynchronize(P->work_stream));
    return SPX_OK;
}

int spx_segment_info(const spx_plan* P, int32_t seg, double* out)
{
    if (!P || !out) return fail("null argument");
    if (seg < 0 || seg >= P->n_seg) return fail("segment index out of range");
    const SegHost& s = P->seg[seg];
    const double v[16] = {s.Lambda, s.Emax, s.smax, s.a_mm, s.eps_per_eV, s.n_mm3, s.kT, s.E_th,
                          s.lam_th, s.PhiA, s.QB,   s.dPhi, s.mu_red,     s.vth,   s.vg, s.z_mid};
    std::memcpy(out, v, sizeof(v));
    return SPX_OK;
}

int spx_philox(const uint32_t* d_ctr, uint32_t key_lo, uint32_t key_hi, uint32_t* d_out, uint64_t n, void* stream)
{
    if (!d_ctr || !d_out) return fail("null argument");
    if (n == 0) return SPX_OK;
    const uint64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffull) return fail("too many counters");
    hipLaunchKernelGGL(k_philox, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, d_ctr, key_lo, key_hi,
                       d_out, n);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

int spx_area_centres(int32_t n_areas, double pitch, double* h_out)
{
    if (n_areas < 1 || !(pitch > 0.0) || !h_out) return fail("spx_area_centres: invalid arguments");
    const int m = (int)std::ceil(std::sqrt((double)n_areas)) + 2;
    struct Pt {
        int64_t r2;
        double ang;
        int i, j;
    };
    std::vector<Pt> pts;
    for (int i = -m; i <= m; ++i)
        for (int j = -m; j <= m; ++j) {
            double a = std::atan2((double)j, (double)i);
            if (a < 0.0) a += 2.0 * PI;
            pts.push_back({(int64_t)i * i + (int64_t)j * j, a, i, j});
        }
    std::sort(pts.begin(), pts.end(), [](const Pt& a, const Pt& b) {
        return a.r2 != b.r2 ? a.r2 < b.r2 : a.ang < b.ang;
    });
    for (int k = 0; k < n_areas; ++k) {
        h_out[2 * k] = pitch * pts[k].i;
        h_out[2 * k + 1] = pitch * pts[k].j;
    }
    return SPX_OK;
}

int spx_phase_times(spx_plan* P, float* ms_ballistic, float* ms_diffusive)
{
    if (!P || !ms_ballistic || !ms_diffusive) return fail("null argument");
    if (P->params.precision != 32 || !P->graph_exec) {
        set_error("no batched FP32 run of this plan yet");
        return SPX_ESTATE;
    }
    SPX_HIP(hipSetDevice(P->device));
    const size_t n_ev = 3 * (size_t)rounds_of(P->n_tickets);
    float b = 0.f, d = 0.f;
    for (size_t r = 0; r + 2 < n_ev; r += 3) {
        SPX_HIP(hipEventSynchronize(P->phase_events[r + 2]));
        float t1 = 0.f, t2 = 0.f;
        SPX_HIP(hipEventElapsedTime(&t1, P->phase_events[r], P->phase_events[r + 1]));
        SPX_HIP(hipEventElapsedTime(&t2, P->phase_events[r + 1], P->phase_events[r + 2]));
        b += t1;
        d += t2;
    }
    *ms_ballistic = b;
    *ms_diffusive = d;
    return SPX_OK;
}

int spx_graph_info(const spx_plan* P, uint64_t* instantiations, uint64_t* node_updates)
{
    if (!P) return fail("null plan");
    if (instantiations) *instantiations = P->graph_instantiations;
    if (node_updates) *node_updates = P->graph_updates;
    return SPX_OK;
}

void spx_plan_destroy(spx_plan* P)
{
    if (P) (void)hipSetDevice(P->device);
    release(P);
}

const char* spx_last_error(void) { return g_error.c_str(); }

int32_t spx_version(void) { return 100; }

}  // extern "C"
