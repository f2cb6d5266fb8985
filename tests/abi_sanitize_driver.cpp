// Test fixture: drives the host side of the C-ABI (validation of configurations and parameters,
// the host-only entry points, the argument checks of the device entry points) in a process
// built with the host sanitizers, against a copy of the library whose host code is built with
// them too.  Prints "ok" and returns 0 when every call behaves as include/spx.h states.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "spx.h"

static int g_fail = 0;

static void check(bool ok, const char* what)
{
    if (!ok) {
        std::printf("FAILED: %s (last error: %s)\n", what, spx_last_error());
        ++g_fail;
    }
}

struct Setup {
    spx_cathode cat{};
    spx_config cfg{};
    spx_params prm{};
    std::vector<double> profile;
    std::vector<spx_object> objects;
};

// A single planar Ni target 100 mm below a 100 x 100 mm substrate in Ar at 0.5 Pa.
static Setup valid()
{
    Setup s;
    spx_cathode& c = s.cat;
    c.center[2] = 50.0;
    c.normal[2] = 1.0;
    c.u_axis[0] = 1.0;
    c.radius = 25.4;
    c.rt_mu = 12.0;
    c.rt_sigma = 3.0;
    c.rt_lo = 2.0;
    c.rt_hi = 24.0;
    c.U_s = 4.44;
    c.E_i = 400.0;
    c.k_cut = 1.0;
    c.mass = 58.69;
    c.Z = 28;
    c.rt_n = 0;
    c.cos_coeff[1] = 1.0;
    c.n_particles = 1000;
    spx_config& g = s.cfg;
    g.chamber = spx_chamber{200.0, 0.0, 300.0, 0.5, 300.0, 39.948, 18, 1};
    g.grid.center[2] = 150.0;
    g.grid.normal[2] = -1.0;
    g.grid.u_axis[0] = 1.0;
    g.grid.half_u = g.grid.half_v = 50.0;
    g.grid.shape = 0;
    g.grid.nu = g.grid.nv = 50;
    g.n_cathodes = 1;
    g.cathodes = &s.cat;
    s.prm = spx_params{0.1, 3.0, 1u << 20, 256, 257, 32, -10.0, 0.0};
    return s;
}

static int create(Setup& s)
{
    s.cfg.cathodes = &s.cat;
    if (!s.profile.empty()) {
        s.cat.rt_profile = s.profile.data();
        s.cat.rt_n = (int32_t)(s.profile.size() / 2);
    }
    if (!s.objects.empty()) {
        s.cfg.objects = s.objects.data();
        s.cfg.n_objects = (int32_t)s.objects.size();
    }
    spx_plan* p = nullptr;
    const int rc = spx_plan_create(&s.cfg, 1, &s.prm, &p);
    if (p) spx_plan_destroy(p);
    return rc;
}

static void rejects(Setup s, const char* what)
{
    const int rc = create(s);
    check(rc == SPX_EINVAL, what);
    check(std::strlen(spx_last_error()) > 0, what);
}

int main()
{
    check(spx_version() >= 100, "version");
    {
        Setup s = valid();
        const int rc = create(s);
        // without a GPU the valid plan fails at the device (SPX_EDEVICE); with one it is built
        check(rc == SPX_OK || rc == SPX_EDEVICE, "valid configuration");
    }
    { Setup s = valid(); s.cfg.chamber.pressure = -1.0; rejects(s, "negative pressure"); }
    { Setup s = valid(); s.cfg.chamber.T = 0.0; rejects(s, "zero temperature"); }
    { Setup s = valid(); s.cat.n_particles = 0; rejects(s, "no particles"); }
    { Setup s = valid(); s.cat.n_particles = 1ull << 32; rejects(s, "too many particles"); }
    { Setup s = valid(); s.cat.rt_lo = 30.0; rejects(s, "racetrack bounds"); }
    { Setup s = valid(); s.cat.mass = -1.0; rejects(s, "negative mass"); }
    { Setup s = valid(); s.cat.E_i = 1.0; rejects(s, "E_max below zero"); }
    { Setup s = valid(); std::memset(s.cat.cos_coeff, 0, sizeof s.cat.cos_coeff); rejects(s, "empty emission law"); }
    { Setup s = valid(); s.cat.cos_coeff[5] = -2.0; rejects(s, "negative emission law"); }
    { Setup s = valid(); s.cat.center[0] = 190.0; rejects(s, "target outside the chamber"); }
    { Setup s = valid(); s.cfg.grid.nu = 0; rejects(s, "empty grid"); }
    { Setup s = valid(); s.cfg.grid.normal[2] = -2.0; rejects(s, "grid frame not orthonormal"); }
    { Setup s = valid(); s.cfg.n_cathodes = 0; rejects(s, "no cathodes"); }
    { Setup s = valid(); s.profile = {0.0, 1.0}; rejects(s, "one-node racetrack profile"); }
    { Setup s = valid(); s.profile = {0.0, 1.0, 5.0, 1.0, 4.0, 1.0}; rejects(s, "radii not increasing"); }
    { Setup s = valid(); s.profile = {0.0, 1.0, 5.0, -1.0}; rejects(s, "negative depth"); }
    { Setup s = valid(); s.profile = {0.0, 0.0, 5.0, 0.0}; rejects(s, "no erosion"); }
    { Setup s = valid(); s.profile = {0.0, 1.0, 30.0, 1.0}; rejects(s, "profile beyond the target"); }
    {
        Setup s = valid();
        s.profile.clear();
        for (int i = 0; i <= 256; ++i) {
            s.profile.push_back(0.09 * i);
            s.profile.push_back(1.0);
        }
        rejects(s, "too many racetrack nodes");
    }
    {
        Setup s = valid();
        spx_object o{};
        o.kind = SPX_OBJ_TUBE;
        o.normal[2] = 1.0;
        o.half_u = 10.0;
        o.length = 0.0;
        s.objects = {o};
        rejects(s, "tube without length");
    }
    {
        Setup s = valid();
        spx_object o{};
        o.kind = SPX_OBJ_DISC;
        o.center[2] = 50.0;
        o.normal[2] = 1.0;
        o.half_u = 1.0;
        s.objects.assign(33, o);
        rejects(s, "too many objects");
    }
    {
        Setup s = valid();
        spx_object o{};
        o.kind = 7;
        o.normal[2] = 1.0;
        o.half_u = 1.0;
        s.objects = {o};
        rejects(s, "unknown object kind");
    }
    { Setup s = valid(); s.prm.theta_min = 0.0; rejects(s, "theta_min"); }
    { Setup s = valid(); s.prm.table_ne = 1; rejects(s, "table size"); }
    { Setup s = valid(); s.prm.log_eps_lo = 0.0; s.prm.log_eps_hi = -1.0; rejects(s, "table range"); }
    { Setup s = valid(); s.prm.E_th_kT = -1.0; rejects(s, "thermalisation threshold"); }
    { Setup s = valid(); s.prm.precision = 16; rejects(s, "precision"); }
    {
        spx_plan* p = nullptr;
        check(spx_plan_create(nullptr, 1, nullptr, &p) == SPX_EINVAL && p == nullptr, "null configurations");
    }

    // host-only entry points
    std::vector<double> e64(SPX_ARRIVAL_E_BINS + 1), c64(SPX_ARRIVAL_A_BINS + 1);
    std::vector<float> e32(SPX_ARRIVAL_E_BINS + 1), c32(SPX_ARRIVAL_A_BINS + 1);
    check(spx_arrival_edges(e64.data(), c64.data(), e32.data(), c32.data()) == SPX_OK, "arrival edges");
    check(spx_arrival_edges(nullptr, nullptr, nullptr, nullptr) == SPX_OK, "arrival edges, no outputs");
    for (int i = 1; i <= SPX_ARRIVAL_E_BINS; ++i) check(e64[i] > e64[i - 1], "energy edges increase");
    std::vector<double> cen(2 * 342);
    check(spx_area_centres(342, 4.5, cen.data()) == SPX_OK, "area centres");
    check(std::fabs(cen[0]) + std::fabs(cen[1]) == 0.0, "first area at the centre");
    check(spx_area_centres(0, 4.5, cen.data()) == SPX_EINVAL, "no areas");
    check(spx_area_centres(342, -1.0, cen.data()) == SPX_EINVAL, "negative pitch");
    check(spx_area_centres(342, 4.5, nullptr) == SPX_EINVAL, "null output");

    // argument checks of device entry points, before any device work
    check(spx_run(nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr) != SPX_OK, "run without a plan");
    check(spx_get_launch(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == SPX_EINVAL, "get_launch null");
    check(spx_autotune(nullptr, nullptr) == SPX_EINVAL, "autotune null");
    spx_outputs out{};
    check(spx_run_noalloc(nullptr, 0, &out, nullptr) == SPX_EINVAL, "noalloc without a plan");

    if (g_fail == 0) std::printf("ok\n");
    return g_fail == 0 ? 0 : 1;
}
