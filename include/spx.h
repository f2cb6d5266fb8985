/*
 * spx.h -- C-ABI of libspx: Monte Carlo transport of sputtered atoms on MI355X (gfx950).
 *
 * The method is the one of Thelen et al., "A Python-Based Approach to Sputter
 * Deposition Simulations in Combinatorial Materials Science" (arXiv 2411.14413):
 * Methods, "The SIMTRA model" (launch from the racetrack with a Thompson energy
 * and a cosine emission law, exponential free flights, surface intersection and
 * deposition on collecting "dummy" objects, elastic collisions with the gas), the
 * calculation paragraph that closes Methods (Moliere-screened Coulomb potential,
 * gas motion, diffusion of thermalised atoms, arrival fractions converted to at.%
 * with sputter rates, bulk densities and atomic masses), and the Euclidean
 * distance d_e of compositions (Results).  A multi-cathode system is split into
 * independent single-cathode runs, one per (configuration, cathode) "segment"
 * (Methods, "The SIMTRA Python wrapper"); all segments of a plan run in one launch.
 *
 * Conventions
 *   Units: mm, eV, u (atomic mass unit), K, Pa.  Host structs are double precision.
 *   Pointers named d_* are device pointers (HBM of the current HIP device); h_* are
 *   host pointers.  The caller owns every buffer it passes; the library owns the
 *   plan and what the plan allocates.  `stream` is a hipStream_t (NULL = default).
 *   Every function returns SPX_OK (0) or a negative SPX_E* code; on error the
 *   outputs are unspecified and spx_last_error() describes the failure.  No C++
 *   exception crosses this boundary.  Work is enqueued on `stream`; device-side
 *   faults surface at the next synchronising call.  A plan is not thread-safe: call
 *   it from one host thread at a time.  Runs of one plan share its queue of
 *   thermalised atoms and its ticket counters, so each spx_run / spx_run_ex and
 *   spx_autotune first makes its stream wait for the plan's previous run (an event
 *   recorded after every run); runs on different streams are therefore executed one
 *   after the other.  Inside a stream capture spx_run / spx_run_ex enqueue their
 *   kernels directly on the capturing stream (they become nodes of the caller's graph;
 *   the plan's own graph is not used), the wait and the record are left out, and the
 *   capturing caller orders the runs of a plan itself: they share its queue.
 *
 * Random numbers: Philox4x32-10, counter (particle, event, (config << 8) | cathode,
 * sub-block), key (seed low word, seed high word); a 32-bit word x gives
 * u = ((x >> 8) + 1) * 2^-24 in ]0,1] (the paper's RN_1 range).  Results are a
 * function of (configs, params, seed) only: integer tallies are bit-identical
 * whatever the launch shape.
 */
#ifndef SPX_H
#define SPX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPX_OK 0
#define SPX_EINVAL (-1)   /* invalid argument or configuration */
#define SPX_ENOMEM (-2)   /* device or host allocation failed */
#define SPX_EDEVICE (-3)  /* HIP runtime error, or no usable gfx950 device */
#define SPX_ESTATE (-4)   /* call not valid in the plan's current state */

/* Terminal states of a particle (spx_record.state). */
#define SPX_DEPOSITED 1   /* front face of the substrate, inside the plate: tallied */
#define SPX_WALL 2        /* chamber, cathode disc, or substrate back face */
#define SPX_ESCAPED 3     /* event cap reached or non-finite state */

/* Counters per segment, in this order (spx_run d_counters[seg * SPX_N_COUNTERS + i]). */
#define SPX_C_LAUNCHED 0
#define SPX_C_DEPOSITED 1
#define SPX_C_WALL 2
#define SPX_C_ESCAPED 3
#define SPX_C_COLLISIONS 4      /* ballistic flights that ended in a gas collision */
#define SPX_C_DIFFUSIVE 5       /* diffusive steps that ended in the gas */
#define SPX_C_THERMALIZED 6     /* particles that reached the diffusive (thermalised) state */
#define SPX_C_TESTED 7          /* diffusive steps tested against the surfaces: a work counter, not a
                                   result (the batched FP32 walk tests only the steps that leave their
                                   clearance balls; the plain FP64 path tests every step) */
#define SPX_N_COUNTERS 8

/* Magnetron cathode: planar circular target (Methods, "The SIMTRA Python wrapper": the
 * magnetron object holds the element, the racetrack and the geometry). */
typedef struct spx_cathode {
    double center[3];      /* target centre, mm */
    double normal[3];      /* unit normal pointing into the gas */
    double u_axis[3];      /* unit in-plane axis; v = normal x u_axis */
    double radius;         /* target radius, mm; the disc absorbs on both faces */
    double rt_mu, rt_sigma;/* racetrack (rt_n == 0): start radius ~ normal(rt_mu, rt_sigma) ... */
    double rt_lo, rt_hi;   /* ... truncated to [rt_lo, rt_hi], azimuth uniform */
    double U_s;            /* surface binding energy, eV (Thompson distribution) */
    double E_i;            /* incident ion energy, eV */
    double k_cut;          /* E_max = k_cut * Lambda * E_i - U_s, Lambda = 4 M_i M_t/(M_i+M_t)^2,
                              M_i = gas mass (the working-gas ion) */
    double mass;           /* sputtered atom mass, u */
    int32_t Z;             /* sputtered atom number */
    int32_t rt_n;          /* 0: racetrack from rt_mu .. rt_hi; 2 .. 256: nodes of rt_profile */
    double cos_coeff[6];   /* nascent angular law d2Y/dOmega = sum_i c_i cos^i(theta) (Methods, "The
                              SIMTRA model"); must be >= 0 for theta in [0, 90 deg] with
                              sum c_i/(i+1) > 0; {0,1,0,0,0,0} is the cosine law */
    uint64_t n_particles;  /* particles launched from this cathode, < 2^32 */
    const double* rt_profile; /* measured racetrack (Methods, "The SIMTRA model" and "Racetrack
                              measurement"): host array [rt_n][2] of (radius mm, erosion depth >= 0),
                              radii strictly increasing, first >= 0, last <= radius, positive weight;
                              depth linear between nodes, start radius with density depth(r) r,
                              azimuth uniform.  Deep-copied; NULL when rt_n == 0 */
} spx_cathode;

/* Vacuum chamber: absorbing cylinder on the z axis with a homogeneous gas in thermal
 * equilibrium (Methods, "The SIMTRA model"). */
typedef struct spx_chamber {
    double radius, z_lo, z_hi;   /* mm */
    double pressure;             /* Pa; 0 = vacuum (straight flights) */
    double T;                    /* K */
    double gas_mass;             /* u */
    int32_t gas_Z;
    int32_t gas_motion;          /* 1: thermal velocity of the collision partner is sampled */
} spx_chamber;

/* Collecting substrate ("dummy" object) carrying the tally grid. */
typedef struct spx_grid {
    double center[3];
    double normal[3];            /* faces the cathodes; hits from the other side are WALL */
    double u_axis[3];            /* v = normal x u_axis */
    double half_u, half_v;       /* rectangle half-sizes, mm; disc radius = half_u */
    int32_t shape;               /* 0 rectangle, 1 disc (then half_v == half_u) */
    int32_t nu, nv;              /* bins, row-major [iv][iu]; nu * nv <= 2^24 */
    int32_t reserved0;
} spx_grid;

/* An absorbing "dummy" object (Methods, "The SIMTRA model": masks, shutters, chimneys
 * collect the atoms that reach them); both faces absorb (the atom ends as SPX_WALL). */
#define SPX_OBJ_DISC 0   /* disc: centre, unit normal, radius = half_u */
#define SPX_OBJ_RECT 1   /* rectangle: centre, unit normal, unit u_axis, half sizes half_u x half_v */
#define SPX_OBJ_TUBE 2   /* open cylinder (chimney): axis from centre along the unit normal,
                            radius = half_u, length; no end caps */
typedef struct spx_object {
    int32_t kind;
    int32_t reserved0;
    double center[3];
    double normal[3];
    double u_axis[3];            /* rectangles only (v = normal x u_axis) */
    double half_u, half_v;       /* mm */
    double length;               /* tubes, mm */
} spx_object;

typedef struct spx_config {
    spx_chamber chamber;
    spx_grid grid;
    int32_t n_cathodes;          /* 1 .. 255 */
    int32_t cross_absorb;        /* 1: the other targets of this configuration absorb (lifts the
                                    no-cross-deposition assumption of split single-cathode runs,
                                    "The SIMTRA Python wrapper"); 0: each run holds its own target only */
    const spx_cathode* cathodes; /* host array of n_cathodes; deep-copied by spx_plan_create */
    int32_t n_objects;           /* absorbing objects of this configuration; with cross_absorb,
                                    n_objects + n_cathodes - 1 <= 32 */
    int32_t reserved1;
    const spx_object* objects;   /* host array of n_objects (deep-copied; NULL if none) */
} spx_config;

typedef struct spx_params {
    double theta_min;            /* rad; CM deflection at the cross-section cut-off (0.1) */
    double E_th_kT;              /* thermalisation threshold in units of k_B T (3) */
    uint32_t event_cap;          /* flights per particle before ESCAPED (2^20) */
    int32_t table_ne, table_ns;  /* scattering-table nodes in log10(eps) and b/b_max (256, 257) */
    int32_t precision;           /* 32: batched FP32 transport; 64: plain FP64 per-segment comparator */
    double log_eps_lo, log_eps_hi; /* table range of log10(eps) (-10, 0) */
} spx_params;

/* Per-particle terminal record (optional output of spx_run), segment-major:
 * index = first particle index of the segment + particle index. */
typedef struct spx_record {
    double x, y, z;              /* end point (chamber frame, mm) */
    double E;                    /* energy at the end, eV (last ballistic value if thermalised) */
    uint32_t state;              /* SPX_DEPOSITED / SPX_WALL / SPX_ESCAPED */
    uint32_t bin;                /* iv * nu + iu if DEPOSITED, else 0xFFFFFFFF */
    uint32_t events;             /* flights taken */
    uint32_t diffusive;          /* diffusive steps that ended in the gas */
    double cos_in;               /* DEPOSITED: cosine of the incidence angle from the substrate
                                    normal (-d . normal, in (0, 1]); else 0 */
} spx_record;

/* Arrival tallies of the atoms deposited on the substrate (Introduction: a Monte Carlo model
 * yields the energy and angular distributions of arriving particles besides the profile).
 * Energy bin = number of k in 1..59 with E >= 10^(-3 + k/10) eV (so 60 bins, ends open);
 * angle bin = number of k in 1..89 with cos_in <= cos(k deg) (90 bins of 1 deg of the
 * incidence angle).  A thermalised atom arrives with the energy it had when it thermalised. */
#define SPX_ARRIVAL_E_BINS 60
#define SPX_ARRIVAL_A_BINS 90
#define SPX_ESUM_SCALE 16777216.0   /* energy sums count units of 2^-24 eV: rint(E * 2^24) */

/* Output buffers of spx_run_ex (device pointers, caller-owned, overwritten).  counts and
 * counters are required; the others may be NULL (the three arrival outputs together). */
typedef struct spx_outputs {
    uint64_t* counts;            /* uint64[n_bins_total] deposits per bin */
    uint64_t* counters;          /* uint64[n_segments * SPX_N_COUNTERS] */
    double* profiles;            /* double[n_bins_total] counts / (N_seg * bin area) */
    spx_record* records;         /* spx_record[n_particles_total] */
    uint64_t* arrival_energy;    /* uint64[n_segments][SPX_ARRIVAL_E_BINS] deposits per energy bin */
    uint64_t* arrival_angle;     /* uint64[n_segments][SPX_ARRIVAL_A_BINS] deposits per angle bin */
    uint64_t* energy_sum;        /* uint64[n_bins_total] sum over the bin's deposits of rint(E * 2^24) */
} spx_outputs;

typedef struct spx_plan spx_plan;

/* Validate and deep-copy `n_cfgs` configurations; derive per-segment constants in
 * double precision; build the scattering table with an FP64 kernel on the current
 * device (Moliere potential, Firsov screening length; theta_cm(log10 eps, b/b_max)
 * and b_max(eps) where theta_cm = theta_min), synchronously.  Rejects: pressure < 0,
 * T <= 0, zero cathodes, all cathodes with n_particles == 0, n_particles >= 2^32,
 * a cathode or substrate outside the chamber, nu*nv > 2^24 or < 1, rt_lo >= rt_hi (rt_n == 0),
 * an invalid racetrack profile (rt_n == 1 or > 256, radii not increasing, outside [0, radius],
 * negative depths, zero weight), E_max <= 0, masses <= 0, an emission law negative somewhere on
 * [0, 90 deg] or with zero integral, non-unit or non-orthogonal axes, an object of unknown kind,
 * with non-positive sizes or outside the chamber, more than 32 absorbing objects in one run,
 * more than 2^24 configurations.  Device memory: the tables, the segment constants and, for
 * FP32 plans, a queue of thermalised atoms of 48 B per ticket of a round (the particles run in
 * equal rounds of at most 2^28 tickets, so at most ~12.9 GB); SPX_ENOMEM if an allocation
 * fails.  *out is set only on success. */
int spx_plan_create(const spx_config* h_cfgs, int32_t n_cfgs, const spx_params* h_params, spx_plan** out);

/* Sizes of spx_run's outputs: total tally bins over all segments, counters
 * (n_segments * SPX_N_COUNTERS), total particles, segments.  Any pointer may be NULL. */
int spx_plan_query(const spx_plan* plan, uint64_t* n_bins_total, uint64_t* n_counters,
                   uint64_t* n_particles_total, int32_t* n_segments);

/* Offsets of each segment in the outputs: h_bin_off[seg] (into d_counts/d_profiles)
 * and h_first[seg] (into d_records), arrays of n_segments entries each (nullable). */
int spx_plan_layout(const spx_plan* plan, uint64_t* h_bin_off, uint64_t* h_first);

/* Run every particle of every segment with the given seed.
 *   d_counts    uint64[n_bins_total]  deposits per bin (overwritten)
 *   d_counters  uint64[n_counters]    SPX_C_* per segment (overwritten)
 *   d_profiles  double[n_bins_total]  counts / (N_seg * bin area), mm^-2 per launched atom; nullable
 *   d_records   spx_record[n_particles_total]; nullable
 * precision 32 runs the whole plan as one persistent launch (replayed from a HIP
 * graph built on the first run and updated in place for new seeds and buffers);
 * precision 64 runs one plain FP64 launch per segment.  Asynchronous. */
int spx_run(spx_plan* plan, uint64_t seed, uint64_t* d_counts, uint64_t* d_counters,
            double* d_profiles, spx_record* d_records, void* stream);

/* Graph bookkeeping of an FP32 plan: how many times spx_run / spx_run_ex built and
 * instantiated the plan's graph, and how many kernel nodes of the instantiated graph had their
 * arguments replaced.  The graph is rebuilt only when the launch geometry or the set of
 * non-NULL outputs changes; a new seed or new output buffers replace the arguments of the
 * affected kernel nodes (hipGraphExecKernelNodeSetParams), after the host has waited for the
 * plan's previous run to finish (a run with the same seed and buffers does not wait).  Either
 * pointer may be NULL. */
int spx_graph_info(const spx_plan* plan, uint64_t* instantiations, uint64_t* node_updates);

/* spx_run with the outputs in a struct, including the arrival tallies (Introduction:
 * energy and angular distributions of arriving particles).  Asynchronous on `stream`;
 * SPX_EINVAL for missing required outputs or a partial set of arrival outputs. */
int spx_run_ex(spx_plan* plan, uint64_t seed, const spx_outputs* out, void* stream);

/* spx_run_ex for callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): a batched FP32 plan's run that allocates
 * nothing.  Its kernels keep the queue of thermalised atoms and the ticket counters in a
 * static device array of the library (64 MiB per device, held from the library's load until
 * the process ends) instead of the plan's memory, and are enqueued on `stream` directly (no
 * graph).  Outputs as spx_run_ex (caller-owned, overwritten), bit-identical to its results.
 * The particles run in rounds of at most (64 MiB - 1 KiB) / 48 B - (queue slots the launch
 * shape's waves may leave unused: 64 per wave) tickets, so any plan size runs, in more rounds
 * than spx_run uses.  Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (another stream, another host thread, another plan) race and corrupt each other's
 * results, so order them.  SPX_EINVAL for precision 64 plans, missing outputs, and a launch
 * shape whose unused-slot slack alone exceeds the array; SPX_EDEVICE if the array's device
 * address cannot be found.  No hipMalloc, hipFree or graph instantiation. */
int spx_run_noalloc(spx_plan* plan, uint64_t seed, const spx_outputs* out, void* stream);

/* Bin edges of the arrival tallies as the kernels use them: energy edges [61] (eV) and the
 * cosines of the angle edges [91], in double (plain FP64 path) and float (batched FP32 path;
 * the double values rounded).  Any pointer may be NULL. */
int spx_arrival_edges(double* h_energy_edges, double* h_cos_edges, float* h_energy_edges32, float* h_cos_edges32);

/* Choose launch parameters of the FP32 transport by timing short runs on `stream` (a sample
 * with the plan's mix, its outputs in scratch memory the call allocates and frees): per block
 * size, the ballistic refill threshold by the ballistic kernel's time and the diffusive one by
 * the diffusive kernel's, then the deferral threshold by the diffusive kernel's time.
 * Synchronous; not allowed inside a stream capture (SPX_ESTATE); results are unaffected. */
int spx_autotune(spx_plan* plan, void* stream);

/* Current FP32-transport launch parameters of its two persistent kernels (the ballistic
 * phase, launch to thermalisation, and the diffusive phase): blocks (the ballistic grid; the
 * diffusive kernel runs the smaller of it and its own resident limit), threads per block
 * (both), the diffusive phase's refill threshold (a wave refills its dead lanes once at least
 * this many are dead), the ballistic phase's, and the diffusive phase's deferral threshold (a
 * wave tests the steps that left their clearance balls once at least this many lanes hold
 * one; default 8).  Any pointer may be NULL. */
int spx_get_launch(const spx_plan* plan, int32_t* blocks, int32_t* threads, int32_t* refill_min,
                   int32_t* refill_ballistic, int32_t* defer_min);
/* Override them: threads a multiple of 64 in [64, 1024], thresholds in [1, 64]; blocks <= 0
 * (or above the ballistic kernel's resident limit) fills the device at that limit. */
int spx_set_launch(spx_plan* plan, int32_t blocks, int32_t threads, int32_t refill_min, int32_t refill_ballistic,
                   int32_t defer_min);

/* Device time [ms] of the two phases of the last FP32 spx_run of this plan, summed over its
 * rounds (HIP events recorded between the kernels; waits for that run to finish).
 * SPX_ESTATE before the first FP32 run. */
int spx_phase_times(spx_plan* plan, float* ms_ballistic, float* ms_diffusive);

/* Copy the FP64 scattering table to the host: h_theta[ne * ns] (row i = log10 eps node),
 * h_betamax[ne]. */
int spx_get_table(const spx_plan* plan, double* h_theta, double* h_betamax);

/* Derived FP64 constants of one segment (host copy), 16 doubles:
 * Lambda, E_max, s_max, a_mm, eps_per_eV, n_mm3, kT, E_th, lam_th, PhiA, QB, dPhi,
 * mu_red, vth, vg, z_mid. */
int spx_segment_info(const spx_plan* plan, int32_t seg, double* h_out16);

/* Philox4x32-10 blocks on the device: d_out[4i..4i+3] = philox(d_ctr[4i..4i+3], key). */
int spx_philox(const uint32_t* d_ctr, uint32_t key_lo, uint32_t key_hi, uint32_t* d_out, uint64_t n,
               void* stream);

/* Measurement-area centres (host): lattice points (pitch*i, pitch*j) closest to the
 * substrate centre, ties in distance ordered by polar angle in [0, 2 pi); h_out[2*n_areas]. */
int spx_area_centres(int32_t n_areas, double pitch, double* h_out);

/* Area average of n_prof profiles on one grid: d_out[p * n_areas + a] = mean of the
 * profile over the square of half-width `half_width` around centre a, each bin
 * weighted by its overlap with the square.  d_profiles double[n_prof * nv * nu],
 * d_centres double[2 * n_areas] (u, v in the grid frame). */
int spx_area_gather(const double* d_profiles, int32_t n_prof, int32_t nu, int32_t nv, double half_u,
                    double half_v, const double* d_centres, int32_t n_areas, double half_width,
                    double* d_out, void* stream);

/* Composition map, FP32 (Methods, conversion of arrival fractions to at.%):
 *   w[b,k]   = (a[k] P[b,k] + bb[k]) rho[k] / (M[k] fref[k])
 *   c[b,j,k] = 100 w[b,k] f[k,j] / sum_l w[b,l] f[l,j]
 * f [K,J] arrival fraction per area, P [B,K], a/bb/M/rho/fref [K], c [B,J,K]; 0 < K <= 16. */
int spx_comp_forward(const float* d_f, const float* d_a, const float* d_b, const float* d_P,
                     const float* d_M, const float* d_rho, const float* d_fref, float* d_c,
                     int32_t B, int32_t J, int32_t K, void* stream);

/* Backward of spx_comp_forward for an upstream gradient d_gc [B,J,K]: gradients of
 * sum(gc * c) with respect to every input (same shapes).  Each output is written
 * (not accumulated); deterministic (no floating-point atomics). */
int spx_comp_backward(const float* d_f, const float* d_a, const float* d_b, const float* d_P,
                      const float* d_M, const float* d_rho, const float* d_fref, const float* d_gc,
                      float* d_gf, float* d_ga, float* d_gb, float* d_gP, float* d_gM, float* d_grho,
                      float* d_gfref, int32_t B, int32_t J, int32_t K, void* stream);

/* Squared Euclidean distance of compositions summed over areas (Results, d_e):
 * d_loss[b] = sum_{j,k} (c[b,j,k] - ct[b or 0,j,k])^2; ct has B_t = 1 or B rows.
 * If d_gc is non-NULL it also receives d loss_total / d c scaled by d_gloss[b]
 * (d_gloss nullable = all ones): gc = 2 (c - ct) gloss[b]. */
int spx_comp_sqdist(const float* d_c, const float* d_ct, int32_t B_t, const float* d_gloss, float* d_loss,
                    float* d_gc, int32_t B, int32_t J, int32_t K, void* stream);

/* ---- Inversion of a geometry parameter over a sweep (Results, the cathode-tilt study and
 * Figure 8: the simulation is repeated over a range of cathode tilts and each simulated library
 * is compared with the measured one by the compositional area it covers and by d_e). ---- */

/* Compositions of the T libraries of a sweep, all made with the same powers, each normalised
 * by its own calibration value fref[t,k] = mean over j of f[t,k,j] (the default of the
 * composition map):
 *   w[t,k] = (a[k] P[k] + bb[k]) rho[k] / (M[k] fref[t,k]),
 *   c[t,j,k] = 100 w[t,k] f[t,k,j] / sum_l w[t,l] f[t,l,j].
 * d_f double[T][K][J]: the area values of the K segments of each sweep point, as
 * spx_area_gather writes them for T*K profiles of one grid; d_a, d_b, d_P, d_M, d_rho
 * double[K]; d_c float[T][J][K] (written).  Computed in double, stored as float.
 * Rejects T <= 0, J <= 0, K outside 1..16, null pointers (SPX_EINVAL). */
int spx_sweep_composition(const double* d_f, const double* d_a, const double* d_b, const double* d_P,
                          const double* d_M, const double* d_rho, float* d_c, int32_t T, int32_t J, int32_t K,
                          void* stream);

/* Compositional area covered by each of B ternary libraries: the area of the convex hull of
 * its J compositions in the ternary diagram, as a fraction of the whole diagram.  The pure
 * elements 0, 1, 2 sit at (0, 0), (100, 0), (50, 50 sqrt 3), so c (at.%) maps to
 * x = c1 + c2/2, y = c2 sqrt(3)/2.  The hull is Andrew's monotone chain over the points
 * sorted by (x, y), in double precision; a point that does not make a strict left turn is
 * dropped; fewer than three points cover 0.  d_c float[B][J][3], d_area float[B] (written).
 * Rejects B <= 0, J outside 1..2048, null pointers (SPX_EINVAL). */
int spx_hull_area(const float* d_c, int32_t B, int32_t J, float* d_area, void* stream);

#define SPX_FIT_MIN 0    /* the sweep value that minimises the curve */
#define SPX_FIT_MATCH 1  /* the sweep value at which the curve reaches a target */

/* Fit of one parameter over a sweep.  h_x: host double[T], the sweep values, finite and
 * strictly increasing (copied into the launch); d_y float[B][T], one curve per row;
 * d_xfit double[B] (written).
 *   SPX_FIT_MIN:   the vertex of the least-squares parabola through all samples, kept inside
 *                  the sweep, if it opens upwards; otherwise, or with fewer than three
 *                  samples, the sweep value of the smallest sample (the first on ties).
 *   SPX_FIT_MATCH: the sweep value at which the least-squares line through all samples
 *                  reaches d_target[b] (device float[B]); NaN if that lies outside the sweep,
 *                  if the line is flat, or with fewer than two samples.
 * Least squares over the whole sweep average the Monte Carlo noise of the sweep points.
 * Computed in double (sweep values scaled to [-1, 1], curves centred on their mean).  Rejects B <= 0, T outside 1..256, x not strictly increasing, an
 * unknown mode, SPX_FIT_MATCH without targets, null pointers (SPX_EINVAL). */
int spx_sweep_fit(const double* h_x, const float* d_y, int32_t B, int32_t T, int32_t mode, const float* d_target,
                  double* d_xfit, void* stream);

void spx_plan_destroy(spx_plan* plan);

/* Description of the last error on this thread; valid until the next spx_* call on it. */
const char* spx_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int32_t spx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPX_H */
