// spx_host.hpp -- host-side plan object and error plumbing of libspx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/spx.h"
#include "spx_device.hpp"

namespace spx {

void set_error(const std::string& msg);

#define SPX_HIP(call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) {                                                                         \
            ::spx::set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " + __FILE__ + ":" + \
                             std::to_string(__LINE__));                                                 \
            return SPX_EDEVICE;                                                                         \
        }                                                                                               \
    } while (0)

#define SPX_TRY(call)                          \
    do {                                       \
        int r_ = (call);                       \
        if (r_ != SPX_OK) return r_;           \
    } while (0)

// FP64 constants of one (config, cathode) segment, in the chamber frame.
struct SegHost {
    int cfg, cath;
    double cat_c[3], cat_n[3], cat_u[3], cat_v[3], cat_R;
    double sub_c[3], sub_n[3], sub_u[3], sub_v[3], half_u, half_v, du, dv;
    int shape, nu, nv;
    double ch_R, zlo, zhi, z_mid;
    double rt_mu, rt_sig, PhiA, QB, dPhi;
    double Us, Emax, smax, Lambda;
    double Ms, Mg, mu_red, a_mm, eps_per_eV;
    double n_mm3, kT, vth, vg, E_th, lam_th;
    int gas_motion;
    double pressure;
    std::vector<double> rt_r, rt_d;   // measured racetrack nodes (empty: truncated normal)
    std::vector<spx_object> objs;     // absorbing objects of the run (chamber frame)
    double cosc[6];                   // emission law coefficients
    uint64_t N, bin_off, first_rec;
    double cost;          // relative expected work per particle (ticket ordering)
};

// A thermalised atom handed from the ballistic to the diffusive phase (48 B).
struct alignas(16) ThermRec {
    float x[3], xc[3];          // compensated position (chamber frame)
    float E;                    // energy at thermalisation (reported in the record)
    uint32_t pid;               // particle index within its segment
    uint32_t seg;               // segment
    uint32_t e;                 // events taken so far
    uint32_t lam_bits;          // the segment's lam_th ln 2 (float bits) and Philox counter word: the
    uint32_t cfgcat;            // two numbers of the segment a diffusive step needs
};
static_assert(sizeof(ThermRec) == 48, "ThermRec layout");

// Launch arguments of the two batched FP32 transport kernels (one round = one chunk of the
// ticket space: the ballistic phase of every ticket, then the diffusive phase of the atoms
// it thermalised).
struct TransportArgs {
    const SegDev<float>* segs;
    TabDev<float> tab;
    const uint64_t* tfirst;     // [n_seg + 1] first ticket of each position in ticket order
    const uint32_t* torder;     // [n_seg] segment at each position
    ThermRec* queue;            // thermalised atoms of the round (capacity >= tickets of a round)
    uint64_t* qstate;           // [QS_TICKETS] ballistic ticket counter, [QS_QUEUE] queue length,
                                // [QS_DIFFUSIVE] diffusive ticket counter
    unsigned long long* counts;
    unsigned long long* counters;
    spx_record* records;
    unsigned long long* arr_E;  // arrival energy histograms [n_seg][SPX_ARRIVAL_E_BINS] (nullable)
    unsigned long long* arr_A;  // arrival angle histograms [n_seg][SPX_ARRIVAL_A_BINS] (nullable with arr_E)
    unsigned long long* esum;   // per tally bin: arrival energies in units of 2^-24 eV (nullable with arr_E)
    const float* e_edges;       // [SPX_ARRIVAL_E_BINS + 1] energy edges, eV
    const float* c_edges;       // [SPX_ARRIVAL_A_BINS + 1] cos(k deg)
    uint64_t tbase;             // first ticket of the round
    uint64_t total;             // tickets of the round
    uint32_t k0, k1;            // Philox key (seed words)
    uint32_t cap;
    int32_t n_seg;
    int32_t refill_min;         // diffusive phase: refill a wave's dead lanes once at least this many
    int32_t refill_ballistic;   // ballistic phase: the same threshold
    int32_t defer_min;          // diffusive phase: held steps that trigger a wave's surface tests
    uint32_t chunk_ballistic;   // ballistic phase: tickets a wave claims per atomic
    uint32_t n_bins;            // tally bins of the plan
    int32_t lds_counters;       // per-segment counters privatised in LDS
    int32_t lds_tally;          // whole tally privatised in LDS (u32 per bin)
    int32_t lds_arrivals;       // arrival histograms privatised in LDS (u32)
};

// Output buffers of one run (device pointers; all but counts and counters nullable).
struct Outputs {
    uint64_t* counts = nullptr;
    uint64_t* counters = nullptr;
    double* profiles = nullptr;
    spx_record* records = nullptr;
    uint64_t* arr_E = nullptr;
    uint64_t* arr_A = nullptr;
    uint64_t* esum = nullptr;
};

constexpr uint64_t ROUND_MAX = 1ull << 28;   // tickets per round: a 12.9 GB queue of thermalised atoms
constexpr uint64_t QUEUE_CHUNK = 64;         // queue slots a wave reserves per atomic
// exactly one lane per slot: a hand-over of up to 64 atoms continues into at most one fresh
// run, and a wave marks its unused reserved slots one per lane
static_assert(QUEUE_CHUNK == 64, "queue runs hold one slot per lane of a wave");
// The round's three counters (ballistic tickets, queue length, diffusive tickets) sit 256 bytes
// apart: every wave's claims and queue reservations are atomics on them, and on one cache line
// the two kinds of atomics of the ballistic phase would queue behind each other.
constexpr uint64_t QS_TICKETS = 0, QS_QUEUE = 32, QS_DIFFUSIVE = 64, QSTATE_WORDS = 96;
constexpr uint64_t QUEUE_SLACK_WAVES = 8192;  // waves that may leave slots unused (32 per CU, 256 CUs)
constexpr size_t LDS_COUNTERS_MAX = 16384;   // bytes: up to 256 segments
constexpr int RT_MAX_NODES = 256;             // nodes of a measured racetrack profile
constexpr int OBJ_MAX_SEG = 32;               // absorbing objects of one (config, cathode) run
constexpr uint64_t TICKET_CHUNK = 128;       // queued atoms a diffusive wave claims per global atomic
// launch tickets a ballistic wave claims per global atomic, at most: ballistic histories are
// short, so their waves come back for tickets often and small chunks queue them on the one
// counter; the chunk of a round is also kept small enough for every wave to take several
constexpr uint64_t TICKET_CHUNK_BALLISTIC_MAX = 512;
constexpr int DEFER_MIN = 8;                  // default: held diffusive steps that trigger a wave's surface tests
// advances (two diffusive steps each) a wave takes between its checks for held steps, dead
// lanes and the end of the walk; the checks (ballots, branches) then cost little per step
constexpr int ADVANCES_PER_CHECK = 7;
constexpr int COOP_MAX = 8;                   // drained waves with at most this many live lanes walk cooperatively
constexpr size_t LDS_TALLY_MAX = 49152;      // bytes: up to 12288 bins
constexpr size_t LDS_ARRIVALS_MAX = 4096;     // bytes: arrival histograms of up to 6 segments

// One kernel launch of a run with its arguments stored by value.  A run of the batched path
// is a list of these: enqueued on a stream as they are made, or made into the kernel nodes of
// a graph whose arguments can later be replaced in the instantiated graph (a new seed or new
// output buffers then need no new graph).
struct KLaunch {
    const void* func = nullptr;
    dim3 grid{1, 1, 1}, block{1, 1, 1};
    uint32_t smem = 0;
    int phase = 0;              // 1: the ballistic kernel of a round, 2: its diffusive kernel, else 0
    int n_args = 0;
    uint16_t off[8] = {};
    uint16_t last_size = 0;
    alignas(16) unsigned char buf[384] = {};

    template <typename T> void arg(const T& v)
    {
        static_assert(std::is_trivially_copyable<T>::value, "kernel arguments are copied bytewise");
        size_t o = n_args ? (size_t)off[n_args - 1] + last_size : 0;
        o = (o + alignof(T) - 1) / alignof(T) * alignof(T);
        if (n_args >= 8 || o + sizeof(T) > sizeof(buf)) {
            n_args = -1;              // reported by the sinks: never launched
            return;
        }
        std::memcpy(buf + o, &v, sizeof(T));
        off[n_args++] = (uint16_t)o;
        last_size = (uint16_t)sizeof(T);
    }
    // pointers to the stored arguments, as hipLaunchKernel and graph kernel nodes take them
    void pointers(void** p) const
    {
        for (int i = 0; i < n_args; ++i) p[i] = const_cast<unsigned char*>(buf) + off[i];
    }
    // same kernel and launch geometry (the arguments may differ)
    bool same_shape(const KLaunch& o) const
    {
        return func == o.func && grid.x == o.grid.x && block.x == o.block.x && smem == o.smem && phase == o.phase &&
               n_args == o.n_args;
    }
    bool same_args(const KLaunch& o) const { return std::memcmp(buf, o.buf, sizeof(buf)) == 0; }
};

// Receiver of the launches of a run, in order.
struct LaunchSink {
    virtual int put(const KLaunch& k) = 0;
    virtual ~LaunchSink() = default;
};

// Launch geometry and thresholds of the two persistent transport kernels.
struct Shape {
    int blocks = 0, blocks_diff = 0, threads = 256, refill_min = 8, refill_ballistic = 8, defer_min = DEFER_MIN;
};

// Queue of thermalised atoms and ticket counters a run works in: the plan's own allocation, or
// caller-independent static scratch.  Rounds hold at most round_max tickets.
struct QueueMem {
    ThermRec* queue = nullptr;
    uint64_t cap = 0;            // slots
    uint64_t* qstate = nullptr;  // QSTATE_WORDS words: the round's counters
    uint64_t round_max = ROUND_MAX;
};

}  // namespace spx

struct spx_plan {
    int device = 0;
    spx_params params{};
    std::vector<spx::SegHost> seg;
    int n_seg = 0;
    uint64_t n_bins_total = 0, n_particles_total = 0;
    std::vector<uint64_t> h_bin_off, h_first;
    std::vector<double> h_betamax;          // FP64 beta_max table copy (host)
    std::vector<double> seg_norm;           // 1 / (N * bin area) per segment

    hipStream_t work_stream = nullptr;
    double* d_theta64 = nullptr;
    double* d_betamax64 = nullptr;
    float* d_theta32 = nullptr;
    float* d_betamax32 = nullptr;
    spx::SegDev<float>* d_seg32 = nullptr;
    spx::SegDev<double>* d_seg64 = nullptr;
    float* d_edges32 = nullptr;               // arrival bin edges: energy [61] then cos [91]
    double* d_edges64 = nullptr;
    spx::ObjDev<float>* d_obj32 = nullptr;    // absorbing objects of all segments
    spx::ObjDev<double>* d_obj64 = nullptr;
    spx::RtNode<float>* d_rt32 = nullptr;     // measured racetracks of all segments
    spx::RtNode<double>* d_rt64 = nullptr;
    uint64_t* d_tfirst = nullptr;
    uint32_t* d_torder = nullptr;
    spx::ThermRec* d_queue = nullptr;       // thermalised atoms of a round (FP32 plans)
    uint64_t queue_cap = 0;
    uint64_t* d_qstate = nullptr;           // ticket counters and queue length
    std::vector<hipEvent_t> phase_events;   // recorded in the graph: round start, ballistic end, diffusive end
    uint64_t* d_bin_off = nullptr;          // [n_seg + 1]
    double* d_seg_norm = nullptr;           // [n_seg]
    uint64_t n_tickets = 0;

    int blocks = 0, threads = 256, refill_min = 8, refill_ballistic = 8, defer_min = spx::DEFER_MIN;
    int blocks_diff = 0;                    // grid of the diffusive kernel: blocks, capped at its resident limit
    int max_blocks_per_cu = 0, n_cu = 0;

    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<spx::KLaunch> graph_launches;   // the kernel nodes' launches, in graph order
    std::vector<hipGraphNode_t> graph_nodes;     // ... and their nodes
    uint64_t graph_instantiations = 0;           // graphs built and instantiated
    uint64_t graph_updates = 0;                  // kernel nodes whose arguments were replaced
    // stream order between runs on different streams: recorded after each run, waited for by
    // the next run or autotune (all of them share the plan's queue and ticket counters)
    hipEvent_t done_event = nullptr;
    bool done_recorded = false;
};

namespace spx {
using Plan = spx_plan;
int build_tables(Plan* P);
// events (nullable, not while capturing): 3 per round, recorded at the round's start, after
// its ballistic phase and after its diffusive phase.
// The launches of one batched FP32 run over tickets [0, total) of `tfirst` in rounds of at most
// q.round_max tickets: zero the outputs, per round reset / ballistic / diffusive, normalise.
int build_transport32(Plan* P, uint64_t seed, const Outputs& o, const uint64_t* tfirst, uint64_t total,
                      const Shape& sh, const QueueMem& q, LaunchSink& sink);
// A sink that launches on `st`; with `events` (3 per round, not while capturing) it records one
// before each ballistic kernel, one after it and one after the diffusive kernel.
struct StreamSink : LaunchSink {
    hipStream_t st;
    const hipEvent_t* events;
    size_t round = 0;
    StreamSink(hipStream_t s, const hipEvent_t* e) : st(s), events(e) {}
    int put(const KLaunch& k) override;
};
uint64_t rounds_of(uint64_t total, uint64_t round_max = ROUND_MAX);
// The plan's current launch geometry and thresholds.
Shape plan_shape(const Plan* P);
int launch_transport64(Plan* P, uint64_t seed, const Outputs& o, hipStream_t st);
// Arrival bin edges in double (as the comparator uses them); the batched path rounds them to float.
void arrival_edges(double* e_edges, double* c_edges);
// resident blocks per CU of the ballistic and of the diffusive kernel at this block size
int occupancy_transport32(const Plan* P, int threads, int* bpc_ballistic, int* bpc_diffusive);
}  // namespace spx
