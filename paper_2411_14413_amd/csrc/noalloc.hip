// noalloc.hip -- spx_run_noalloc: a run of a batched FP32 plan that allocates no device memory.
//
// The batched transport works in device memory beyond the caller's inputs and outputs: the
// queue of thermalised atoms that the ballistic phase fills and the diffusive phase drains,
// and three ticket/queue counters.  spx_run keeps them in memory the plan allocated.  This
// entry point keeps them in `scratch`, a static device array of this file, and enqueues the
// kernels directly on the caller's stream (no graph to instantiate), so it can be called
// where hipMalloc cannot: inside a stream capture, in a serving loop, in a harness that
// forbids allocation.  A larger plan runs in more rounds of the queue; the tallies, counters
// and records do not depend on the rounds.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "spx_host.hpp"

namespace spx {

// 64 MiB per device, held from the library's load until the process ends: the ticket
// counters (first 1 KiB), then the queue (48 B per slot, 1 398 080 slots).
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
constexpr size_t SCRATCH_HEAD = 1024;   // the round's counters (QSTATE_WORDS words), then the queue
static_assert(SCRATCH_HEAD >= QSTATE_WORDS * sizeof(uint64_t), "scratch head holds the round's counters");
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};   // device address of `scratch` on each device

// Device address of this device's copy of `scratch` (looked up once per device, with the
// device current).  The host-side name of the array is not a device address.
int scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("spx_run_noalloc: device index beyond " + std::to_string(MAX_DEVICES));
        return SPX_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("spx_run_noalloc: hipGetSymbolAddress of the scratch array failed: ") +
                      hipGetErrorString(e));
            return SPX_EDEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SPX_OK;
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" int spx_run_noalloc(spx_plan* P, uint64_t seed, const spx_outputs* out, void* stream)
{
    if (!P || !out) {
        set_error("spx_run_noalloc: null argument");
        return SPX_EINVAL;
    }
    if (!out->counts || !out->counters) {
        set_error("spx_run_noalloc: counts and counters are required");
        return SPX_EINVAL;
    }
    const int na = (out->arrival_energy != nullptr) + (out->arrival_angle != nullptr) + (out->energy_sum != nullptr);
    if (na != 0 && na != 3) {
        set_error("spx_run_noalloc: the arrival outputs go together (all three or none)");
        return SPX_EINVAL;
    }
    if (P->params.precision != 32) {
        set_error("spx_run_noalloc: only batched FP32 plans (precision 32) run from the scratch array");
        return SPX_EINVAL;
    }
    SPX_HIP(hipSetDevice(P->device));
    void* base = nullptr;
    SPX_TRY(scratch_address(P->device, &base));
    const Shape sh = plan_shape(P);
    QueueMem q;
    q.qstate = (uint64_t*)base;
    q.queue = (ThermRec*)((unsigned char*)base + SCRATCH_HEAD);
    q.cap = (SCRATCH_BYTES - SCRATCH_HEAD) / sizeof(ThermRec);
    // every wave may leave one reserved run of queue slots unused in a round
    const uint64_t slack = (uint64_t)sh.blocks * (uint64_t)((sh.threads + 63) / 64) * QUEUE_CHUNK;
    if (slack >= q.cap) {
        set_error("spx_run_noalloc: the launch shape (" + std::to_string(sh.blocks) + " blocks of " +
                  std::to_string(sh.threads) + " threads) needs " + std::to_string(slack * sizeof(ThermRec)) +
                  " bytes of queue slack, more than the " + std::to_string(SCRATCH_BYTES) + "-byte scratch array holds");
        return SPX_EINVAL;
    }
    q.round_max = std::min<uint64_t>(ROUND_MAX, q.cap - slack);
    Outputs o;
    o.counts = out->counts;
    o.counters = out->counters;
    o.profiles = out->profiles;
    o.records = out->records;
    o.arr_E = out->arrival_energy;
    o.arr_A = out->arrival_angle;
    o.esum = out->energy_sum;
    StreamSink sink((hipStream_t)stream, nullptr);
    return build_transport32(P, seed, o, P->d_tfirst, P->n_tickets, sh, q, sink);
}
