// transport.hip -- the two transport paths and their tally kernels.
//
// Batched FP32 path (k_transport32): one persistent launch covers every
// (configuration, cathode) segment of a plan.  Each lane holds one particle in
// registers; when lanes die the wave claims a run of tickets with a single atomic
// (ballot + mbcnt prefix gives each dead lane its ticket), maps each ticket to
// (segment, particle) through the prefix table, and launches the new particles.
// Every iteration advances each live lane by one flight.  Because the random
// numbers are keyed by (seed, segment, particle, event), the result does not depend
// on which lane or wave ran a particle, nor on the ticket order.  Deposits go to
// the integer tally with 64-bit atomics; per-segment counters are accumulated in
// registers while a lane stays in one segment and flushed when it changes.
//
// Plain FP64 path (k_transport64): one thread per particle runs the whole history;
// one launch per segment.  It is the comparator for the batched path.
#include <hip/hip_runtime.h>

#include "spx_host.hpp"

namespace spx {

__device__ __forceinline__ void add_counters(unsigned long long* C, const uint32_t* acc)
{
#pragma unroll
    for (int i = 0; i < N_COUNTERS; ++i)
        if (acc[i]) atomicAdd(&C[i], (unsigned long long)acc[i]);
}

template <typename R>
__device__ __forceinline__ void write_record(spx_record* rec, const SegDev<R>& s, uint32_t pid, const Particle<R>& p,
                                             const Term& t)
{
    spx_record r;
    r.x = (double)p.x[0] - (double)p.xc[0];
    r.y = (double)p.x[1] - (double)p.xc[1];
    r.z = ((double)p.x[2] - (double)p.xc[2]) + (double)s.z_mid;
    r.E = (double)p.E;
    r.state = (uint32_t)t.state;
    r.bin = t.state == HIT_DEPOSITED ? (uint32_t)t.bin : 0xFFFFFFFFu;
    r.events = p.e;
    r.diffusive = p.ndiff;
    rec[s.first_rec + pid] = r;
}

// Per-lane bookkeeping of the batched kernel: counters of the lane's current segment,
// flushed to the block's LDS counters (or HBM) when the lane moves to another segment.
struct LaneAcc {
    int seg = -1;
    uint32_t c[N_COUNTERS] = {0, 0, 0, 0, 0, 0, 0};
};

struct BlockTally {
    unsigned long long* lcnt;   // LDS per-segment counters (valid if a.lds_counters)
    uint32_t* ltally;           // LDS tally (valid if a.lds_tally)
};

__device__ __forceinline__ void flush_acc(const TransportArgs& a, const BlockTally& bt, LaneAcc& acc)
{
    if (acc.seg < 0) return;
    if (a.lds_counters) {
#pragma unroll
        for (int i = 0; i < N_COUNTERS; ++i)
            if (acc.c[i]) atomicAdd(&bt.lcnt[acc.seg * N_COUNTERS + i], (unsigned long long)acc.c[i]);
    } else {
        add_counters(a.counters + (size_t)acc.seg * N_COUNTERS, acc.c);
    }
#pragma unroll
    for (int i = 0; i < N_COUNTERS; ++i) acc.c[i] = 0;
}

// End of a history: counters, tally, optional record; the lane becomes free.
__device__ __forceinline__ void terminate(const TransportArgs& a, const BlockTally& bt, const SegDev<float>& s,
                                          uint32_t pid, Particle<float>& p, const Term& t, LaneAcc& acc)
{
    // static indices only: the counters stay in registers
    acc.c[C_DEPOSITED] += (t.state == HIT_DEPOSITED) ? 1u : 0u;
    acc.c[C_WALL] += (t.state == HIT_WALL) ? 1u : 0u;
    acc.c[C_ESCAPED] += (t.state == HIT_ESCAPED) ? 1u : 0u;
    acc.c[C_COLLISIONS] += p.ncoll;
    acc.c[C_DIFFUSIVE] += p.ndiff;
    acc.c[C_THERMALIZED] += (p.st == ST_DIFFUSIVE) ? 1u : 0u;
    if (t.state == HIT_DEPOSITED) {
        const uint64_t b = s.bin_off + (uint64_t)t.bin;
        if (a.lds_tally) atomicAdd(&bt.ltally[b], 1u);
        else atomicAdd(&a.counts[b], 1ull);
    }
    if (a.records) write_record(a.records, s, pid, p, t);
    p.st = ST_DEAD;
}

// Flights of the lanes in state MODE while the wave's situation allows: every such lane
// in segment S (uniform, so its constants stay in scalar registers across the loop).
// Leaves when the wave should refill, switch event kind, or has nothing left in MODE.
template <int MODE>
__device__ __forceinline__ void uniform_loop(const TransportArgs& a, const BlockTally& bt, const SegDev<float>& S,
                                             uint32_t pid, Particle<float>& p, LaneAcc& acc, bool drained)
{
    for (;;) {
        if (p.st == MODE) {
            const Term t = (MODE == ST_BALLISTIC) ? step_mode<float, ST_BALLISTIC>(S, a.tab, a.k0, a.k1, pid, a.cap, p)
                                                  : step_diffusive_ball(S, a.k0, a.k1, pid, a.cap, p);
            if (t.state != HIT_NONE) terminate(a, bt, S, pid, p, t, acc);
        }
        const uint64_t M = __ballot(p.st == MODE);
        if (M == 0) break;
        if (!drained && __popcll(__ballot(p.st == ST_DEAD)) >= a.refill_min) break;
        if (drained && __popcll(__ballot(p.st != ST_DEAD)) <= COOP_MAX) break;   // cooperative walks
        if (MODE == ST_BALLISTIC && __popcll(M) < a.ballistic_min && __ballot(p.st == ST_DIFFUSIVE) != 0) break;
    }
}

// Diffusive steps of the lanes in segment S with deferred surface tests: a lane whose
// step leaves its clearance ball holds the step and idles until at least DEFER_MIN lanes
// hold one (or every diffusive lane does, or the loop is about to end); then the held
// steps are tested together, so the long test runs in few iterations.  No step is held
// when the loop returns.
__device__ __forceinline__ void diffusive_loop(const TransportArgs& a, const BlockTally& bt, const SegDev<float>& S,
                                               uint32_t pid, Particle<float>& p, LaneAcc& acc, bool drained)
{
    bool held = false;
    for (;;) {
        if (p.st == ST_DIFFUSIVE && !held) {
            const Term t = diffusive_advance(S, a.k0, a.k1, pid, a.cap, p, held);
            if (t.state != HIT_NONE) terminate(a, bt, S, pid, p, t, acc);
        }
        const uint64_t H = __ballot(held);
        const uint64_t M = __ballot(p.st == ST_DIFFUSIVE);
        bool stop = M == 0 || (!drained && __popcll(__ballot(p.st == ST_DEAD)) >= a.refill_min) ||
                    (drained && __popcll(__ballot(p.st != ST_DEAD)) <= COOP_MAX);
        if (H != 0 && (stop || H == M || __popcll(H) >= DEFER_MIN)) {
            if (held) {
                held = false;
                const Term t = diffusive_resolve(S, p);
                if (t.state != HIT_NONE) terminate(a, bt, S, pid, p, t, acc);
            }
            stop = __ballot(p.st == ST_DIFFUSIVE) == 0 ||
                   (!drained && __popcll(__ballot(p.st == ST_DEAD)) >= a.refill_min) ||
                   (drained && __popcll(__ballot(p.st != ST_DEAD)) <= COOP_MAX);
        }
        if (stop) break;
    }
}

// Dynamic LDS: per-segment counters (u64, when lds_counters) then the tally (u32, when lds_tally).
// At most 96 VGPRs: five waves per SIMD hide the latency of the transcendental and
// integer-multiply chains.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5)))
k_transport32(TransportArgs a, const SegDev<float>* __restrict__ segs)
{
    extern __shared__ unsigned long long lds[];
    BlockTally bt;
    bt.lcnt = lds;
    bt.ltally = (uint32_t*)(lds + (a.lds_counters ? (size_t)a.n_seg * N_COUNTERS : 0));
    if (a.lds_counters)
        for (int i = threadIdx.x; i < a.n_seg * N_COUNTERS; i += blockDim.x) bt.lcnt[i] = 0;
    if (a.lds_tally)
        for (uint32_t i = threadIdx.x; i < a.n_bins; i += blockDim.x) bt.ltally[i] = 0;
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    Particle<float> p;
    p.st = ST_DEAD;
    p.e = p.ndiff = p.ncoll = 0;
    uint32_t pid = 0;
    int seg = 0;
    LaneAcc acc;
    bool drained = false;   // wave-uniform: the ticket space is exhausted
    // Wave-private run of tickets [tk, tk_end), claimed TICKET_CHUNK at a time with one
    // atomic, so that refills rarely touch the global counter.
    uint64_t tk = 0, tk_end = 0;

    for (;;) {
        // refill: dead lanes take consecutive tickets of the wave's run (ballot + mbcnt prefix)
        const uint64_t dead = __ballot(p.st == ST_DEAD);
        const int n_dead = __popcll(dead);
        if (!drained && n_dead > 0 && (n_dead >= a.refill_min || n_dead == 64)) {
            if (tk == tk_end) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd((unsigned long long*)a.ticket, (unsigned long long)TICKET_CHUNK);
                base = __shfl(base, 0);
                if (base >= a.total) {
                    drained = true;
                } else {
                    tk = base;
                    tk_end = (base + TICKET_CHUNK < a.total) ? base + TICKET_CHUNK : a.total;
                }
            }
            const uint64_t avail = tk_end - tk;
            const uint64_t take = avail < (uint64_t)n_dead ? avail : (uint64_t)n_dead;
            const uint64_t base = tk;
            tk += take;
            if (p.st == ST_DEAD) {
                const uint64_t rank = (uint64_t)__popcll(dead & lt_mask);
                const uint64_t my = base + rank;
                if (rank < take) {
                    int lo = 0, hi = a.n_seg;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (a.tfirst[mid] <= my) lo = mid; else hi = mid;
                    }
                    const int sg = (int)a.torder[lo];
                    pid = (uint32_t)(my - a.tfirst[lo]);
                    if (sg != acc.seg) {
                        flush_acc(a, bt, acc);
                        acc.seg = sg;
                    }
                    seg = sg;
                    start(segs[seg], a.k0, a.k1, pid, p);
                    acc.c[C_LAUNCHED] += 1;
                }
            }
        }
        const uint64_t B = __ballot(p.st == ST_BALLISTIC);
        const uint64_t D = __ballot(p.st == ST_DIFFUSIVE);
        if ((B | D) == 0) {
            if (drained) break;
            continue;
        }
        // Last histories of a drained wave: each thermalised lane is walked by the whole
        // wave (up to 64 steps per pass) before the regular step below.
        if (drained && __popcll(B | D) <= COOP_MAX) {
            for (uint64_t W = D; W != 0; W &= W - 1) {
                const int L = __ffsll((unsigned long long)W) - 1;
                coop_walk(segs[__builtin_amdgcn_readlane(seg, L)], a.k0, a.k1, a.cap, pid, p, L, lane);
            }
        }
        // One kind of event at a time: ballistic flights only once enough lanes are
        // ballistic (or nothing else is left), so that rare ballistic lanes do not drag the
        // long collision path into most iterations of a thermalised wave.
        const int mode = (B != 0 && (__popcll(B) >= a.ballistic_min || D == 0)) ? ST_BALLISTIC : ST_DIFFUSIVE;
        const uint64_t Mm = (mode == ST_BALLISTIC) ? B : D;
        const int s0 = __builtin_amdgcn_readlane(seg, __ffsll((unsigned long long)Mm) - 1);
        if (__ballot(p.st == mode && seg != s0) == 0) {
            const SegDev<float>& S = segs[s0];
            if (mode == ST_BALLISTIC) uniform_loop<ST_BALLISTIC>(a, bt, S, pid, p, acc, drained);
            else diffusive_loop(a, bt, S, pid, p, acc, drained);
        } else if (p.st == mode) {
            // lanes of several segments: one flight with per-lane constants
            const SegDev<float>& s = segs[seg];
            const Term t = (mode == ST_BALLISTIC) ? step_mode<float, ST_BALLISTIC>(s, a.tab, a.k0, a.k1, pid, a.cap, p)
                                                  : step_diffusive_ball(s, a.k0, a.k1, pid, a.cap, p);
            if (t.state != HIT_NONE) terminate(a, bt, s, pid, p, t, acc);
        }
    }
    flush_acc(a, bt, acc);
    __syncthreads();
    if (a.lds_counters)
        for (int i = threadIdx.x; i < a.n_seg * N_COUNTERS; i += blockDim.x)
            if (bt.lcnt[i]) atomicAdd(&a.counters[i], bt.lcnt[i]);
    if (a.lds_tally)
        for (uint32_t i = threadIdx.x; i < a.n_bins; i += blockDim.x)
            if (bt.ltally[i]) atomicAdd(&a.counts[i], (unsigned long long)bt.ltally[i]);
}

__global__ void __launch_bounds__(256) k_transport64(const SegDev<double>* __restrict__ segp, TabDev<double> tab,
                                                     uint32_t k0, uint32_t k1, uint32_t cap,
                                                     unsigned long long* __restrict__ counts,
                                                     unsigned long long* __restrict__ counters,
                                                     spx_record* __restrict__ records)
{
    const SegDev<double>& s = *segp;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc[N_COUNTERS] = {0, 0, 0, 0, 0, 0, 0};
    if (i < s.N) {
        const uint32_t pid = (uint32_t)i;
        Particle<double> p;
        start(s, k0, k1, pid, p);
        Term t;
        do {
            t = step(s, tab, k0, k1, pid, cap, p);
        } while (t.state == HIT_NONE);
        acc[C_LAUNCHED] = 1;
        acc[t.state == HIT_DEPOSITED ? C_DEPOSITED : (t.state == HIT_WALL ? C_WALL : C_ESCAPED)] = 1;
        acc[C_COLLISIONS] = p.ncoll;
        acc[C_DIFFUSIVE] = p.ndiff;
        acc[C_THERMALIZED] = (p.st == ST_DIFFUSIVE) ? 1u : 0u;
        if (t.state == HIT_DEPOSITED) atomicAdd(&counts[s.bin_off + (uint64_t)t.bin], 1ull);
        if (records) write_record(records, s, pid, p, t);
    }
    // wave sum of the counters, one atomic per counter and wave
#pragma unroll
    for (int c = 0; c < N_COUNTERS; ++c) {
        unsigned long long v = acc[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(&counters[c], v);
    }
}

// Zero the outputs and the ticket counter (a kernel, so that it can sit in a graph).
__global__ void k_zero(unsigned long long* counts, uint64_t n_counts, unsigned long long* counters, uint64_t n_counters,
                       uint64_t* ticket)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_counts; i += stride) counts[i] = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_counters; i += stride) counters[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && ticket) *ticket = 0;
}

// profiles = counts / (N_seg * bin area); FP64.
__global__ void k_normalize(const unsigned long long* __restrict__ counts, const uint64_t* __restrict__ bin_off,
                            const double* __restrict__ seg_norm, int n_seg, uint64_t n_bins,
                            double* __restrict__ profiles)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_bins; b += stride) {
        int lo = 0, hi = n_seg;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bin_off[mid] <= b) lo = mid; else hi = mid;
        }
        profiles[b] = (double)counts[b] * seg_norm[lo];
    }
}

static int launch_zero_and_tail(Plan* P, uint64_t* d_counts, uint64_t* d_counters, uint64_t* ticket, hipStream_t st)
{
    const uint64_t n = P->n_bins_total;
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 + 1 : 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, (unsigned long long*)d_counts, n,
                       (unsigned long long*)d_counters, (uint64_t)P->n_seg * N_COUNTERS, ticket);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

static int launch_normalize(Plan* P, const uint64_t* d_counts, double* d_profiles, hipStream_t st)
{
    const uint64_t n = P->n_bins_total;
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 + 1 : 4096);
    hipLaunchKernelGGL(k_normalize, dim3(blocks), dim3(256), 0, st, (const unsigned long long*)d_counts,
                       P->d_bin_off, P->d_seg_norm, P->n_seg, n, d_profiles);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// Dynamic LDS of the FP32 transport for a plan: counters if they fit, tally if it fits.
size_t transport32_lds(const Plan* P, bool* lds_counters, bool* lds_tally)
{
    const size_t cbytes = (size_t)P->n_seg * N_COUNTERS * sizeof(unsigned long long);
    const size_t tbytes = (size_t)P->n_bins_total * sizeof(uint32_t);
    *lds_counters = cbytes <= LDS_COUNTERS_MAX;
    *lds_tally = tbytes <= LDS_TALLY_MAX;
    return (*lds_counters ? cbytes : 0) + (*lds_tally ? tbytes : 0);
}

int occupancy_transport32(const Plan* P, int threads, int* blocks_per_cu)
{
    bool lc, lt;
    const size_t smem = transport32_lds(P, &lc, &lt);
    SPX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_transport32, threads, smem));
    return SPX_OK;
}

int launch_transport32(Plan* P, uint64_t seed, uint64_t* d_counts, uint64_t* d_counters, double* d_profiles,
                       spx_record* d_records, hipStream_t st, const uint64_t* tfirst, uint64_t total, int blocks,
                       int threads, int refill_min, int ballistic_min)
{
    SPX_TRY(launch_zero_and_tail(P, d_counts, d_counters, P->d_ticket, st));
    TransportArgs a;
    a.segs = P->d_seg32;
    a.tab.theta = P->d_theta32;
    a.tab.betamax = P->d_betamax32;
    a.tab.ne = P->params.table_ne;
    a.tab.ns = P->params.table_ns;
    a.tab.xs = (float)((P->params.table_ne - 1) / ((P->params.log_eps_hi - P->params.log_eps_lo) * 3.321928094887362));
    a.tfirst = tfirst;
    a.torder = P->d_torder;
    a.ticket = P->d_ticket;
    a.counts = (unsigned long long*)d_counts;
    a.counters = (unsigned long long*)d_counters;
    a.records = d_records;
    a.total = total;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.cap = P->params.event_cap;
    a.n_seg = P->n_seg;
    a.refill_min = refill_min;
    a.ballistic_min = ballistic_min;
    a.n_bins = (uint32_t)P->n_bins_total;
    bool lc, lt;
    const size_t smem = transport32_lds(P, &lc, &lt);
    a.lds_counters = lc ? 1 : 0;
    a.lds_tally = lt ? 1 : 0;
    hipLaunchKernelGGL(k_transport32, dim3(blocks), dim3(threads), smem, st, a,
                       (const SegDev<float>*)P->d_seg32);
    SPX_HIP(hipGetLastError());
    if (d_profiles) SPX_TRY(launch_normalize(P, d_counts, d_profiles, st));
    return SPX_OK;
}

int launch_transport64(Plan* P, uint64_t seed, uint64_t* d_counts, uint64_t* d_counters, double* d_profiles,
                       spx_record* d_records, hipStream_t st)
{
    SPX_TRY(launch_zero_and_tail(P, d_counts, d_counters, nullptr, st));
    TabDev<double> tab;
    tab.theta = P->d_theta64;
    tab.betamax = P->d_betamax64;
    tab.ne = P->params.table_ne;
    tab.ns = P->params.table_ns;
    tab.xs = (P->params.table_ne - 1) / ((P->params.log_eps_hi - P->params.log_eps_lo) * 3.321928094887362);
    for (int k = 0; k < P->n_seg; ++k) {
        const uint64_t N = P->seg[k].N;
        if (N == 0) continue;
        const uint64_t blocks = (N + 255) / 256;
        hipLaunchKernelGGL(k_transport64, dim3((unsigned)blocks), dim3(256), 0, st, P->d_seg64 + k, tab,
                           (uint32_t)seed, (uint32_t)(seed >> 32), P->params.event_cap,
                           (unsigned long long*)d_counts, (unsigned long long*)(d_counters + (size_t)k * N_COUNTERS),
                           d_records);
        SPX_HIP(hipGetLastError());
    }
    if (d_profiles) SPX_TRY(launch_normalize(P, d_counts, d_profiles, st));
    return SPX_OK;
}

}  // namespace spx
