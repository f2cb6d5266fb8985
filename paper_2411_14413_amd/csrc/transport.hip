// transport.hip -- the two transport paths and their tally kernels.
//
// Batched FP32 path: every (configuration, cathode) segment of a plan runs in rounds of
// at most ROUND_MAX tickets, each round as two persistent launches.  k_ballistic32 takes
// every ticket of the round from its launch through its ballistic flights and collisions;
// an atom that ends on a surface (or escapes) is finished there, an atom that thermalises
// is handed over to a queue in HBM (48 B, with the two numbers of its segment a step needs).  k_diffusive32 then runs the diffusive walks of
// the queued atoms.  Each lane holds one atom in registers; when lanes die, the wave claims
// a run of tickets with a single atomic (ballot + mbcnt prefix gives each dead lane its
// ticket).  Splitting the history at thermalisation keeps every lane of a wave in the same
// kind of event: new atoms (ballistic) and walkers (diffusive) never share a wave.  The
// random numbers are keyed by (seed, segment, particle, event), so the result does not
// depend on which lane, wave or launch ran an atom, nor on the queue order.  Deposits go
// to a per-block LDS tally (or 64-bit global atomics when it does not fit); per-segment
// counters are accumulated in registers while a lane stays in one segment.
//
// Plain FP64 path (k_transport64): one thread per particle runs the whole history;
// one launch per segment.  It is the comparator for the batched path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

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
    r.cos_in = (double)t.cos_in;
    rec[s.first_rec + pid] = r;
}

// Per-lane bookkeeping of the batched kernel: counters of the lane's current segment,
// flushed to the block's LDS counters (or HBM) when the lane moves to another segment.
struct LaneAcc {
    int seg = -1;
    uint32_t c[N_COUNTERS] = {};
};

struct BlockTally {
    unsigned long long* lcnt;   // LDS per-segment counters (valid if a.lds_counters)
    uint32_t* ltally;           // LDS tally (valid if a.lds_tally)
    uint32_t* larr;             // LDS arrival histograms [n_seg][E bins + A bins] (valid if a.lds_arrivals)
};

constexpr int ARR_BINS = SPX_ARRIVAL_E_BINS + SPX_ARRIVAL_A_BINS;

// Arrival tallies of one deposit: energy and angle histograms of its segment, energy sum of
// its tally bin.
__device__ __forceinline__ void tally_arrival(const TransportArgs& a, const BlockTally& bt, int seg, uint64_t bin,
                                              double E, double cos_in)
{
    const int be = energy_bin(a.e_edges, (float)E);
    const int ba = angle_bin(a.c_edges, (float)cos_in);
    if (a.lds_arrivals) {
        atomicAdd(&bt.larr[seg * ARR_BINS + be], 1u);
        atomicAdd(&bt.larr[seg * ARR_BINS + SPX_ARRIVAL_E_BINS + ba], 1u);
    } else {
        atomicAdd(&a.arr_E[(size_t)seg * SPX_ARRIVAL_E_BINS + be], 1ull);
        atomicAdd(&a.arr_A[(size_t)seg * SPX_ARRIVAL_A_BINS + ba], 1ull);
    }
    atomicAdd(&a.esum[bin], energy_units(E));
}

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
template <bool ARR>
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
        if (ARR) tally_arrival(a, bt, acc.seg, b, (double)p.E, (double)t.cos_in);
    }
    if (a.records) write_record(a.records, s, pid, p, t);
    p.st = ST_DEAD;
}

// Number of set bits of the wave-wide mask m in the lanes below this one (mbcnt).
__device__ __forceinline__ uint64_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Wave-private run of tickets [tk, tk_end), claimed CHUNK at a time from a global counter with
// one atomic, so that refills rarely touch the counter.
struct Tickets {
    uint64_t tk = 0, tk_end = 0;
    bool drained = false;     // wave-uniform: the ticket space is exhausted
};

// Tickets for the dead lanes `dead` of the wave: consecutive tickets of the wave's run in lane
// order.  Returns this lane's ticket, or ~0 when it gets none.
__device__ __forceinline__ uint64_t claim(Tickets& T, uint64_t* counter, uint64_t chunk, uint64_t total, uint64_t dead,
                                          int lane)
{
    if (T.tk == T.tk_end) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long*)counter, (unsigned long long)chunk);
        base = __shfl(base, 0);
        if (base >= total) {
            T.drained = true;
            return ~0ull;
        }
        T.tk = base;
        T.tk_end = (base + chunk < total) ? base + chunk : total;
    }
    const uint64_t n_dead = (uint64_t)__popcll(dead);
    const uint64_t avail = T.tk_end - T.tk;
    const uint64_t take = avail < n_dead ? avail : n_dead;
    const uint64_t base = T.tk;
    T.tk += take;
    const uint64_t rank = lanes_below(dead);
    return (((dead >> lane) & 1ull) && rank < take) ? base + rank : ~0ull;
}

__device__ __forceinline__ void lds_setup(const TransportArgs& a, BlockTally& bt, unsigned long long* lds)
{
    bt.lcnt = lds;
    bt.ltally = (uint32_t*)(lds + (a.lds_counters ? (size_t)a.n_seg * N_COUNTERS : 0));
    bt.larr = bt.ltally + (a.lds_tally ? a.n_bins : 0u);
    if (a.lds_counters)
        for (int i = threadIdx.x; i < a.n_seg * N_COUNTERS; i += blockDim.x) bt.lcnt[i] = 0;
    if (a.lds_tally)
        for (uint32_t i = threadIdx.x; i < a.n_bins; i += blockDim.x) bt.ltally[i] = 0;
    if (a.lds_arrivals)
        for (int i = threadIdx.x; i < a.n_seg * ARR_BINS; i += blockDim.x) bt.larr[i] = 0;
    __syncthreads();
}

__device__ __forceinline__ void lds_flush(const TransportArgs& a, const BlockTally& bt, LaneAcc& acc)
{
    flush_acc(a, bt, acc);
    __syncthreads();
    if (a.lds_counters)
        for (int i = threadIdx.x; i < a.n_seg * N_COUNTERS; i += blockDim.x)
            if (bt.lcnt[i]) atomicAdd(&a.counters[i], bt.lcnt[i]);
    if (a.lds_tally)
        for (uint32_t i = threadIdx.x; i < a.n_bins; i += blockDim.x)
            if (bt.ltally[i]) atomicAdd(&a.counts[i], (unsigned long long)bt.ltally[i]);
    if (a.lds_arrivals)
        for (int i = threadIdx.x; i < a.n_seg * ARR_BINS; i += blockDim.x)
            if (bt.larr[i]) {
                const int k = i / ARR_BINS, j = i % ARR_BINS;
                unsigned long long* dst = j < SPX_ARRIVAL_E_BINS
                                              ? &a.arr_E[(size_t)k * SPX_ARRIVAL_E_BINS + j]
                                              : &a.arr_A[(size_t)k * SPX_ARRIVAL_A_BINS + (j - SPX_ARRIVAL_E_BINS)];
                atomicAdd(dst, (unsigned long long)bt.larr[i]);
            }
}

// Wave-private run of queue slots [q, q_end), reserved QUEUE_CHUNK at a time with one
// atomic on the queue length.  Slots a wave leaves unused are marked empty when it exits.
struct QRun {
    uint64_t q = 0, q_end = 0;
};

// Lanes whose atom thermalised in the last flight hand it to the diffusive queue and become
// free.  Slots come from the wave's run (a hand-over may continue into a fresh run).  Their
// collisions are counted here; thermalisation itself is counted when the walk ends.
__device__ __forceinline__ void hand_over(const TransportArgs& a, const SegDev<float>& S, uint32_t pid, int seg,
                                          Particle<float>& p, LaneAcc& acc, QRun& Q, int lane)
{
    const uint64_t T = __ballot(p.st == ST_DIFFUSIVE);
    if (T == 0) return;
    const uint64_t n = (uint64_t)__popcll(T);
    const uint64_t rem = Q.q_end - Q.q;
    uint64_t fresh = 0;
    if (rem < n) {
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd((unsigned long long*)&a.qstate[QS_QUEUE], (unsigned long long)QUEUE_CHUNK);
        fresh = __shfl(b, 0);
    }
    if (p.st == ST_DIFFUSIVE) {
        const uint64_t rank = lanes_below(T);
        const uint64_t slot = rank < rem ? Q.q + rank : fresh + (rank - rem);   // < queue capacity
        ThermRec r;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            r.x[i] = p.x[i];
            r.xc[i] = p.xc[i];
        }
        r.E = p.E;
        r.pid = pid;
        r.seg = (uint32_t)seg;
        r.e = p.e;
        r.lam_bits = __float_as_uint(S.lam_l2);
        r.cfgcat = S.cfgcat;
        a.queue[slot] = r;
        acc.c[C_COLLISIONS] += p.ncoll;
        p.st = ST_DEAD;
    }
    if (rem < n) {
        Q.q = fresh + (n - rem);
        Q.q_end = fresh + QUEUE_CHUNK;
    } else {
        Q.q += n;
    }
}

// Mark the wave's unused reserved slots as empty (pid ~0).
__device__ __forceinline__ void close_run(const TransportArgs& a, const QRun& Q, int lane)
{
    if (Q.q + (uint64_t)lane < Q.q_end) a.queue[Q.q + lane].pid = 0xFFFFFFFFu;
}

// A history that ended in the ballistic phase waits for the wave's next refill point, where the
// ended histories and the thermalised atoms of the wave are settled together (a lane would idle
// until then anyway): its outcome is packed into the clearance-radius register, unused in this
// phase, as state | bin << 2.
constexpr int ST_ENDED = 3;

__device__ __forceinline__ void mark_ended(Particle<float>& p, const Term& t)
{
    p.st = ST_ENDED;
    p.r2 = __uint_as_float((uint32_t)t.state | ((uint32_t)(t.bin < 0 ? 0 : t.bin) << 2));
}

// Settle the wave's ended histories (counters, tally, record) and queue its thermalised atoms.
// The incidence cosine of a deposit is recomputed from its direction, with the operations of
// hit_term.
template <bool ARR>
__device__ __forceinline__ void settle_ballistic(const TransportArgs& a, const BlockTally& bt,
                                                 const SegDev<float>* __restrict__ segs, uint32_t pid, int seg,
                                                 Particle<float>& p, LaneAcc& acc, QRun& Q, int lane)
{
    if (__ballot(p.st == ST_ENDED) != 0 && p.st == ST_ENDED) {
        const SegDev<float>& s = segs[seg];
        const uint32_t bits = __float_as_uint(p.r2);
        Term t;
        t.state = (int)(bits & 3u);
        t.bin = t.state == HIT_DEPOSITED ? (int)(bits >> 2) : -1;
        t.cos_in = t.state == HIT_DEPOSITED ? (float)(-dot3(p.d, s.sub_n)) : 0.f;
        terminate<ARR>(a, bt, s, pid, p, t, acc);
    }
    if (__ballot(p.st == ST_DIFFUSIVE) != 0) hand_over(a, segs[seg], pid, seg, p, acc, Q, lane);
}

// Ballistic flights of the lanes in segment S (uniform: its constants stay in scalar
// registers) until the wave should refill (lanes that ended, thermalised or are free count) or
// has no ballistic lane left.
__device__ __forceinline__ void ballistic_loop(const TransportArgs& a, const SegDev<float>& S, uint32_t pid,
                                               Particle<float>& p, bool drained)
{
    for (;;) {
        if (p.st == ST_BALLISTIC) {
            const Term t = step_mode<float, ST_BALLISTIC>(S, a.tab, a.k0, a.k1, pid, a.cap, p);
            if (t.state != HIT_NONE) mark_ended(p, t);
        }
        if (__ballot(p.st == ST_BALLISTIC) == 0) break;
        if (!drained && __popcll(__ballot(p.st != ST_BALLISTIC)) >= a.refill_ballistic) break;
    }
}

// Histories of lanes at the event cap (rare) escape, ended one segment at a time.
template <bool ARR>
__device__ __forceinline__ void escape_capped(const TransportArgs& a, const BlockTally& bt,
                                              const SegDev<float>* __restrict__ segs, int seg, uint32_t pid,
                                              Particle<float>& p, LaneAcc& acc, bool capped)
{
    for (uint64_t R = __ballot(capped); R != 0;) {
        const int sL = __builtin_amdgcn_readlane(seg, __ffsll((unsigned long long)R) - 1);
        const bool mine = capped && seg == sL;
        R &= ~__ballot(mine);
        if (mine) {
            capped = false;
            terminate<ARR>(a, bt, segs[sL], pid, p, Term{HIT_ESCAPED, -1, 0.f}, acc);
        }
    }
}

// The held steps of the wave (mask H != 0), tested together: with the geometry read once for
// the wave when they share a segment (the common case), else each lane reading its own.
template <bool ARR>
__device__ __forceinline__ void resolve_held(const TransportArgs& a, const BlockTally& bt,
                                             const SegDev<float>* __restrict__ segs, int seg, uint32_t pid,
                                             Particle<float>& p, LaneAcc& acc, bool& held, uint64_t H)
{
    const int sL = __builtin_amdgcn_readlane(seg, __ffsll((unsigned long long)H) - 1);
    acc.c[C_TESTED] += held ? 1u : 0u;
    if (__ballot(held && seg != sL) == 0) {
        if (held) {
            held = false;
            const SegDev<float>& S = segs[sL];
            const Term t = diffusive_resolve(S, p);
            if (t.state != HIT_NONE) terminate<ARR>(a, bt, S, pid, p, t, acc);
        }
    } else if (held) {
        held = false;
        const SegDev<float>& S = segs[seg];
        const Term t = diffusive_resolve(S, p);
        if (t.state != HIT_NONE) terminate<ARR>(a, bt, S, pid, p, t, acc);
    }
}

// Diffusive steps of the lanes in segment S with deferred surface tests: a lane whose
// step leaves its clearance ball holds the step and idles until at least a.defer_min lanes
// hold one (or every diffusive lane does, or the loop is about to end); then the held
// steps are tested together, so the long test runs in few iterations.  No step is held
// when the loop returns.
template <bool ARR>
__device__ __forceinline__ void diffusive_loop(const TransportArgs& a, const BlockTally& bt,
                                               const SegDev<float>* __restrict__ segs, int seg, float lam_l2,
                                               uint32_t cfgcat, uint32_t pid, Particle<float>& p, LaneAcc& acc,
                                               bool drained)
{
    bool held = false;
    for (;;) {
        // several advances (two steps each) between the wave's checks below: a lane that holds
        // a step, or reaches the cap, sits out the rest of them
        bool capped = false;
#pragma unroll
        for (int rep = 0; rep < ADVANCES_PER_CHECK; ++rep)
            if (p.st == ST_DIFFUSIVE && !held && !capped)
                capped = diffusive_advance(lam_l2, cfgcat, a.k0, a.k1, pid, a.cap, p, held).state != HIT_NONE;
        escape_capped<ARR>(a, bt, segs, seg, pid, p, acc, capped);
        const uint64_t H = __ballot(held);
        const uint64_t M = __ballot(p.st == ST_DIFFUSIVE);
        bool stop = M == 0 || (!drained && __popcll(__ballot(p.st == ST_DEAD)) >= a.refill_min) ||
                    (drained && __popcll(M) <= COOP_MAX);
        if (H != 0 && (stop || H == M || __popcll(H) >= a.defer_min)) {
            resolve_held<ARR>(a, bt, segs, seg, pid, p, acc, held, H);
            const uint64_t M2 = __ballot(p.st == ST_DIFFUSIVE);
            stop = M2 == 0 || (!drained && __popcll(__ballot(p.st == ST_DEAD)) >= a.refill_min) ||
                   (drained && __popcll(M2) <= COOP_MAX);
        }
        if (stop) break;
    }
}

// Ballistic phase of one round: every ticket of the round, from launch until the atom ends
// on a surface, escapes, or thermalises (then it is queued for the diffusive phase).
// Dynamic LDS: per-segment counters (u64, when lds_counters) then the tally (u32, when lds_tally).
// At most 96 VGPRs: five waves per SIMD hide the latency of the transcendental and
// integer-multiply chains.
template <bool ARR>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5)))
k_ballistic32(TransportArgs a, const SegDev<float>* __restrict__ segs)
{
    extern __shared__ unsigned long long lds[];
    BlockTally bt;
    lds_setup(a, bt, lds);
    const int lane = threadIdx.x & 63;
    Particle<float> p;
    p.st = ST_DEAD;
    p.e = p.ndiff = p.ncoll = 0;
    uint32_t pid = 0;
    int seg = 0;
    LaneAcc acc;
    Tickets T;
    QRun Q;
    int cur_pos = 0, last_pos = 0;        // wave-uniform current position in ticket order ...
    uint64_t cur_lo = 0, cur_hi = 0;      // ... and its ticket range (empty until the first refill)
    for (;;) {
        settle_ballistic<ARR>(a, bt, segs, pid, seg, p, acc, Q, lane);
        const uint64_t dead = __ballot(p.st == ST_DEAD);
        const int n_dead = __popcll(dead);
        if (!T.drained && n_dead > 0 && (n_dead >= a.refill_ballistic || n_dead == 64)) {
            const uint64_t my = claim(T, &a.qstate[QS_TICKETS], a.chunk_ballistic, a.total, dead, lane);
            if (my != ~0ull) {
                const uint64_t g = a.tbase + my;
                // the ticket's position in ticket order: the wave's current one (tickets of a
                // run are consecutive, segments long), else a binary search of the prefix table
                int lo = cur_pos;
                if (!(g >= cur_lo && g < cur_hi)) {
                    lo = 0;
                    int hi = a.n_seg;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (a.tfirst[mid] <= g) lo = mid; else hi = mid;
                    }
                }
                last_pos = lo;
                const int sg = (int)a.torder[lo];
                pid = (uint32_t)(g - a.tfirst[lo]);
                if (sg != acc.seg) {
                    flush_acc(a, bt, acc);
                    acc.seg = sg;
                }
                seg = sg;
                start(segs[seg], a.k0, a.k1, pid, p);
                acc.c[C_LAUNCHED] += 1;
            }
            // the position of the wave's last new ticket becomes the current one
            const uint64_t got = __ballot(my != ~0ull);
            if (got != 0) {
                cur_pos = __builtin_amdgcn_readlane(last_pos, 63 - __clzll((long long)got));
                cur_lo = a.tfirst[cur_pos];
                cur_hi = a.tfirst[cur_pos + 1];
            }
        }
        const uint64_t B = __ballot(p.st == ST_BALLISTIC);
        if (B == 0) {
            if (T.drained) break;
            continue;
        }
        const int s0 = __builtin_amdgcn_readlane(seg, __ffsll((unsigned long long)B) - 1);
        if (__ballot(p.st == ST_BALLISTIC && seg != s0) == 0) {
            ballistic_loop(a, segs[s0], pid, p, T.drained);
        } else if (p.st == ST_BALLISTIC) {
            // lanes of several segments: one flight with per-lane constants
            const SegDev<float>& s = segs[seg];
            const Term t = step_mode<float, ST_BALLISTIC>(s, a.tab, a.k0, a.k1, pid, a.cap, p);
            if (t.state != HIT_NONE) mark_ended(p, t);
        }
    }
    close_run(a, Q, lane);
    lds_flush(a, bt, acc);
}

// Diffusive phase of one round: the walks of the atoms queued by the ballistic phase.  Lanes
// of any segments walk together (the step needs only two per-lane numbers of the segment), so
// a wave never falls back to one step at a time.
template <bool ARR>
__device__ __forceinline__ void diffusive_phase(TransportArgs& a, const SegDev<float>* __restrict__ segs)
{
    extern __shared__ unsigned long long lds[];
    BlockTally bt;
    lds_setup(a, bt, lds);
    const uint64_t total = a.qstate[QS_QUEUE];   // written by the ballistic phase of this round
    const int lane = threadIdx.x & 63;
    Particle<float> p;
    p.st = ST_DEAD;
    p.e = p.ndiff = p.ncoll = 0;
    uint32_t pid = 0;
    int seg = 0;
    float lam_l2 = 0.f;        // the lane's segment: thermal mean free path (times ln 2), Philox word
    uint32_t cfgcat = 0;
    LaneAcc acc;
    Tickets T;
    for (;;) {
        const uint64_t dead = __ballot(p.st == ST_DEAD);
        const int n_dead = __popcll(dead);
        if (!T.drained && n_dead > 0 && (n_dead >= a.refill_min || n_dead == 64)) {
            const uint64_t my = claim(T, &a.qstate[QS_DIFFUSIVE], TICKET_CHUNK, total, dead, lane);
            const uint32_t qpid = my != ~0ull ? a.queue[my].pid : 0xFFFFFFFFu;
            if (qpid != 0xFFFFFFFFu) {                 // empty slots (left unused by a wave) are skipped
                const ThermRec r = a.queue[my];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    p.x[i] = r.x[i];
                    p.xc[i] = r.xc[i];
                }
                p.E = r.E;
                p.e = r.e;
                p.ndiff = 0;
                p.ncoll = 0;
                p.r2 = -1.f;           // no clearance ball yet: the first step is tested
                p.st = ST_DIFFUSIVE;
                pid = r.pid;
                const int sg = (int)r.seg;
                if (sg != acc.seg) {
                    flush_acc(a, bt, acc);
                    acc.seg = sg;
                }
                seg = sg;
                lam_l2 = __uint_as_float(r.lam_bits);
                cfgcat = r.cfgcat;
            }
        }
        const uint64_t D = __ballot(p.st == ST_DIFFUSIVE);
        if (D == 0) {
            if (T.drained) break;
            continue;
        }
        // Last walks of a drained wave: walked by the whole wave, up to four at a time (up to 64,
        // 32 or 16 steps each per pass), until their steps leave the balls; then the held steps
        // are tested together.
        // Every pass takes or holds a step of each walker, or leaves it at the cap, where it
        // escapes, so the walks end.
        if (T.drained && __popcll(D) <= COOP_MAX) {
            bool held = false;
            for (uint64_t W = D; W != 0;) {
                uint64_t G = 0;                  // the next (up to) four walkers
                for (int q = 0; q < 4 && W != 0; ++q) {
                    G |= W & (~W + 1);
                    W &= W - 1;
                }
                coop_walk(a.k0, a.k1, a.cap, G, lam_l2, cfgcat, pid, p, held, lane);
            }
            escape_capped<ARR>(a, bt, segs, seg, pid, p, acc, p.st == ST_DIFFUSIVE && !held && p.e >= a.cap);
            const uint64_t H = __ballot(held);
            if (H != 0) resolve_held<ARR>(a, bt, segs, seg, pid, p, acc, held, H);
            continue;
        }
        diffusive_loop<ARR>(a, bt, segs, seg, lam_l2, cfgcat, pid, p, acc, T.drained);
    }
    lds_flush(a, bt, acc);
}

// At most 96 VGPRs (five waves per SIMD, as the ballistic phase).  With the arrival tallies
// a few values spill to scratch at five waves, outside the steps of the walk; that still runs
// faster than four waves without spills.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5)))
k_diffusive32(TransportArgs a, const SegDev<float>* __restrict__ segs)
{
    diffusive_phase<false>(a, segs);
}
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5)))
k_diffusive32_arr(TransportArgs a, const SegDev<float>* __restrict__ segs)
{
    diffusive_phase<true>(a, segs);
}

// Arrival outputs of the comparator (nullable as a group) with its FP64 bin edges.
struct Arrivals64 {
    unsigned long long* E;      // this segment's energy histogram
    unsigned long long* A;      // this segment's angle histogram
    unsigned long long* esum;   // per tally bin of the plan
    const double* e_edges;
    const double* c_edges;
};

__global__ void __launch_bounds__(256) k_transport64(const SegDev<double>* __restrict__ segp, TabDev<double> tab,
                                                     uint32_t k0, uint32_t k1, uint32_t cap,
                                                     unsigned long long* __restrict__ counts,
                                                     unsigned long long* __restrict__ counters,
                                                     spx_record* __restrict__ records, Arrivals64 arr)
{
    const SegDev<double>& s = *segp;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc[N_COUNTERS] = {};
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
        // every diffusive step is tested here: those that ended in the gas and the last one
        // (unless the history stopped at the event cap)
        acc[C_TESTED] = p.ndiff + ((p.st == ST_DIFFUSIVE && t.state != HIT_ESCAPED) ? 1u : 0u);
        if (t.state == HIT_DEPOSITED) {
            const uint64_t b = s.bin_off + (uint64_t)t.bin;
            atomicAdd(&counts[b], 1ull);
            if (arr.E) {
                atomicAdd(&arr.E[energy_bin(arr.e_edges, p.E)], 1ull);
                atomicAdd(&arr.A[angle_bin(arr.c_edges, (double)t.cos_in)], 1ull);
                atomicAdd(&arr.esum[b], energy_units(p.E));
            }
        }
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

// Zero the outputs (a kernel, so that it can sit in a graph).
__global__ void k_zero(unsigned long long* counts, uint64_t n_counts, unsigned long long* counters, uint64_t n_counters)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_counts; i += stride) counts[i] = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_counters; i += stride) counters[i] = 0;
}

// Reset a round's ticket counters and queue length.
__global__ void k_round_reset(uint64_t* qstate)
{
    for (uint32_t i = threadIdx.x; i < QSTATE_WORDS; i += blockDim.x) qstate[i] = 0;
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

static int zero_u64(uint64_t* p, uint64_t n, LaunchSink& sink)
{
    if (!p || n == 0) return SPX_OK;
    KLaunch k;
    k.func = (const void*)k_zero;
    k.grid = dim3((unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 + 1 : 4096));
    k.block = dim3(256);
    k.arg((unsigned long long*)p);
    k.arg(n);
    k.arg((unsigned long long*)nullptr);
    k.arg((uint64_t)0);
    return sink.put(k);
}

static int put_zero(Plan* P, const Outputs& o, LaunchSink& sink)
{
    SPX_TRY(zero_u64(o.counts, P->n_bins_total, sink));
    SPX_TRY(zero_u64(o.counters, (uint64_t)P->n_seg * N_COUNTERS, sink));
    if (o.arr_E) {
        SPX_TRY(zero_u64(o.arr_E, (uint64_t)P->n_seg * SPX_ARRIVAL_E_BINS, sink));
        SPX_TRY(zero_u64(o.arr_A, (uint64_t)P->n_seg * SPX_ARRIVAL_A_BINS, sink));
        SPX_TRY(zero_u64(o.esum, P->n_bins_total, sink));
    }
    return SPX_OK;
}

static int put_normalize(Plan* P, const uint64_t* d_counts, double* d_profiles, LaunchSink& sink)
{
    const uint64_t n = P->n_bins_total;
    KLaunch k;
    k.func = (const void*)k_normalize;
    k.grid = dim3((unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 + 1 : 4096));
    k.block = dim3(256);
    k.arg((const unsigned long long*)d_counts);
    k.arg((const uint64_t*)P->d_bin_off);
    k.arg((const double*)P->d_seg_norm);
    k.arg((int)P->n_seg);
    k.arg(n);
    k.arg(d_profiles);
    return sink.put(k);
}

int StreamSink::put(const KLaunch& k)
{
    if (k.n_args < 0 || !k.func) {
        set_error("internal: malformed kernel launch");
        return SPX_ESTATE;
    }
    if (events && k.phase == 1) SPX_HIP(hipEventRecord(events[3 * round], st));
    void* args[8];
    k.pointers(args);
    SPX_HIP(hipLaunchKernel(k.func, k.grid, k.block, args, k.smem, st));
    if (events && k.phase == 1) SPX_HIP(hipEventRecord(events[3 * round + 1], st));
    if (events && k.phase == 2) SPX_HIP(hipEventRecord(events[3 * round++ + 2], st));
    return SPX_OK;
}

// Dynamic LDS of the FP32 transport for a plan: counters if they fit, tally if it fits, arrival
// histograms (when requested) if they fit.
size_t transport32_lds(const Plan* P, bool arrivals, bool* lds_counters, bool* lds_tally, bool* lds_arrivals)
{
    const size_t cbytes = (size_t)P->n_seg * N_COUNTERS * sizeof(unsigned long long);
    const size_t tbytes = (size_t)P->n_bins_total * sizeof(uint32_t);
    const size_t abytes = (size_t)P->n_seg * ARR_BINS * sizeof(uint32_t);
    *lds_counters = cbytes <= LDS_COUNTERS_MAX;
    *lds_tally = tbytes <= LDS_TALLY_MAX;
    *lds_arrivals = arrivals && abytes <= LDS_ARRIVALS_MAX;
    return (*lds_counters ? cbytes : 0) + (*lds_tally ? tbytes : 0) + (*lds_arrivals ? abytes : 0);
}

int occupancy_transport32(const Plan* P, int threads, int* bpc_ballistic, int* bpc_diffusive)
{
    bool lc, lt, la;
    const size_t smem = transport32_lds(P, false, &lc, &lt, &la);
    int b1 = 0, b2 = 0;
    SPX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, k_ballistic32<false>, threads, smem));
    SPX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, k_diffusive32, threads, smem));
    *bpc_ballistic = b1;
    *bpc_diffusive = b2;
    return SPX_OK;
}

// Rounds of a ticket space of `total` tickets: as few as round_max allows, of equal size.
uint64_t rounds_of(uint64_t total, uint64_t round_max)
{
    return total == 0 ? 0 : (total + round_max - 1) / round_max;
}

int build_transport32(Plan* P, uint64_t seed, const Outputs& o, const uint64_t* tfirst, uint64_t total,
                      const Shape& sh, const QueueMem& q, LaunchSink& sink)
{
    SPX_TRY(put_zero(P, o, sink));
    TransportArgs a;
    std::memset(&a, 0, sizeof(a));     // padding too: launches are compared bytewise
    a.segs = P->d_seg32;
    a.tab.theta = P->d_theta32;
    a.tab.betamax = P->d_betamax32;
    a.tab.ne = P->params.table_ne;
    a.tab.ns = P->params.table_ns;
    a.tab.xs = (float)((P->params.table_ne - 1) / ((P->params.log_eps_hi - P->params.log_eps_lo) * 3.321928094887362));
    a.tfirst = tfirst;
    a.torder = P->d_torder;
    a.queue = q.queue;
    a.qstate = q.qstate;
    a.counts = (unsigned long long*)o.counts;
    a.counters = (unsigned long long*)o.counters;
    a.records = o.records;
    a.arr_E = (unsigned long long*)o.arr_E;
    a.arr_A = (unsigned long long*)o.arr_A;
    a.esum = (unsigned long long*)o.esum;
    a.e_edges = P->d_edges32;
    a.c_edges = P->d_edges32 + SPX_ARRIVAL_E_BINS + 1;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.cap = P->params.event_cap;
    a.n_seg = P->n_seg;
    a.refill_min = sh.refill_min;
    a.refill_ballistic = sh.refill_ballistic;
    a.defer_min = sh.defer_min;
    a.n_bins = (uint32_t)P->n_bins_total;
    bool lc, lt, la;
    const size_t smem = transport32_lds(P, o.arr_E != nullptr, &lc, &lt, &la);
    int blocks_diff_arr = sh.blocks_diff;
    if (o.arr_E) {
        int bpc_arr = 0;
        SPX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc_arr, k_diffusive32_arr, sh.threads, smem));
        if (bpc_arr > 0) blocks_diff_arr = std::min(sh.blocks_diff, bpc_arr * P->n_cu);
    }
    a.lds_counters = lc ? 1 : 0;
    a.lds_tally = lt ? 1 : 0;
    a.lds_arrivals = la ? 1 : 0;
    const uint64_t n_rounds = rounds_of(total, q.round_max);
    const uint64_t per_round = n_rounds ? (total + n_rounds - 1) / n_rounds : 0;
    // every queue slot a round can reserve: its atoms plus at most one unused run per wave
    const uint64_t waves = (uint64_t)sh.blocks * (uint64_t)((sh.threads + 63) / 64);
    if (n_rounds && per_round + waves * QUEUE_CHUNK > q.cap) {
        set_error("internal: round larger than the thermalisation queue");
        return SPX_ESTATE;
    }
    const SegDev<float>* segs = P->d_seg32;
    for (uint64_t r = 0; r < n_rounds; ++r) {
        a.tbase = r * per_round;
        a.total = (a.tbase + per_round < total) ? per_round : total - a.tbase;
        // the largest power-of-two chunk in [TICKET_CHUNK, TICKET_CHUNK_BALLISTIC_MAX] that
        // still gives every wave about four chunks of the round
        uint64_t cb = TICKET_CHUNK;
        while (2 * cb <= TICKET_CHUNK_BALLISTIC_MAX && 2 * cb * 4 * waves <= a.total) cb *= 2;
        a.chunk_ballistic = (uint32_t)cb;
        KLaunch reset;
        reset.func = (const void*)k_round_reset;
        reset.block = dim3(64);
        reset.arg(q.qstate);
        SPX_TRY(sink.put(reset));
        KLaunch bal;
        bal.func = a.arr_E ? (const void*)k_ballistic32<true> : (const void*)k_ballistic32<false>;
        bal.grid = dim3((unsigned)sh.blocks);
        bal.block = dim3((unsigned)sh.threads);
        bal.smem = (uint32_t)smem;
        bal.phase = 1;
        bal.arg(a);
        bal.arg(segs);
        SPX_TRY(sink.put(bal));
        // the instance with the arrival tallies has its own resident limit (fewer waves per SIMD)
        KLaunch dif;
        dif.func = a.arr_E ? (const void*)k_diffusive32_arr : (const void*)k_diffusive32;
        dif.grid = dim3((unsigned)(a.arr_E ? blocks_diff_arr : sh.blocks_diff));
        dif.block = dim3((unsigned)sh.threads);
        dif.smem = (uint32_t)smem;
        dif.phase = 2;
        dif.arg(a);
        dif.arg(segs);
        SPX_TRY(sink.put(dif));
    }
    if (o.profiles) SPX_TRY(put_normalize(P, o.counts, o.profiles, sink));
    return SPX_OK;
}

int launch_transport64(Plan* P, uint64_t seed, const Outputs& o, hipStream_t st)
{
    StreamSink sink(st, nullptr);
    SPX_TRY(put_zero(P, o, sink));
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
        Arrivals64 arr{nullptr, nullptr, nullptr, P->d_edges64, P->d_edges64 + SPX_ARRIVAL_E_BINS + 1};
        if (o.arr_E) {
            arr.E = (unsigned long long*)(o.arr_E + (size_t)k * SPX_ARRIVAL_E_BINS);
            arr.A = (unsigned long long*)(o.arr_A + (size_t)k * SPX_ARRIVAL_A_BINS);
            arr.esum = (unsigned long long*)o.esum;
        }
        hipLaunchKernelGGL(k_transport64, dim3((unsigned)blocks), dim3(256), 0, st, P->d_seg64 + k, tab,
                           (uint32_t)seed, (uint32_t)(seed >> 32), P->params.event_cap,
                           (unsigned long long*)o.counts, (unsigned long long*)(o.counters + (size_t)k * N_COUNTERS),
                           o.records, arr);
        SPX_HIP(hipGetLastError());
    }
    if (o.profiles) SPX_TRY(put_normalize(P, o.counts, o.profiles, sink));
    return SPX_OK;
}

void arrival_edges(double* e_edges, double* c_edges)
{
    for (int k = 0; k <= SPX_ARRIVAL_E_BINS; ++k) e_edges[k] = std::pow(10.0, -3.0 + k / 10.0);
    for (int k = 0; k <= SPX_ARRIVAL_A_BINS; ++k) c_edges[k] = std::cos(k * 3.14159265358979323846 / 180.0);
}

}  // namespace spx
