// ssa_sim.hpp -- the per-lane event loop of the direct method (paper Section 2) with the
// grid alignment of Section 3.2.1, shared by the compiled generic kernel and the kernels
// specialised per network at run time.
//
// One lane runs one trajectory at a time.  A persistent grid of 256-lane workgroups pulls
// work items (a network and a chunk of up to 64 trajectory indices) from a global
// counter; each wave hands indices to its lanes as they finish, so lanes whose
// trajectories end early are refilled instead of idling (trajectories end after very
// different event counts).  A wave only switches network once all its lanes are idle, so
// every reaction-table read stays wave-uniform.
//
// How a network's state is held (registers or LDS), how its propensities are formed and
// how a reaction changes the state is delegated to a policy class:
//   switch_net(n)                   the wave starts working on network n
//   reset(n)                        start a trajectory at x0
//   eval<MM>(n, a)                  a_j for j < MM (entries at or beyond n.M must be 0)
//   one(n, j)                       a_j for a single reaction (rare path)
//   total(n), select(n, u)          MM == 0 (many reactions): a0, and the count of partial
//                                   sums <= u, each from a fresh pass over the reactions
//   for_each_species(f)             f(s, x_s) for every species
//   apply(n, sel, f)                apply reaction sel: f(s, x_old, x_new) per changed species
//                                   (a policy may also call f with x_new == x_old)
//
// Selective memory (Section 3.2.1) in difference form: the grid value x(t_g) of a
// trajectory is x0 plus every change with t_e <= t_g, so an event at t_e contributes its
// change nu and its change of x^2, (2x + nu) nu, to the first grid bin b with
// t_b >= t_e; a prefix sum over the bins then gives sum x and sum x^2 at every grid point.
// All of it is exact integer arithmetic, so the order of the additions does not matter
// and the result is deterministic.
//
// The forward pass (sim_fwd) keeps these sums the way the paper's selective memory keeps
// stream items: a wave simulates a generation of up to 64 trajectories and holds a
// window of W grid bins in LDS that follows the wavefront of simulation time.  The window
// starts at the smallest pending bin over the wave's lanes; a lane whose next event falls
// beyond the window waits (it is ahead in simulation time, so it has slack), and bins
// that every lane has passed are flushed out of LDS and the window slides on.  Flushes go
// either to a slab of global memory private to the wave (plain coalesced read-modify-
// writes, summed by a reduction kernel afterwards) or, for batched launches, into the
// network's accumulators with atomic adds.
#pragma once

#include "ssa_device.hpp"

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC_RTC__)
#define SSA_CONST __attribute__((address_space(4)))
#define SSA_GLOBAL __attribute__((address_space(1)))
#else
#define SSA_CONST
#define SSA_GLOBAL
#endif

namespace ssa {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kChunk = 64;         // trajectory indices per work item
constexpr int kChg = 4;            // changed species per reaction in the packed tables and the event log
constexpr int kSmallD2 = 1 << 24;  // |(2x+nu)nu| below this goes whole to the low accumulator;
                                   // larger values add their low 24 bits there and value >> 24
                                   // to the high accumulator, so low words grow by < 2^24 per event

enum Mode : int { kFwd = 0, kRec = 1, kBwd = 2, kEvt = 3 };

enum Flags : uint32_t { kFlagOverflow = 1u, kFlagEventLimit = 2u, kFlagRecordsFull = 4u };

constexpr unsigned kLogChunk = 1024;   // event-log slots a wave reserves at a time (>= 64 kChg)

// A wave's event-log slots: the rest of its current chunk [next, end) and, once that may
// be too short for a step (64 kChg records), the following chunk nxt (~0: none yet).  All
// fields change only where the wave is converged, so they are wave-uniform.
struct LogSlots {
    unsigned long long next = 0, end = 0, nxt = ~0ull;
    // slot of the j-th record of this step
    __device__ __forceinline__ unsigned long long at(unsigned long long j) const {
        return next + j < end ? next + j : nxt + (next + j - end);
    }
    // after a step that took `used` slots; reserve ahead when a step might not fit (only a
    // wave with an active lane, so only waves that hold work reserve)
    __device__ __forceinline__ void advance(uint32_t used, bool busy, unsigned long long *resv, uint32_t lane) {
        next += used;
        if (next >= end && nxt != ~0ull) {
            const unsigned long long over = next - end;
            next = nxt + over;
            end = nxt + kLogChunk;
            nxt = ~0ull;
        }
        if (busy && nxt == ~0ull && end - next < (unsigned long long)(kWave * kChg)) {
            unsigned long long b = 0;
            if (lane == 0) b = atomicAdd(resv, (unsigned long long)kLogChunk);
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, 0);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), 0);
            nxt = ((unsigned long long)hi << 32) | lo;
        }
    }
};

// Time grid description.  A grid with t_g = fl(fl(T g) / D) for every g (the uniform grid
// of the workloads) is "uniform": its points are recomputed exactly from (T, D) instead of
// being loaded, which keeps the event loop free of vector-memory loads.  Any other
// non-decreasing grid is read from memory.
struct GridInfo {
    double T, D;        // uniform: t_g = (T * g) / D
    double lo, scale;   // affine guess ceil((t - lo) * scale) of the first index >= t
    int32_t uniform, pad;
};

// One network in a launch.  The reaction tables (rx, rate, chg) are read by the generic
// policy only; run-time specialised kernels carry the structure as constants and read
// just the rates.
struct NetDev {
    int32_t S, M, G, nb_hist;
    int64_t n_traj;          // trajectories of this network in the run (partition sizes)
    double t_end;
    uint32_t key0, key1;     // Philox key = seed
    uint64_t max_events;
    const uint32_t *rx;      // [>= M] packed reactant encoding (generic policy)
    const double *rate;      // [>= M] rate constants (zero-padded for the generic policy)
    const int32_t *chg;      // [M * 4] packed changes (generic policy)
    const int32_t *x0;       // [S]
    const double *grid;
    const GridInfo *ginfo;
    // forward: difference sums [G][S][2] (atomic flush mode), high parts of large
    // (2x+nu)nu contributions [G][S] (value >> 24, atomic), histogram diffs [G][nb]
    unsigned long long *D;
    unsigned long long *Dhi;
    int32_t *Hd;
    int32_t h_species, h_lo, h_width;
    int32_t q;               // 64-chunk sum order: reactions per lane (one trajectory per wave)
    // 64-chunk order above 8 reactions per lane: dependency lists of the fired reaction,
    // entries (LDS slot i * 64 + l of reaction l q + i, packed reactant code), [M + 1] offsets
    const int2 *dep;
    const double *dep_rate;  // rate constant of each entry's reaction (this run's rates)
    const int32_t *dep_ptr;
    // record
    int64_t rec_begin;
    int32_t *rec_states;
    uint64_t *rec_events, *rec_draws;
    double *rec_tlast;
    int64_t *rec_nf;
    double *rec_aint;
    // backward: prefix rows [G+1] (see PrefixRow), per-trajectory rows [n_traj][M]; bp_quad:
    // the rows carry the variance columns (one-trajectory-per-wave kernels read it; the
    // lane kernels are instantiated per layout)
    const void *bp;
    const double *bpt;       // the column values of each grid point [G][ncol] (one-crossing intervals)
    double *gtraj;
    int32_t bp_quad;
    // event log: one record per changed species of every applied event (key: the event
    // time's bits; value: packed species, change, old count); ev_cursor counts the records;
    // with ev_key == nullptr nothing else is written
    unsigned long long *ev_key, *ev_val, *ev_cursor;
    // slot allocator of the lane kernels: a wave reserves kLogChunk slots at a time (the
    // next chunk before the current one may run short, so no slot is skipped), so records
    // land in [0, *ev_resv) with gaps only at the end of each wave's last two chunks (the
    // caller fills the keys with ~0 first, which sorts after every event time); *ev_cursor
    // still counts the records exactly.  The one-trajectory-per-wave kernels place records
    // at the cursor.
    unsigned long long *ev_resv;
    int64_t ev_cap;
    // event log in epochs: each trajectory starts from a saved state (rs_*, or the initial
    // state when rs_t is NULL) and stops before its first event beyond t_pause, saving its
    // state to ws_*: counts [n_traj][S], time (-1 once the trajectory has ended), the next
    // draw's index and the events applied so far
    const int32_t *rs_x;
    const double *rs_t;
    const uint64_t *rs_k, *rs_ev;
    int32_t *ws_x;
    double *ws_t;
    uint64_t *ws_k, *ws_ev;
    double t_pause;
    // forward in generations: each trajectory's event count (saturated to 32 bits), or NULL
    uint32_t *len_out;
};

// Event-log record value: species (12 bits) | change (20-bit two's complement) << 12 |
// count before the event << 32.
__host__ __device__ __forceinline__ unsigned long long ev_pack(int32_t s, int32_t dl, int32_t xo) {
    return ((unsigned long long)(uint32_t)xo << 32) | ((unsigned long long)((uint32_t)dl & 0xfffffu) << 12) |
           (unsigned long long)(uint32_t)s;
}

// Work description.  A single-network launch passes its network by value (net0) and the
// trajectory range [range_begin, range_end) cut into chunks of kChunk; a batched launch
// passes a device table of networks and an explicit work-item list.
struct WorkList {
    NetDev net0;
    int64_t range_begin, range_end;
    const NetDev *nets;
    const int32_t *item_net;     // [n_items]
    const int64_t *item_begin;   // [n_items] first trajectory index of the chunk
    const int32_t *item_count;   // [n_items]
    int32_t n_items;
    int32_t s_rows;              // species rows per block in LDS (generic policy)
    int32_t m_rows;              // reactions per LDS change table (generic policy)
    int32_t win_bins;            // forward: grid bins per wave window (power of two)
    int32_t win_words;           // forward: 64-bit LDS words per wave window (win_bins * S_max * 2)
    unsigned long long *slabs;   // forward, slab mode: [waves][G][S][2] wave-private sums
    double *jac_slabs;           // forward with Jacobian: [items][G][S+1][M] per-work-item sums
    unsigned int *counter;       // work-item counter (zeroed before launch)
    unsigned long long *stats;   // [0] events, [1] max steps, [2] flags
    // single-network forward in generations, record, backward, event log: the trajectory at
    // each position of [range_begin, range_end), or NULL for the positions themselves (any
    // order gives the same results: a trajectory keeps its index, its random numbers and its
    // output row)
    const uint32_t *perm;
};

// Error-free transformations (Knuth's two-sum) for double-double prefix sums.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void dd_add(double &h, double &l, double bh, double bl) {
    double s, e;
    two_sum(h, bh, s, e);
    e = e + (l + bl);
    h = s + e;
    l = e - (h - s);
}

// (bh + bl) - (ah + al) within about 1 ulp of the result: bh - ah is exact when the two
// lie within a factor of 2 (Sterbenz) and otherwise the result is at least |bh| / 2, so
// its one rounding costs at most half an ulp of the result either way; the lo parts'
// difference is then added.
__device__ __forceinline__ double dd_diff(double ah, double al, double bh, double bl) {
    return (bh - ah) + (bl - al);
}

// Backward prefix rows (built by bwd_prefix_kernel): row g holds the ncol = 2S + 2 binary64
// hi parts followed by the ncol lo parts stored as binary32 (a double-double's lo part is
// below half an ulp of its hi part, so binary32 keeps the pair to 2^-77 relative),
// 12 ncol bytes per row.
struct PrefixRow {
    const double *hi;
    const float *lo;
    __device__ __forceinline__ PrefixRow(const void *table, int32_t ncol, int32_t g) {
        const char *r = (const char *)table + (size_t)g * 12 * ncol;
        hi = (const double *)r;
        lo = (const float *)(r + 8 * (size_t)ncol);
    }
    // (column c of row b) - (column c of this row)
    __device__ __forceinline__ double diff_to(const PrefixRow &b, int32_t c) const {
        return dd_diff(hi[c], (double)lo[c], b.hi[c], (double)b.lo[c]);
    }
};

// Backward sums over the crossings g in [ga, gb) of one inter-event interval starting at t
// (state x): alpha = sum_g phi_g, beta = sum_g phi_g (t_g - t), from two rows: prefix rows
// (their differences) or, for a single crossing, the point's own row.  QUAD: the rows also
// hold the variance columns Q, QT (weights quadratic in x).
template <bool QUAD, class Policy, class Row>
__device__ __forceinline__ void interval_sums_rows(const Policy &p, const Row &ra, const Row &rb, int32_t S, double t,
                                                   double &alpha, double &beta) {
    double sw = 0.0, swt = 0.0;
    p.for_each_species([&](int32_t s, int32_t xs) {
        const double x = (double)xs;
        const double dW = ra.diff_to(rb, s);
        const double dWT = ra.diff_to(rb, S + s);
        sw = sw + x * dW;
        swt = swt + x * (dWT - t * dW);
        if (QUAD) {
            const double x2 = x * x;
            const double dQ = ra.diff_to(rb, 2 * S + 2 + s);
            const double dQT = ra.diff_to(rb, 3 * S + 2 + s);
            sw = sw + x2 * dQ;
            swt = swt + x2 * (dQT - t * dQ);
        }
    });
    const double dC = ra.diff_to(rb, 2 * S);
    const double dCT = ra.diff_to(rb, 2 * S + 1);
    alpha = sw - dC;
    beta = swt - (dCT - t * dC);
}

template <bool QUAD = false, class Policy>
__device__ __forceinline__ void interval_sums(const Policy &p, const void *P, const double *PT, int32_t S,
                                              int32_t ga, int32_t gb, double t, double &alpha, double &beta) {
    const int32_t ncol = QUAD ? 4 * S + 2 : 2 * S + 2;
    // A single crossing reads its point's row against the zero row 0 of the prefix table
    // (dd_diff(0, 0, v, 0) = v), so both kinds of interval run the same code without a
    // divergent branch.
    const bool one = PT && gb == ga + 1;
    PrefixRow ra(P, ncol, one ? 0 : ga), rb(P, ncol, gb);
    if (one) {
        rb.hi = PT + (size_t)ga * ncol;
        rb.lo = ra.lo;
    }
    interval_sums_rows<QUAD>(p, ra, rb, S, t, alpha, beta);
}

// Wave-uniform copies (scalar registers) of values every lane holds identically.
__device__ __forceinline__ int32_t wave_uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double wave_uniform(double v) {
    return __longlong_as_double(wave_uniform((int64_t)__double_as_longlong(v)));
}
template <class T>
__device__ __forceinline__ T *wave_uniform(T *p) {
    return (T *)wave_uniform((int64_t)(uintptr_t)p);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lane = __lane_id();
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// The current network.  Single-network launches read it from the kernel arguments; a
// batched launch from the device table (scalar loads, indexed by the wave's network).
// The Philox key is laundered once per event so its round-key schedule is recomputed
// with scalar adds rather than pinned in scalar registers.
template <bool BATCH>
__device__ __forceinline__ NetDev current_net(const WorkList &wl, int32_t cur) {
    NetDev n;
    if (BATCH) n = ((const SSA_CONST NetDev *)wl.nets)[wave_uniform(cur)];
    else n = wl.net0;
    asm volatile("" : "+s"(n.key0), "+s"(n.key1));
    return n;
}

// Grid state of the current network, held in wave-uniform registers.
struct GridView {
    const double *grid;
    double T, D, lo, scale;
    int32_t G, uniform;

    __device__ __forceinline__ double at(int32_t g) const {
        return uniform ? (T * (double)g) / D : ((const SSA_GLOBAL double *)grid)[g];
    }
    // First index b > g0 with t_b >= t, given t_{g0} < t (G if none); also returns t_b.
    // The uniform and the memory variant are separate code paths so that the uniform one
    // never waits on vector memory (which would also wait for the event's atomics).
    template <bool UNIFORM>
    __device__ __forceinline__ int32_t next_bin_impl(int32_t g0, double t, double &tb) const {
        auto pt = [&](int32_t g) { return UNIFORM ? (T * (double)g) / D : ((const SSA_GLOBAL double *)grid)[g]; };
        const double gf = ceil((t - lo) * scale);
        int32_t b = gf <= (double)(g0 + 1) ? g0 + 1 : (gf >= (double)G ? G : (int32_t)gf);
        double v = b < G ? pt(b) : __builtin_inf();
        while (b < G && v < t) {
            ++b;
            v = b < G ? pt(b) : __builtin_inf();
        }
        while (b > g0 + 1) {
            const double tp = pt(b - 1);
            if (tp < t) break;
            --b;
            v = tp;
        }
        tb = v;
        return b;
    }
    __device__ __forceinline__ int32_t next_bin(int32_t g0, double t, double &tb) const {
        return uniform ? next_bin_impl<true>(g0, t, tb) : next_bin_impl<false>(g0, t, tb);
    }

    // Division-free form for the event loops: the first index b >= g with t_b >= t (G if
    // none), for a t past t_{g-1}; tg holds t_g on a grid read from memory and moves to t_b
    // (it is ignored on a uniform grid).  On a uniform grid lo = 0, f = fl(t * scale) is
    // t D / T within a relative 5 ulp and t_g = fl(fl(T g) / D) is T g / D within 2 ulp, so
    // when f lies farther than 2^-40 (f + 1) from every integer, ceil(f) is b.  Only a t
    // that close to a grid point (or t = inf) takes the exact search, as a rare
    // wave-uniform branch.
    __device__ __forceinline__ int32_t bin_of(int32_t g, double t, double &tg) const {
        if (!uniform) return (g < G && t > tg) ? next_bin_impl<false>(g, t, tg) : g;
        const double f = (t - lo) * scale;
        const double gf = ceil(f);
        const double m = 0x1p-40 * (f + 1.0);
        const bool near = !(gf - f > m) || !(f - (gf - 1.0) > m);
        int32_t b = (int32_t)fmin(fmax(gf, (double)g), (double)G);   // in [g, G]: converts exactly
        if (__ballot(near)) {
            if (near) {
                double tu;
                b = (g < G && t > (T * (double)g) / D) ? next_bin_impl<true>(g, t, tu) : g;
            }
        }
        return b;
    }
};

// The event loop.  MM is the number of propensity slots the policy evaluates (>= M), or 0
// for networks too large to keep a_j and S_j in registers (forward only).
// Record and backward passes: lanes are refilled as soon as their trajectory ends, or, with
// GEN, only once every lane of the wave is idle (generations of 64 trajectories: for
// launches of about one wave per SIMD, where the longest trajectory sets the time anyway
// and the simpler loop runs each event faster).
template <int MODE, int MM, bool BATCH, class Policy, bool QUAD = false, bool GEN = false>
__device__ __forceinline__ void sim_loop(const WorkList &wl, Policy &p) {
    static_assert(MODE != kFwd && MM > 0, "record, backward and the event log need the per-reaction registers");
    constexpr int MR = MM > 0 ? MM : 1;
    const uint32_t lane = __lane_id();

    // wave-uniform work state
    int32_t cur = -1;
    int64_t pool_next = 0, pool_end = 0;
    int32_t pending = -1;
    bool exhausted = false;
    GridView gv;
    gv.grid = nullptr;
    gv.T = gv.D = gv.lo = gv.scale = 0.0;
    gv.G = 0;
    gv.uniform = 0;

    // lane state
    bool active = false;
    int64_t traj = 0;
    double t = 0.0;
    uint64_t k = 0, ev = 0;
    int32_t g = 0;
    double tg_cur = 0.0;       // backward: time of grid point g (the first one not yet passed)
    uint32_t ovf = 0;
    uint32_t flags = 0;
    unsigned long long tot_events = 0, max_steps = 0;
    uint64_t ev_start = 0;     // event log in epochs: events before this epoch
    bool gone = false;         // event log in epochs: the trajectory ended in an earlier epoch
    unsigned long long rec_count = 0;   // event log: this lane's records (added to the cursor at the end)
    LogSlots slots;             // event log: the wave's reserved slots
    int32_t step_nrec = 0;      // event log: this lane's records of the last step
    double a[MR];
    double Ssum[MR];
    // record: A_j and n_j; backward: the score B_j = n_j - A_j at the current event time
    // (updated by [j fired] - a_j tau per event) and the gradient accumulator
    double A[MODE == kRec ? MR : 1];
    int32_t nf[MODE == kRec ? MR : 1];
    double B[MODE == kBwd ? MR : 1];
    double gacc[MODE == kBwd ? MR : 1];

    for (;;) {
        // ---------------- refill idle lanes ----------------
        const uint64_t idle = __ballot(!active);
        // (once the work is exhausted, idle lanes cost nothing per event)
        if (GEN ? idle == ~0ull && !exhausted : idle && !(exhausted && pending < 0 && pool_next >= pool_end)) {
            if (pool_next >= pool_end && !exhausted && pending < 0) {
                int32_t item = 0;
                if (lane == 0) item = (int32_t)atomicAdd(wl.counter, 1u);
                item = wave_uniform(__shfl(item, 0));
                if (item >= wl.n_items) exhausted = true; else pending = item;
            }
            if (pending >= 0) {
                const int32_t b = BATCH ? wave_uniform(((const SSA_CONST int32_t *)wl.item_net)[pending]) : 0;
                if (b == cur || idle == ~0ull) {
                    if (BATCH) {
                        pool_next = ((const SSA_CONST int64_t *)wl.item_begin)[pending];
                        pool_end = pool_next + ((const SSA_CONST int32_t *)wl.item_count)[pending];
                    } else {
                        pool_next = wl.range_begin + (int64_t)pending * kChunk;
                        pool_end = min(pool_next + (int64_t)kChunk, wl.range_end);
                    }
                    pool_next = wave_uniform(pool_next);
                    pool_end = wave_uniform(pool_end);
                    pending = -1;
                    if (b != cur) {
                        // switch network: the policy's per-wave tables and the grid view
                        cur = b;
                        const NetDev nn = current_net<BATCH>(wl, cur);
                        p.switch_net(nn);
                        const GridInfo gi = *(const SSA_CONST GridInfo *)nn.ginfo;
                        gv.grid = wave_uniform(nn.grid);
                        gv.T = wave_uniform(gi.T);
                        gv.D = wave_uniform(gi.D);
                        gv.lo = wave_uniform(gi.lo);
                        gv.scale = wave_uniform(gi.scale);
                        gv.G = wave_uniform(nn.G);
                        gv.uniform = wave_uniform(gi.uniform);
                    }
                }
            }
            const int32_t n_idle = __popcll(idle);
            if (!active && pool_next < pool_end) {
                const int64_t mine = pool_next + __popcll(idle & lanemask_lt());
                if (mine < pool_end) {
                    const NetDev n = current_net<BATCH>(wl, cur);
                    active = true;
                    traj = (!BATCH && wl.perm) ? (int64_t)wl.perm[mine] : mine;
                    t = 0.0;
                    k = 0;
                    ev = 0;
                    g = 0;
                    tg_cur = gv.uniform ? 0.0 : ((const SSA_CONST double *)gv.grid)[0];
                    ovf = 0;
                    p.reset(n);
                    ev_start = 0;
                    if (MODE == kEvt && n.rs_t) {
                        t = n.rs_t[traj];
                        k = n.rs_k[traj];
                        ev = n.rs_ev[traj];
                        p.load_state(n.rs_x + (size_t)traj * n.S);
                        ev_start = ev;
                        if (t < 0.0) {            // ended in an earlier epoch
                            t = n.t_end;
                            gone = true;
                        }
                    }
                    if (MODE == kRec) {
#pragma unroll
                        for (int j = 0; j < MM; ++j) { A[j] = 0.0; nf[j] = 0; }
                    }
                    if (MODE == kBwd) {
#pragma unroll
                        for (int j = 0; j < MM; ++j) { B[j] = 0.0; gacc[j] = 0.0; }
                    }
                }
            }
            pool_next = min(pool_next + (int64_t)n_idle, pool_end);
        }
        if (MODE == kEvt && wl.net0.ev_key) {
            // the last step's records took slots; make sure this step's fit
            uint32_t used = 0;
#pragma unroll
            for (int q = 0; q < kChg; ++q) used += __popcll(__ballot(step_nrec > q));
            step_nrec = 0;
            slots.advance(used, __ballot(active) != 0, wl.net0.ev_resv, lane);
        }
        if (__ballot(active) == 0) {
            if (exhausted && pending < 0) break;
            continue;
        }
        if (!active) continue;

        // ---------------- one event of the direct method ----------------
        const NetDev n = current_net<BATCH>(wl, cur);
        const int32_t M = n.M;
        double acc;
        if constexpr (MM > 0) {
            p.template eval<MM>(n, a);
            acc = a[0];
            Ssum[0] = acc;
#pragma unroll
            for (int j = 1; j < MM; ++j) {
                acc = acc + a[j];          // S_j = S_{j-1} + a_j; padded slots add +0
                Ssum[j] = acc;
            }
        } else {
            acc = p.total(n);
        }
        // the draw (not consumed when the state is absorbing), computed without a branch so
        // that its chain interleaves with the propensities
        const u32x4 o = philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), (uint32_t)traj,
                                      (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
        const double En = neg_log(uniform_open0(o.v0, o.v1));
        const bool drawn = acc != 0.0;
        const double r2 = drawn ? uniform_open1(o.v2, o.v3) : 0.0;
        const double tau = drawn ? En / acc : __builtin_inf();
        k = drawn ? k + 1 : k;
        const double t_next = t + tau;
        // the count of partial sums <= u (the smallest j with S_j > u), taken now so the
        // partial sums are dead before the grid work below
        int32_t sel = 0;
        {
            const double u = r2 * acc;
#pragma unroll
            for (int j = 0; j < MM; ++j) sel += (Ssum[j] <= u) ? 1 : 0;
        }

        // grid points passed before the event: record / backward see the pre-event state
        if (MODE == kRec) {
            int32_t *row = n.rec_states + (size_t)(traj - n.rec_begin) * n.G * n.S;
            while (g < n.G && gv.at(g) < t_next) {
                p.for_each_species([&](int32_t s, int32_t xs) { row[(size_t)g * n.S + s] = xs; });
                ++g;
            }
        } else if (MODE == kBwd) {
            // all crossings of [t, t_next) share the state x and the score line
            // z_j(t_g) = (n_j - A_j) - a_j (t_g - t): fold them into
            //   alpha = sum_g phi_g,  beta = sum_g phi_g (t_g - t),  phi_g = sum_s w_gs (x_s - mhat_gs)
            // (two rows of the prefix table) and update the M accumulators once per interval.
            const int32_t gb = gv.bin_of(g, t_next, tg_cur);
            if (gb > g) {
                double alpha, beta;
                interval_sums<QUAD>(p, n.bp, n.bpt, n.S, g, gb, t, alpha, beta);
#pragma unroll
                for (int j = 0; j < MM; ++j) gacc[j] = gacc[j] + (B[j] * alpha - a[j] * beta);
                g = gb;
            }
        }

        bool finish = t_next > n.t_end;
        bool pause = false;
        if (MODE == kEvt && n.ws_t) {
            // epochs: an ended trajectory stays ended; an event beyond the epoch waits for the
            // next one, which redraws the same Philox block from the same state
            if (gone) {
                finish = true;
            } else if (!finish && t_next > n.t_pause) {
                finish = true;
                pause = true;
                if (acc != 0.0) k = k - 1;
            }
        }
        if (!finish && ev >= n.max_events) {
            flags |= kFlagEventLimit;
            finish = true;
        }
        if (!finish) {
            if (__ballot(sel >= M)) {
                // rare: rounding left no S_j > u; take the largest j with a_j > 0
                if (sel >= M) {
                    for (int32_t j = M - 1; j >= 0; --j) {
                        if (p.one(n, j) > 0.0) { sel = j; break; }
                    }
                    sel = min(sel, M - 1);   // a0 > 0 guarantees some a_j > 0; keeps the index in range
                }
            }
            // event log: the changed species of this event (at most kChg), kept in registers
            int32_t nrec = 0;
            int32_t rs[kChg], rd[kChg], rx[kChg];
            p.apply(n, sel, [&](int32_t sp, int32_t xo, int32_t xn) {
                ovf |= (uint32_t)xn;
                if (MODE == kEvt && xn != xo) {
#pragma unroll
                    for (int i = 0; i < kChg; ++i)
                        if (nrec == i) {
                            rs[i] = sp;
                            rd[i] = xn - xo;
                            rx[i] = xo;
                        }
                    ++nrec;
                }
            });
            if ((int32_t)ovf < 0) {
                flags |= kFlagOverflow;
                finish = true;
            } else {
                if (MODE == kRec) {
#pragma unroll
                    for (int j = 0; j < MM; ++j) {
                        A[j] = A[j] + a[j] * tau;
                        nf[j] += (j == sel) ? 1 : 0;
                    }
                }
                if (MODE == kBwd) {
#pragma unroll
                    for (int j = 0; j < MM; ++j) B[j] = B[j] + ((j == sel ? 1.0 : 0.0) - a[j] * tau);
                }
                if (MODE == kEvt) {
                    nrec = min(nrec, kChg);
                    rec_count += (unsigned long long)nrec;
                }
                if (MODE == kEvt && n.ev_key) {
                    // this step's records take consecutive slots of the wave's reservation
                    step_nrec = nrec;
                    uint32_t before = 0;
#pragma unroll
                    for (int i = 0; i < kChg; ++i) before += __popcll(__ballot(nrec > i) & lanemask_lt());
                    {
                        const unsigned long long key = (unsigned long long)__double_as_longlong(t_next);
#pragma unroll
                        for (int i = 0; i < kChg; ++i) {
                            if (i < nrec) {
                                const int64_t at = (int64_t)slots.at((unsigned long long)(before + i));
                                if (at < n.ev_cap) {
                                    n.ev_key[at] = key;
                                    n.ev_val[at] = ev_pack(rs[i], rd[i], rx[i]);
                                } else {
                                    flags |= kFlagRecordsFull;
                                }
                            }
                        }
                    }
                }
                t = t_next;
                ev = ev + 1;
            }
        }
        if (finish) {
            if (MODE == kRec) {
                const int64_t r = traj - n.rec_begin;
                n.rec_events[r] = ev;
                n.rec_draws[r] = k;
                n.rec_tlast[r] = t;
                if (n.rec_nf) {
#pragma unroll
                    for (int j = 0; j < MM; ++j)
                        if (j < M) n.rec_nf[r * M + j] = (int64_t)nf[j];
                }
                if (n.rec_aint) {
                    const double tail = n.t_end - t;
#pragma unroll
                    for (int j = 0; j < MM; ++j)
                        if (j < M) n.rec_aint[r * M + j] = A[j] + a[j] * tail;
                }
            }
            if (MODE == kBwd) {
#pragma unroll
                for (int j = 0; j < MM; ++j)
                    if (j < M) n.gtraj[(size_t)traj * M + j] = gacc[j];
            }
            if (MODE == kEvt && n.ws_t) {
                int32_t *wx = n.ws_x + (size_t)traj * n.S;
                p.for_each_species([&](int32_t s, int32_t xs) { wx[s] = xs; });
                n.ws_t[traj] = pause ? t : -1.0;
                n.ws_k[traj] = k;
                n.ws_ev[traj] = ev;
            }
            tot_events += ev - ev_start;
            max_steps = max(max_steps, (unsigned long long)ev);
            active = false;
            gone = false;
        }
    }

    // wave totals -> global statistics
    for (int off = 32; off > 0; off >>= 1) {
        tot_events += __shfl_xor(tot_events, off);
        max_steps = max(max_steps, (unsigned long long)__shfl_xor(max_steps, off));
        flags |= (uint32_t)__shfl_xor((int)flags, off);
        if (MODE == kEvt) rec_count += __shfl_xor(rec_count, off);
    }
    if (lane == 0) {
        if (tot_events) atomicAdd(wl.stats + 0, tot_events);
        atomicMax(wl.stats + 1, max_steps);
        if (flags) atomicOr(wl.stats + 2, (unsigned long long)flags);
        if (MODE == kEvt && rec_count) atomicAdd(wl.net0.ev_cursor, rec_count);
    }
}

// Backward and event log in generations with a second wave drawing the random numbers.  A
// block is two waves: wave 0 simulates a generation of up to 64 trajectories as
// sim_loop<kBwd> / sim_loop<kEvt> do, wave 1 computes the Philox blocks and variates
// (-ln r1, r2) of the next kPcRows steps of every lane into an LDS ring of two halves, one
// barrier per kPcRows steps.  In a generation every active lane applies one event per step,
// so step n consumes draw K0 + n of every lane (K0: 0, or the draw an epoch of the event
// log resumes at); the simulating wave's event chain loses the Philox rounds and the
// logarithm, which the other wave computes on its own SIMD.  For launches of about one block per CU,
// where the simulating waves run alone and their chains set the time.  ring: [2][2][kPcRows]
// [64] doubles (half, E / r2, step, lane); ctl: 3 ints.  Every decision that ends a loop
// around a barrier is read from LDS after a barrier, so both waves take the same path.
constexpr int kPcRows = 16;

template <int MODE, int MM, class Policy, bool QUAD = false>
__device__ __forceinline__ void sim_pc(const WorkList &wl, Policy &p, double *ring, int32_t *ctl) {
    static_assert(MODE == kBwd || MODE == kEvt, "backward or event log");
    const uint32_t lane = __lane_id();
    const bool drawer = __builtin_amdgcn_readfirstlane(threadIdx.x) >= (unsigned)kWave;   // wave-uniform
    const NetDev n = wl.net0;
    const int32_t M = n.M;
    const GridInfo gi = *(const SSA_CONST GridInfo *)n.ginfo;
    GridView gv;
    gv.grid = wave_uniform(n.grid);
    gv.T = wave_uniform(gi.T);
    gv.D = wave_uniform(gi.D);
    gv.lo = wave_uniform(gi.lo);
    gv.scale = wave_uniform(gi.scale);
    gv.G = wave_uniform(n.G);
    gv.uniform = wave_uniform(gi.uniform);
    if (!drawer) p.switch_net(n);
    uint32_t flags = 0;
    unsigned long long tot_events = 0, max_steps = 0;
    unsigned long long rec_count = 0;   // event log: this lane's records (added to the cursor at the end)
    LogSlots slots;             // event log: the wave's reserved slots
    int32_t step_nrec = 0;      // event log: this lane's records of the last step
    double a[MM], Ssum[MM], B[MM], gacc[MM];

    for (;;) {
        if (!drawer && lane == 0) ctl[0] = (int32_t)atomicAdd(wl.counter, 1u);
        __syncthreads();
        const int32_t item = ctl[0];
        if (item >= wl.n_items) break;
        const int64_t begin = wl.range_begin + (int64_t)item * kChunk;
        const int64_t count = min((int64_t)kChunk, wl.range_end - begin);
        const int64_t traj = begin + lane;
        const bool mine = (int64_t)lane < count;
        // event log in epochs: where this lane's trajectory resumes
        const bool resume = MODE == kEvt && n.rs_t != nullptr;
        const double t0 = mine && resume ? n.rs_t[traj] : 0.0;
        const uint64_t K0 = mine && resume ? n.rs_k[traj] : 0;

        // draws K0 + [row0, row0 + kPcRows) of this lane's trajectory into ring half h
        auto fill = [&](int32_t h, uint64_t row0) {
            if (!mine) return;
            double *e = ring + (size_t)(2 * h) * kPcRows * kWave + lane;
            double *r = e + kPcRows * kWave;
#pragma unroll 4
            for (int i = 0; i < kPcRows; ++i) {
                const uint64_t kk = K0 + row0 + (uint64_t)i;
                const u32x4 o = philox4x32_10((uint32_t)kk, (uint32_t)(kk >> 32), (uint32_t)traj,
                                              (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
                e[i * kWave] = neg_log(uniform_open0(o.v0, o.v1));
                r[i * kWave] = uniform_open1(o.v2, o.v3);
            }
        };
        if (drawer) fill(0, 0);

        // simulating lane state
        bool active = !drawer && mine;
        double t = 0.0, tg_cur = gv.uniform ? 0.0 : ((const SSA_CONST double *)gv.grid)[0];
        uint64_t ev = 0, ev_start = 0, k = K0;
        bool gone = false;
        int32_t g = 0;
        uint32_t ovf = 0;
        if (active) {
            p.reset(n);
            if (resume) {
                t = t0;
                ev = n.rs_ev[traj];
                ev_start = ev;
                p.load_state(n.rs_x + (size_t)traj * n.S);
                if (t < 0.0) {          // ended in an earlier epoch
                    t = n.t_end;
                    gone = true;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < MM; ++j) { B[j] = 0.0; gacc[j] = 0.0; }
        __syncthreads();

        for (int32_t c = 0;; ++c) {
            if (drawer) {
                fill((c + 1) & 1, (uint64_t)(c + 1) * kPcRows);
            } else {
                const double *Er = ring + (size_t)(2 * (c & 1)) * kPcRows * kWave + lane;
                const double *Rr = Er + kPcRows * kWave;
                for (int i = 0; i < kPcRows; ++i) {
                    if (MODE == kEvt && n.ev_key) {
                        // the last step's records took slots; make sure this step's fit
                        uint32_t used = 0;
#pragma unroll
                        for (int q = 0; q < kChg; ++q) used += __popcll(__ballot(step_nrec > q));
                        step_nrec = 0;
                        slots.advance(used, __ballot(active) != 0, n.ev_resv, lane);
                    }
                    if (__ballot(active) == 0) break;
                    if (!active) continue;
                    p.template eval<MM>(n, a);
                    double acc = a[0];
                    Ssum[0] = acc;
#pragma unroll
                    for (int j = 1; j < MM; ++j) {
                        acc = acc + a[j];
                        Ssum[j] = acc;
                    }
                    const bool drawn = acc != 0.0;
                    const double r2 = drawn ? Rr[i * kWave] : 0.0;
                    const double tau = drawn ? Er[i * kWave] / acc : __builtin_inf();
                    const double t_next = t + tau;
                    int32_t sel = 0;
                    {
                        const double u = r2 * acc;
#pragma unroll
                        for (int j = 0; j < MM; ++j) sel += (Ssum[j] <= u) ? 1 : 0;
                    }
                    k = drawn ? k + 1 : k;
                    if (MODE == kBwd) {
                        const int32_t gb = gv.bin_of(g, t_next, tg_cur);
                        if (gb > g) {
                            double alpha, beta;
                            interval_sums<QUAD>(p, n.bp, n.bpt, n.S, g, gb, t, alpha, beta);
#pragma unroll
                            for (int j = 0; j < MM; ++j) gacc[j] = gacc[j] + (B[j] * alpha - a[j] * beta);
                            g = gb;
                        }
                    }
                    bool finish = t_next > n.t_end;
                    bool pause = false;
                    if (MODE == kEvt && n.ws_t) {
                        // an ended trajectory stays ended; an event beyond the epoch waits for
                        // the next one, which redraws the same draw from the same state
                        if (gone) {
                            finish = true;
                        } else if (!finish && t_next > n.t_pause) {
                            finish = true;
                            pause = true;
                            if (drawn) k = k - 1;
                        }
                    }
                    if (!finish && ev >= n.max_events) {
                        flags |= kFlagEventLimit;
                        finish = true;
                    }
                    if (!finish) {
                        if (__ballot(sel >= M)) {
                            if (sel >= M) {
                                for (int32_t j = M - 1; j >= 0; --j) {
                                    if (p.one(n, j) > 0.0) { sel = j; break; }
                                }
                                sel = min(sel, M - 1);
                            }
                        }
                        int32_t nrec = 0;
                        int32_t rs[kChg], rd[kChg], rx[kChg];
                        p.apply(n, sel, [&](int32_t sp, int32_t xo, int32_t xn) {
                            ovf |= (uint32_t)xn;
                            if (MODE == kEvt && xn != xo) {
#pragma unroll
                                for (int q = 0; q < kChg; ++q)
                                    if (nrec == q) {
                                        rs[q] = sp;
                                        rd[q] = xn - xo;
                                        rx[q] = xo;
                                    }
                                ++nrec;
                            }
                        });
                        if ((int32_t)ovf < 0) {
                            flags |= kFlagOverflow;
                            finish = true;
                        } else {
                            if (MODE == kBwd) {
#pragma unroll
                                for (int j = 0; j < MM; ++j) B[j] = B[j] + ((j == sel ? 1.0 : 0.0) - a[j] * tau);
                            }
                            if (MODE == kEvt) {
                                nrec = min(nrec, kChg);
                                rec_count += (unsigned long long)nrec;
                            }
                            if (MODE == kEvt && n.ev_key) {
                                // this step's records take consecutive slots of the wave's reservation
                                step_nrec = nrec;
                                uint32_t before = 0;
#pragma unroll
                                for (int q = 0; q < kChg; ++q) before += __popcll(__ballot(nrec > q) & lanemask_lt());
                                {
                                    const unsigned long long key = (unsigned long long)__double_as_longlong(t_next);
#pragma unroll
                                    for (int q = 0; q < kChg; ++q) {
                                        if (q < nrec) {
                                            const int64_t at = (int64_t)slots.at((unsigned long long)(before + q));
                                            if (at < n.ev_cap) {
                                                n.ev_key[at] = key;
                                                n.ev_val[at] = ev_pack(rs[q], rd[q], rx[q]);
                                            } else {
                                                flags |= kFlagRecordsFull;
                                            }
                                        }
                                    }
                                }
                            }
                            t = t_next;
                            ev = ev + 1;
                        }
                    }
                    if (finish) {
                        if (MODE == kBwd) {
#pragma unroll
                            for (int j = 0; j < MM; ++j)
                                if (j < M) n.gtraj[(size_t)traj * M + j] = gacc[j];
                        }
                        if (MODE == kEvt && n.ws_t) {
                            int32_t *wx = n.ws_x + (size_t)traj * n.S;
                            p.for_each_species([&](int32_t sp, int32_t xs) { wx[sp] = xs; });
                            n.ws_t[traj] = pause ? t : -1.0;
                            n.ws_k[traj] = k;
                            n.ws_ev[traj] = ev;
                        }
                        tot_events += ev - ev_start;
                        max_steps = max(max_steps, (unsigned long long)ev);
                        active = false;
                    }
                }
                const bool none = __ballot(active) == 0;
                if (lane == 0) ctl[1 + (c & 1)] = none ? 1 : 0;
            }
            __syncthreads();
            if (ctl[1 + (c & 1)]) break;
        }
    }

    if (!drawer) {
        for (int off = 32; off > 0; off >>= 1) {
            tot_events += __shfl_xor(tot_events, off);
            max_steps = max(max_steps, (unsigned long long)__shfl_xor(max_steps, off));
            flags |= (uint32_t)__shfl_xor((int)flags, off);
            if (MODE == kEvt) rec_count += __shfl_xor(rec_count, off);
        }
        if (lane == 0) {
            if (tot_events) atomicAdd(wl.stats + 0, tot_events);
            atomicMax(wl.stats + 1, max_steps);
            if (flags) atomicOr(wl.stats + 2, (unsigned long long)flags);
            if (MODE == kEvt && rec_count) atomicAdd(wl.net0.ev_cursor, rec_count);
        }
    }
}

// LDS stride, in 8-byte words, of a window row of row_words words: odd, so that the rows of
// the bins a wave's lanes are in start on different LDS banks (an even stride such as the
// 8 words of four species maps every bin to one of a few banks, and lanes in different
// bins then conflict).
__host__ __device__ __forceinline__ int32_t win_stride(int32_t row_words) { return row_words | 1; }

// Smallest value over the wave's lanes (uniform result).
__device__ __forceinline__ int32_t wave_min(int32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    return wave_uniform(v);
}

// Forward pass by generations (see the header comment): a wave takes one work item, runs
// its (up to) 64 trajectories to the end with one window that follows the slowest lane,
// then takes the next item.  The loop is tighter than the cohort form below, which pays
// off for networks compiled into registers.  win: the wave's LDS window, wl.win_bins rows
// of S species x (sum nu, sum (2x+nu)nu) as int64, at a stride of win_stride(2S) words.  HIST: with the per-grid-point histogram
// (a separate instantiation, so runs without one carry none of its code).  COV: also the
// difference sums of the cross products x_s x_r for the species covariance matrix.
//
// PC: blocks of two waves, the second computing the draws (see sim_pc) into an LDS ring
// of 2 kPcRows draws per lane, indexed by draw number mod 2 kPcRows.  A lane whose next
// event lies beyond the window does not draw, so lanes consume draws at their own pace: at
// the barrier that ends each kPcRows steps the simulating wave publishes each lane's next
// draw number K (kl, two halves by chunk parity), and during the next steps the drawing
// wave fills draws up to K + 2 kPcRows.  A lane consumes at most one draw per step, so the
// draws it needs before the next barrier, [K, K + kPcRows), are in the ring, and the slots
// being refilled hold draws below K, already consumed.
// EPOCH: one epoch of a run in epochs of simulation time (resume from n.rs_*, unless NULL,
// pause before the first event beyond n.t_pause and save into n.ws_*); a template flag so
// that the other launches carry none of it.  With PC the drawing wave starts each lane at
// its saved draw number K0 (draws are indexed absolutely, so the ring and the published
// numbers work unchanged).
template <int MM, bool BATCH, bool SLAB, bool HIST, class Policy, bool COV = false, bool PC = false,
          bool EPOCH = false>
__device__ __forceinline__ void sim_fwd_gen(const WorkList &wl, Policy &p, long long *win, double *ring = nullptr,
                                            unsigned long long *kl = nullptr, int32_t *ctl = nullptr) {
    static_assert(!PC || (!BATCH && !SLAB), "the drawing wave serves single-network atomic-flush launches");
    static_assert(!EPOCH || (!BATCH && !SLAB && !COV), "epochs run single-network atomic-flush launches");
    constexpr int MR = MM > 0 ? MM : 1;
    constexpr uint64_t kRing = 2 * kPcRows;
    const uint32_t lane = __lane_id();
    // wave-uniform (a scalar value): the two roles are separate code paths, each with its
    // own barriers, which must not be compiled as one masked path for both waves
    const bool drawer = PC && __builtin_amdgcn_readfirstlane(threadIdx.x) >= (unsigned)kWave;
    const int32_t W = wl.win_bins;
    const int32_t wave_slot = (int32_t)(blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave);

    int32_t cur = -1;
    GridView gv;
    gv.grid = nullptr;
    gv.T = gv.D = gv.lo = gv.scale = 0.0;
    gv.G = 0;
    gv.uniform = 0;
    uint32_t flags = 0;
    unsigned long long tot_events = 0, max_steps = 0;
    double a[MR];
    double Ssum[MR];

    for (;;) {
        // ---------------- next generation: one work item, one trajectory per lane ----------------
        int32_t item = 0;
        if constexpr (PC) {
            if (!drawer && lane == 0) ctl[0] = (int32_t)atomicAdd(wl.counter, 1u);
            __syncthreads();
            item = ctl[0];
        } else {
            if (lane == 0) item = (int32_t)atomicAdd(wl.counter, 1u);
            item = wave_uniform(__shfl(item, 0));
        }
        if (item >= wl.n_items) break;
        int32_t b = 0;
        int64_t begin, count;
        if (BATCH) {
            b = wave_uniform(((const SSA_CONST int32_t *)wl.item_net)[item]);
            begin = wave_uniform(((const SSA_CONST int64_t *)wl.item_begin)[item]);
            count = wave_uniform((int64_t)((const SSA_CONST int32_t *)wl.item_count)[item]);
        } else {
            begin = wl.range_begin + (int64_t)item * kChunk;
            count = min((int64_t)kChunk, wl.range_end - begin);
        }
        if (b != cur) {
            cur = b;
            const NetDev nn = current_net<BATCH>(wl, cur);
            p.switch_net(nn);
            const GridInfo gi = *(const SSA_CONST GridInfo *)nn.ginfo;
            gv.grid = wave_uniform(nn.grid);
            gv.T = wave_uniform(gi.T);
            gv.D = wave_uniform(gi.D);
            gv.lo = wave_uniform(gi.lo);
            gv.scale = wave_uniform(gi.scale);
            gv.G = wave_uniform(nn.G);
            gv.uniform = wave_uniform(gi.uniform);
        }
        const NetDev n0 = current_net<BATCH>(wl, cur);
        const int32_t S = n0.S, G = n0.G, M = n0.M;
        if constexpr (PC) {
            if (drawer) {
                // the drawing wave: draws [F, K + 2 kPcRows) of each lane's trajectory
                const int64_t dtraj = begin + lane;
                // an epoch resumes each trajectory at the draw it did not use (one that ended
                // in an earlier epoch draws nothing)
                const bool ended = EPOCH && (int64_t)lane < count && n0.rs_t && n0.rs_t[dtraj] < 0.0;
                const bool mine = (int64_t)lane < count && !ended;
                uint64_t F = (EPOCH && mine && n0.rs_t) ? n0.rs_k[dtraj] : 0;
                const uint64_t K0 = F;
                auto fill_to = [&](uint64_t upto) {
                    if (!mine) return;
                    for (; F < upto; ++F) {
                        const u32x4 o = philox4x32_10((uint32_t)F, (uint32_t)(F >> 32), (uint32_t)dtraj,
                                                      (uint32_t)((uint64_t)dtraj >> 32), n0.key0, n0.key1);
                        const uint32_t slot = (uint32_t)(F & (kRing - 1));
                        ring[slot * kWave + lane] = neg_log(uniform_open0(o.v0, o.v1));
                        ring[(kRing + slot) * kWave + lane] = uniform_open1(o.v2, o.v3);
                    }
                };
                fill_to(K0 + kRing);
                __syncthreads();
                for (int32_t c = 0;; ++c) {
                    // draw K0 is taken before the first step, so the first steps start at K0 + 1
                    const uint64_t K = c == 0 ? K0 + 1 : kl[((c - 1) & 1) * kWave + lane];
                    fill_to(K + kRing);
                    __syncthreads();
                    if (ctl[1 + (c & 1)]) break;
                }
                continue;
            }
        }
        // window / D row per bin: (sum nu, sum of low parts of (2x+nu)nu) per species, then
        // with COV the low parts of the cross products x_s x_r (s < r); Dhi rows hold the
        // matching high parts
        const int32_t npairs = COV ? S * (S - 1) / 2 : 0;
        const int32_t row_words = S * 2 + npairs;
        const int32_t wstride = win_stride(row_words);
        const int32_t hi_words = S + npairs;
        unsigned long long *slab =
            SLAB ? wl.slabs + (size_t)wave_slot * (size_t)G * row_words : n0.D;
        for (int32_t q = lane; q < W * wstride; q += kWave) win[q] = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        int32_t base = 0;

        // flush bins [lo, hi) of the window (lanes cooperate over consecutive words)
        auto flush = [&](int32_t lo, int32_t hi) {
            // the window's LDS words were written by other lanes of this wave: LDS operations
            // of one wave complete in order, so only compiler reordering must be fenced off
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int32_t words = (hi - lo) * row_words;
            for (int32_t e = lane; e < words; e += kWave) {
                const int32_t bin = lo + e / row_words, r = e - (e / row_words) * row_words;
                long long *slot = win + (bin & (W - 1)) * wstride + r;
                const long long v = *slot;
                if (v != 0) {
                    unsigned long long *dst = slab + (size_t)bin * row_words + r;
                    if (SLAB) *dst = *dst + (unsigned long long)v;
                    else atomicAdd(dst, (unsigned long long)v);
                    *slot = 0;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };

        // lane state; every active lane holds a drawn event at t_next (bin binp) to apply
        bool active = (int64_t)lane < count;
        // a single-network forward in generations may take its positions in an order of
        // recorded lengths (a permutation: the sums are exact integers, so order changes no bit)
        const int64_t traj = (!BATCH && !PC && !EPOCH && wl.perm && active) ? (int64_t)wl.perm[begin + lane]
                                                                            : begin + lane;
        double t = 0.0, t_next = 0.0, u = 0.0;
        double tg_next = gv.uniform ? 0.0 : ((const SSA_CONST double *)gv.grid)[0];
        uint64_t k = 0, ev = 0, ev_start = 0;
        int32_t g = 0, binp = G;
        uint32_t ovf = 0;
        if (active) p.reset(n0);
        // a run in epochs of simulation time resumes every trajectory from its saved state
        // (its next draw is the Philox block it did not use; the window follows its lanes
        // from wherever they are)
        if (EPOCH && active && n0.rs_t) {
            const double ts = n0.rs_t[traj];
            ev = ev_start = n0.rs_ev[traj];
            if (ts < 0.0) {
                // ended in an earlier epoch: it stays ended in this epoch's saved states too
                // (the two state buffers alternate from epoch to epoch)
                active = false;
                n0.ws_t[traj] = -1.0;
                n0.ws_ev[traj] = ev;
            } else {
                t = ts;
                k = n0.rs_k[traj];
                p.load_state(n0.rs_x + (size_t)traj * S);
            }
        }

        // draw the event after t from the exponential variate En and the uniform r2n; a lane
        // whose state is absorbing, whose event lies beyond t_end or that reached the event
        // limit ends here (predicated, no branches but the grid search)
        auto draw = [&](const NetDev &n, double En, double r2n) {
            double acc;
            if constexpr (MM > 0) {
                p.template eval<MM>(n, a);
                acc = a[0];
                Ssum[0] = acc;
#pragma unroll
                for (int j = 1; j < MM; ++j) {
                    acc = acc + a[j];
                    Ssum[j] = acc;
                }
            } else {
                acc = p.total(n);
            }
            const bool absorb = acc == 0.0;                 // no draw: the state holds to t_end
            t_next = t + En / acc;
            const bool beyond = !absorb && t_next > n.t_end; // drawn, not applied
            // epochs: an event beyond the epoch's end waits for the next epoch
            const bool pause = EPOCH && !absorb && !beyond && t_next > n.t_pause;
            const bool limit = !absorb && !beyond && !pause && ev >= n.max_events;
            k = absorb ? k : k + 1;
            flags |= limit ? (uint32_t)kFlagEventLimit : 0u;
            u = r2n * acc;
            const bool go = !(absorb || beyond || limit || pause);
            tot_events += go ? 0ull : (unsigned long long)(ev - ev_start);
            max_steps = go ? max_steps : max(max_steps, (unsigned long long)ev);
            if (EPOCH && !go) {
                // save the state for the next epoch: time -1 once the trajectory has ended;
                // a paused lane redraws the block of the event it did not apply
                int32_t *wx = n.ws_x + (size_t)traj * S;
                p.for_each_species([&](int32_t s2, int32_t xs) { wx[s2] = xs; });
                n.ws_t[traj] = pause ? t : -1.0;
                n.ws_k[traj] = pause ? k - 1 : k;
                n.ws_ev[traj] = ev;
            }
            active = go;
        };
        // the grid bin of the drawn event
        auto place = [&]() {
            const int32_t bq = gv.bin_of(g, t_next, tg_next);
            binp = active ? bq : g;
        };
        // the variates of draw kk (they do not depend on the state)
        double E_pre = 0.0, r2_pre = 0.0;
        auto prepare = [&](const NetDev &n, uint64_t kk) {
            const u32x4 o = philox4x32_10((uint32_t)kk, (uint32_t)(kk >> 32), (uint32_t)traj,
                                          (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
            r2_pre = uniform_open1(o.v2, o.v3);
            E_pre = neg_log(uniform_open0(o.v0, o.v1));
        };
        if (active) {
            const NetDev n = current_net<BATCH>(wl, cur);
            prepare(n, k);
            draw(n, E_pre, r2_pre);
            place();
            if (!PC) prepare(n, k);
        }
        if (PC) __syncthreads();    // the drawing wave has filled the ring

        for (int32_t c = 0, step = 0;;) {
            const bool blocked = active && binp < G && binp >= base + W;
            if (active && !blocked) {
                const NetDev n = current_net<BATCH>(wl, cur);
                // the variates of draw k: from the ring, or prepared one event ahead
                const uint32_t slot = (uint32_t)(k & (kRing - 1));
                const double r2n = PC ? ring[(kRing + slot) * kWave + lane] : r2_pre;
                const double En = PC ? ring[slot * kWave + lane] : E_pre;
                const uint64_t k_after = k + 1;
                // apply the pending event at t_next (state unchanged since it was drawn)
                int32_t sel = 0;
                if constexpr (MM > 0) {
#pragma unroll
                    for (int j = 0; j < MM; ++j) sel += (Ssum[j] <= u) ? 1 : 0;
                } else {
                    sel = p.select(n, u);
                }
                if (__ballot(sel >= M)) {          // rare: rounding left no S_j > u
                    if (sel >= M) {
                        for (int32_t j = M - 1; j >= 0; --j) {
                            if (p.one(n, j) > 0.0) { sel = j; break; }
                        }
                        sel = min(sel, M - 1);
                    }
                }
                const int32_t bin = binp;
                const bool inb = bin < G;
                long long *wrow = win + (bin & (W - 1)) * wstride;
                bool big = false;
                int32_t h_old = 0, h_new = 0;       // HIST: the histogram species before and after
                p.apply(n, sel, [&](int32_t sp, int32_t xo, int32_t xn) {
                    // events past the last grid point add zeros
                    ovf |= (uint32_t)xn;
                    const int32_t dl = inb ? xn - xo : 0;
                    // (2x + nu) nu as a 24-bit product when x < 2^19 and |nu| < 16 (its
                    // magnitude then stays below 2^24); any other change goes whole through
                    // the rare path below (low 24 bits to the window, the rest to Dhi)
                    const bool small = (uint32_t)xo < (1u << 19) && (uint32_t)(dl + 15) < 31u;
                    const int32_t d2 = small ? __mul24(2 * xo + dl, dl) : 0;
                    big = big || !small;
                    long long *w = wrow + sp * 2;
                    atomicAdd((unsigned long long *)w, (unsigned long long)(long long)dl);
                    atomicAdd((unsigned long long *)(w + 1), (unsigned long long)(long long)d2);
                    if (COV) {
                        // x_s x_r changes by dl x_r (the other species at their current
                        // values: applied one species at a time, the changes telescope)
                        p.for_each_species([&](int32_t r, int32_t xr) {
                            if (r == sp) return;
                            const int32_t lo_s = min(sp, r), hi_s = max(sp, r);
                            const int32_t pair = lo_s * (2 * S - lo_s - 1) / 2 + (hi_s - lo_s - 1);
                            const long long c = (long long)dl * (long long)xr;
                            const bool csmall = c > -kSmallD2 && c < kSmallD2;
                            atomicAdd((unsigned long long *)(wrow + 2 * S + pair),
                                      (unsigned long long)(csmall ? c : (c & ((1ll << 24) - 1))));
                            if (__ballot(!csmall)) {
                                if (!csmall)
                                    atomicAdd(n.Dhi + (size_t)bin * hi_words + S + pair, (unsigned long long)(c >> 24));
                            }
                        });
                    }
                    if (HIST) {
                        const bool h = sp == n.h_species;       // wave-uniform
                        h_old = h ? xo : h_old;
                        h_new = h ? xn : h_new;
                    }
                });
                if (HIST && inb && h_old != h_new) {
                    // unit-width bins (a wave-uniform test) need no division
                    const int32_t lo = n.h_lo, top = n.nb_hist - 1;
                    const int32_t bo = h_old < lo ? 0 : min(n.h_width == 1 ? h_old - lo : (h_old - lo) / n.h_width, top);
                    const int32_t bn = h_new < lo ? 0 : min(n.h_width == 1 ? h_new - lo : (h_new - lo) / n.h_width, top);
                    if (bo != bn) {
                        atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bo, -1);
                        atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bn, 1);
                    }
                }
                if (__ballot(big)) {                    // rare: a count of 2^19 or more, or |nu| >= 16
                    if (big) {
                        p.replay(n, sel, [&](int32_t sp, int32_t xo, int32_t xn) {
                            const int32_t dl = inb ? xn - xo : 0;
                            if (!((uint32_t)xo < (1u << 19) && (uint32_t)(dl + 15) < 31u)) {
                                const long long d2 = (2ll * xo + dl) * (long long)dl;
                                atomicAdd((unsigned long long *)(wrow + sp * 2 + 1),
                                          (unsigned long long)(d2 & ((1ll << 24) - 1)));
                                atomicAdd(n.Dhi + (size_t)bin * hi_words + sp, (unsigned long long)(d2 >> 24));
                            }
                        });
                    }
                }
                // a count that left the int32 range ends the lane with an error
                const bool bad = (int32_t)ovf < 0;
                flags |= bad ? (uint32_t)kFlagOverflow : 0u;
                t = t_next;
                ev = ev + 1;
                g = bin;
                draw(n, En, r2n);
                if (!PC) {
                    // the next variates (unused when the state turned absorbing), computed here
                    // so that their chain overlaps the propensities and the division above
                    prepare(n, k_after);
                    asm volatile("" : "+v"(E_pre), "+v"(r2_pre));
                }
                place();
                if (EPOCH && bad) n.ws_t[traj] = -1.0;      // an overflow ends the trajectory
                active = active && !bad;
            }
            // window upkeep: slide when a lane is waiting beyond it
            const bool none = __ballot(active) == 0;
            if (!PC && none) break;
            if (!none && __ballot(active && binp < G && binp >= base + W)) {
                const int32_t m = wave_min(active ? binp : G);
                if (m > base) {
                    flush(base, min(m, base + W));
                    base = m;
                }
            }
            if (PC && (++step == kPcRows || none)) {
                // chunk boundary (or no lane left: the drawing wave leaves at this one):
                // publish each lane's next draw, then both waves meet
                kl[(c & 1) * kWave + lane] = k;
                if (lane == 0) ctl[1 + (c & 1)] = none ? 1 : 0;
                __syncthreads();
                if (ctl[1 + (c & 1)]) break;
                ++c;
                step = 0;
            }
        }
        flush(base, min(G, base + W));
        if (!BATCH && !PC && n0.len_out && (int64_t)lane < count)
            n0.len_out[traj] = (uint32_t)min(ev, (uint64_t)0xffffffffu);
    }

    // wave totals -> global statistics
    for (int off = 32; off > 0; off >>= 1) {
        tot_events += __shfl_xor(tot_events, off);
        max_steps = max(max_steps, (unsigned long long)__shfl_xor(max_steps, off));
        flags |= (uint32_t)__shfl_xor((int)flags, off);
    }
    if (lane == 0) {
        if (tot_events) atomicAdd(wl.stats + 0, tot_events);
        atomicMax(wl.stats + 1, max_steps);
        if (flags) atomicOr(wl.stats + 2, (unsigned long long)flags);
    }
}

// Forward pass that also accumulates the likelihood-ratio Jacobian of the grid means
// (single network, specialised kernels).  At every grid crossing t_g of a trajectory the
// score z_j(t_g) = B_j - a_j (t_g - t) (B_j = n_j - A_j at the interval start t, a_j the
// interval's propensities) contributes x_s z_j to F[g][s][j] and z_j to Z[g][j]; the
// Jacobian is J = F/N - mean Z/N (the centred estimator).  The crossings of an interval
// [t, t_next) are the grid points [g, bin of t_next); they are added to a second LDS window
// (jwin, win_bins bins x (S+1) x M doubles) when they fall inside it: a lane whose next
// write lies beyond the window waits, and an interval longer than the window is added in
// pieces as the window slides.  Every trajectory crosses every grid point, so each bin of
// the window is complete when it is flushed and is stored (not added) into the work
// item's own slab; a fixed-order reduction over the items then makes the Jacobian
// independent of scheduling.
template <int MM, class Policy>
__device__ __forceinline__ void sim_fwd_jac(const WorkList &wl, Policy &p, long long *win, double *jwin) {
    static_assert(MM > 0, "the Jacobian needs the per-reaction registers");
    const uint32_t lane = __lane_id();
    const int32_t W = wl.win_bins;
    const NetDev n = wl.net0;
    const int32_t S = n.S, G = n.G, M = n.M;
    const int32_t row_words = S * 2;
    const int32_t jrow = (S + 1) * M;
    const GridInfo gi = *(const SSA_CONST GridInfo *)n.ginfo;
    GridView gv;
    gv.grid = wave_uniform(n.grid);
    gv.T = wave_uniform(gi.T);
    gv.D = wave_uniform(gi.D);
    gv.lo = wave_uniform(gi.lo);
    gv.scale = wave_uniform(gi.scale);
    gv.G = wave_uniform(G);
    gv.uniform = wave_uniform(gi.uniform);
    uint32_t flags = 0;
    unsigned long long tot_events = 0, max_steps = 0;
    double a[MM], Ssum[MM], B[MM];
    p.switch_net(n);

    for (;;) {
        int32_t item = 0;
        if (lane == 0) item = (int32_t)atomicAdd(wl.counter, 1u);
        item = wave_uniform(__shfl(item, 0));
        if (item >= wl.n_items) break;
        const int64_t begin = wl.range_begin + (int64_t)item * kChunk;
        const int64_t count = min((int64_t)kChunk, wl.range_end - begin);
        double *jslab = wl.jac_slabs + (size_t)item * G * jrow;
        for (int32_t q = lane; q < W * row_words; q += kWave) win[q] = 0;
        for (int32_t q = lane; q < W * jrow; q += kWave) jwin[q] = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        int32_t base = 0;

        // flush bins [lo, hi): moments by atomic adds of the non-zero words, the Jacobian
        // window by plain stores into the item's slab
        auto flush = [&](int32_t lo, int32_t hi) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int32_t words = (hi - lo) * row_words;
            for (int32_t e = lane; e < words; e += kWave) {
                const int32_t bin = lo + e / row_words, r = e - (e / row_words) * row_words;
                long long *slot = win + (bin & (W - 1)) * row_words + r;
                const long long v = *slot;
                if (v != 0) {
                    atomicAdd(n.D + (size_t)bin * row_words + r, (unsigned long long)v);
                    *slot = 0;
                }
            }
            const int32_t jwords = (hi - lo) * jrow;
            for (int32_t e = lane; e < jwords; e += kWave) {
                const int32_t bin = lo + e / jrow, r = e - (e / jrow) * jrow;
                double *slot = jwin + (bin & (W - 1)) * jrow + r;
                jslab[(size_t)bin * jrow + r] = *slot;
                *slot = 0.0;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };

        // lane state: the pending interval [t, t_next) with crossings [gj, binp); fin marks
        // the last interval (no event at its end)
        bool active = (int64_t)lane < count;
        const int64_t traj = begin + lane;
        double t = 0.0, t_next = 0.0, u = 0.0, tau = 0.0;
        double tg_next = gv.uniform ? 0.0 : ((const SSA_CONST double *)gv.grid)[0];
        uint64_t k = 0, ev = 0;
        int32_t g = 0, gj = 0, binp = G;
        bool fin = false;
        uint32_t ovf = 0;
        if (active) p.reset(n);
#pragma unroll
        for (int j = 0; j < MM; ++j) B[j] = 0.0;

        // draw the event after t (sets t_next, binp and the crossings [g, binp), or a final
        // interval when the event lies beyond t_end or the state is absorbing)
        auto draw = [&]() {
            const u32x4 o = philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), (uint32_t)traj,
                                          (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
            const double r2 = uniform_open1(o.v2, o.v3);
            const double E = neg_log(uniform_open0(o.v0, o.v1));
            p.template eval<MM>(n, a);
            double acc = a[0];
            Ssum[0] = acc;
#pragma unroll
            for (int j = 1; j < MM; ++j) {
                acc = acc + a[j];
                Ssum[j] = acc;
            }
            tau = E / acc;
            t_next = t + tau;
            gj = g;
            if (acc == 0.0 || t_next > n.t_end) {
                if (acc != 0.0) k = k + 1;
                fin = true;                        // crossings [g, G), no event
                binp = G;
                return;
            }
            k = k + 1;
            if (ev >= n.max_events) {
                flags |= kFlagEventLimit;
                fin = true;
                binp = G;
                return;
            }
            u = r2 * acc;
            binp = g;
            if (g < G && t_next > tg_next) binp = gv.next_bin(g, t_next, tg_next);
        };
        if (active) draw();

        for (;;) {
            // next write position: a crossing still to add, else the event's bin
            const int32_t pnext = gj < binp ? gj : (fin ? G : binp);
            const bool blocked = active && pnext < G && pnext >= base + W;
            if (active && !blocked) {
                // crossings inside the window
                const int32_t hi = min(binp, base + W);
                for (int32_t gg = gj; gg < hi; ++gg) {
                    const double dt = gv.at(gg) - t;
                    double z[MM];
#pragma unroll
                    for (int j = 0; j < MM; ++j) z[j] = B[j] - a[j] * dt;
                    double *jr = jwin + (gg & (W - 1)) * jrow;
                    p.for_each_species([&](int32_t sp, int32_t xs) {
                        const double xd = (double)xs;
#pragma unroll
                        for (int j = 0; j < MM; ++j)
                            if (j < M) atomicAdd(jr + sp * M + j, xd * z[j]);
                    });
#pragma unroll
                    for (int j = 0; j < MM; ++j)
                        if (j < M) atomicAdd(jr + S * M + j, z[j]);
                }
                gj = max(gj, hi);
                if (gj >= binp) {
                    if (fin) {
                        active = false;
                    } else if (binp >= G || binp < base + W) {
                        // apply the event at t_next
                        int32_t sel = 0;
#pragma unroll
                        for (int j = 0; j < MM; ++j) sel += (Ssum[j] <= u) ? 1 : 0;
                        if (sel >= M) {
                            for (int32_t j = M - 1; j >= 0; --j) {
                                if (p.one(n, j) > 0.0) { sel = j; break; }
                            }
                            sel = min(sel, M - 1);
                        }
                        const int32_t bin = binp;
                        const bool inb = bin < G;
                        long long *wrow = win + (bin & (W - 1)) * row_words;
                        p.apply(n, sel, [&](int32_t sp, int32_t xo, int32_t xn) {
                            ovf |= (uint32_t)xn;
                            const int32_t dl = inb ? xn - xo : 0;
                            const long long d2 = (2ll * xo + dl) * (long long)dl;
                            long long *w = wrow + sp * 2;
                            atomicAdd((unsigned long long *)w, (unsigned long long)(long long)dl);
                            if (d2 > -kSmallD2 && d2 < kSmallD2) {
                                atomicAdd((unsigned long long *)(w + 1), (unsigned long long)d2);
                            } else {
                                atomicAdd((unsigned long long *)(w + 1), (unsigned long long)(d2 & ((1ll << 24) - 1)));
                                atomicAdd(n.Dhi + (size_t)bin * S + sp, (unsigned long long)(d2 >> 24));
                            }
                            if (n.Hd && sp == n.h_species && dl != 0) {
                                const int32_t bo = xo < n.h_lo ? 0 : min((xo - n.h_lo) / n.h_width, n.nb_hist - 1);
                                const int32_t bn = xn < n.h_lo ? 0 : min((xn - n.h_lo) / n.h_width, n.nb_hist - 1);
                                if (bo != bn) {
                                    atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bo, -1);
                                    atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bn, 1);
                                }
                            }
                        });
                        if ((int32_t)ovf < 0) {
                            flags |= kFlagOverflow;
                            active = false;
                        } else {
                            // the score moves by [j fired] - a_j tau over the interval
#pragma unroll
                            for (int j = 0; j < MM; ++j) B[j] = B[j] + ((j == sel ? 1.0 : 0.0) - a[j] * tau);
                            t = t_next;
                            ev = ev + 1;
                            g = bin;
                            draw();
                        }
                    }
                }
                if (!active) {
                    tot_events += ev;
                    max_steps = max(max_steps, (unsigned long long)ev);
                }
            }
            if (__ballot(active) == 0) break;
            const int32_t pn = gj < binp ? gj : (fin ? G : binp);
            if (__ballot(active && pn < G && pn >= base + W)) {
                const int32_t m = wave_min(active ? pn : G);
                if (m > base) {
                    flush(base, min(m, base + W));
                    base = m;
                }
            }
        }
        flush(base, min(G, base + W));
    }

    for (int off = 32; off > 0; off >>= 1) {
        tot_events += __shfl_xor(tot_events, off);
        max_steps = max(max_steps, (unsigned long long)__shfl_xor(max_steps, off));
        flags |= (uint32_t)__shfl_xor((int)flags, off);
    }
    if (lane == 0) {
        if (tot_events) atomicAdd(wl.stats + 0, tot_events);
        atomicMax(wl.stats + 1, max_steps);
        if (flags) atomicOr(wl.stats + 2, (unsigned long long)flags);
    }
}

// Forward pass with the selective-memory windows (see the header comment).  A wave keeps
// two windows, wl.win_words int64 each (win_bins bins x S species x (sum nu, sum
// (2x+nu)nu)), so two cohorts of trajectories can be in flight: a cohort is the set of
// lanes started together; its window follows the slowest of its lanes.  A new cohort
// starts on the idle lanes once half the wave is idle and a window is free, so lanes
// whose trajectories end early are refilled instead of waiting for the slowest lane of
// their cohort.
constexpr int kCohorts = 2;
constexpr int kCohortStart = 32;      // idle lanes needed to start a cohort beside another

template <int MM, bool BATCH, bool SLAB, class Policy>
__device__ __forceinline__ void sim_fwd(const WorkList &wl, Policy &p, long long *win) {
    constexpr int MR = MM > 0 ? MM : 1;
    const uint32_t lane = __lane_id();
    const int32_t W = wl.win_bins;
    const int32_t wave_slot = (int32_t)(blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave);

    // wave-uniform work state
    int32_t cur = -1, pool_net = -1;
    int64_t pool_next = 0, pool_end = 0;
    bool exhausted = false;
    int32_t base[kCohorts] = {0, 0};
    bool live[kCohorts] = {false, false};
    GridView gv;
    gv.grid = nullptr;
    gv.T = gv.D = gv.lo = gv.scale = 0.0;
    gv.G = 0;
    gv.uniform = 0;
    int32_t S = 0, G = 0, M = 0, row_words = 0;
    unsigned long long *slab = nullptr;

    // lane state
    bool active = false, pend = false;
    int32_t coh = 0;
    int64_t traj = 0;
    double t = 0.0, t_next = 0.0, u = 0.0, tg_next = 0.0;
    uint64_t k = 0, ev = 0;
    int32_t g = 0, binp = 0;
    uint32_t ovf = 0;
    uint32_t flags = 0;
    unsigned long long tot_events = 0, max_steps = 0;
    double a[MR];
    double Ssum[MR];

    for (int32_t q = lane; q < kCohorts * wl.win_words; q += kWave) win[q] = 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();

    // flush bins [lo, hi) of cohort c's window (lanes cooperate over consecutive words)
    auto flush = [&](int32_t c, int32_t lo, int32_t hi) {
        // the window's LDS words were written by other lanes of this wave: LDS operations
        // of one wave complete in order, so only compiler reordering must be fenced off
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        long long *wc = win + c * wl.win_words;
        const int32_t words = (hi - lo) * row_words;
        for (int32_t e = lane; e < words; e += kWave) {
            const int32_t bin = lo + e / row_words, r = e - (e / row_words) * row_words;
            long long *slot = wc + (bin & (W - 1)) * row_words + r;
            const long long v = *slot;
            if (v != 0) {
                unsigned long long *dst = slab + (size_t)bin * row_words + r;
                if (SLAB) *dst = *dst + (unsigned long long)v;
                else atomicAdd(dst, (unsigned long long)v);
                *slot = 0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };

    for (;;) {
        // ---------------- start a cohort on the idle lanes ----------------
        const uint64_t idle = __ballot(!active);
        const int32_t c_free = !live[0] ? 0 : (!live[1] ? 1 : -1);
        const bool none_live = !live[0] && !live[1];
        if (idle && c_free >= 0 && (none_live || __popcll(idle) >= kCohortStart)) {
            // trajectories for the idle lanes, pulling work items as needed; a wave changes
            // network only when nothing is in flight
            const int32_t n_idle = __popcll(idle);
            const int32_t rank = __popcll(idle & lanemask_lt());
            int32_t assigned = 0;
            while (assigned < n_idle) {
                if (pool_next >= pool_end) {
                    if (exhausted) break;
                    int32_t item = 0;
                    if (lane == 0) item = (int32_t)atomicAdd(wl.counter, 1u);
                    item = wave_uniform(__shfl(item, 0));
                    if (item >= wl.n_items) {
                        exhausted = true;
                        break;
                    }
                    if (BATCH) {
                        pool_net = wave_uniform(((const SSA_CONST int32_t *)wl.item_net)[item]);
                        pool_next = wave_uniform(((const SSA_CONST int64_t *)wl.item_begin)[item]);
                        pool_end = pool_next + wave_uniform((int64_t)((const SSA_CONST int32_t *)wl.item_count)[item]);
                    } else {
                        pool_net = 0;
                        pool_next = wl.range_begin + (int64_t)item * kChunk;
                        pool_end = min(pool_next + (int64_t)kChunk, wl.range_end);
                    }
                }
                if (pool_net != cur) {
                    if (!none_live || assigned > 0) break;
                    cur = pool_net;
                    const NetDev nn = current_net<BATCH>(wl, cur);
                    p.switch_net(nn);
                    const GridInfo gi = *(const SSA_CONST GridInfo *)nn.ginfo;
                    gv.grid = wave_uniform(nn.grid);
                    gv.T = wave_uniform(gi.T);
                    gv.D = wave_uniform(gi.D);
                    gv.lo = wave_uniform(gi.lo);
                    gv.scale = wave_uniform(gi.scale);
                    gv.G = wave_uniform(nn.G);
                    gv.uniform = wave_uniform(gi.uniform);
                    S = wave_uniform(nn.S);
                    G = wave_uniform(nn.G);
                    M = wave_uniform(nn.M);
                    row_words = S * 2;
                    slab = SLAB ? wl.slabs + (size_t)wave_slot * (size_t)G * row_words : nn.D;
                }
                const int32_t take = (int32_t)min((int64_t)(n_idle - assigned), pool_end - pool_next);
                const NetDev nr = current_net<BATCH>(wl, cur);
                if (!active && rank >= assigned && rank < assigned + take) {
                    active = true;
                    pend = false;
                    coh = c_free;
                    traj = pool_next + (rank - assigned);
                    t = 0.0;
                    k = 0;
                    ev = 0;
                    g = 0;
                    ovf = 0;
                    tg_next = gv.uniform ? 0.0 : ((const SSA_CONST double *)gv.grid)[0];
                    p.reset(nr);
                }
                pool_next += take;
                assigned += take;
            }
            if (assigned > 0) {
                live[c_free] = true;
                base[c_free] = 0;
            }
        }
        if (__ballot(active) == 0) {
            if (exhausted && pool_next >= pool_end) break;
            continue;
        }

        // ---------------- one step of every unblocked active lane ----------------
        const int32_t my_base = coh ? base[1] : base[0];
        const bool blocked = active && pend && binp < G && binp >= my_base + W;
        if (active && !blocked) {
            const NetDev n = current_net<BATCH>(wl, cur);
            // the next draw does not depend on the state: start it first
            const u32x4 o = philox4x32_10((uint32_t)(k + (pend ? 1 : 0)), (uint32_t)((k + (pend ? 1 : 0)) >> 32),
                                          (uint32_t)traj, (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
            const double r1 = uniform_open0(o.v0, o.v1);
            const double r2 = uniform_open1(o.v2, o.v3);
            const double E = neg_log(r1);
            if (pend) {
                // apply the pending event at t_next (state unchanged since it was drawn)
                int32_t sel = 0;
                if constexpr (MM > 0) {
#pragma unroll
                    for (int j = 0; j < MM; ++j) sel += (Ssum[j] <= u) ? 1 : 0;
                } else {
                    sel = p.select(n, u);
                }
                if (sel >= M) {
                    for (int32_t j = M - 1; j >= 0; --j) {
                        if (p.one(n, j) > 0.0) { sel = j; break; }
                    }
                    sel = min(sel, M - 1);
                }
                const int32_t bin = binp;
                const bool inb = bin < G;
                long long *wrow = win + coh * wl.win_words + (bin & (W - 1)) * row_words;
                p.apply(n, sel, [&](int32_t sp, int32_t xo, int32_t xn) {
                    ovf |= (uint32_t)xn;
                    const int32_t dl = inb ? xn - xo : 0;
                    const long long d2 = (2ll * xo + dl) * (long long)dl;
                    long long *w = wrow + sp * 2;
                    atomicAdd((unsigned long long *)w, (unsigned long long)(long long)dl);
                    if (d2 > -kSmallD2 && d2 < kSmallD2) {
                        atomicAdd((unsigned long long *)(w + 1), (unsigned long long)d2);
                    } else {
                        atomicAdd((unsigned long long *)(w + 1), (unsigned long long)(d2 & ((1ll << 24) - 1)));
                        atomicAdd(n.Dhi + (size_t)bin * S + sp, (unsigned long long)(d2 >> 24));
                    }
                    if (n.Hd && sp == n.h_species && dl != 0) {
                        const int32_t bo = xo < n.h_lo ? 0 : min((xo - n.h_lo) / n.h_width, n.nb_hist - 1);
                        const int32_t bn = xn < n.h_lo ? 0 : min((xn - n.h_lo) / n.h_width, n.nb_hist - 1);
                        if (bo != bn) {
                            atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bo, -1);
                            atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bn, 1);
                        }
                    }
                });
                pend = false;
                k = k + 1;                 // the applied event's draw
                t = t_next;
                ev = ev + 1;
                g = bin;
                if ((int32_t)ovf < 0) {
                    flags |= kFlagOverflow;
                    active = false;
                }
            }
            if (active) {
                // draw the next event
                double acc;
                if constexpr (MM > 0) {
                    p.template eval<MM>(n, a);
                    acc = a[0];
                    Ssum[0] = acc;
#pragma unroll
                    for (int j = 1; j < MM; ++j) {
                        acc = acc + a[j];
                        Ssum[j] = acc;
                    }
                } else {
                    acc = p.total(n);
                }
                t_next = t + E / acc;
                if (acc == 0.0) {
                    active = false;                // absorbing: the state holds to t_end, no draw
                } else if (t_next > n.t_end) {
                    active = false;                // beyond the horizon: drawn, not applied
                    k = k + 1;
                } else if (ev >= n.max_events) {
                    flags |= kFlagEventLimit;
                    active = false;
                    k = k + 1;
                } else {
                    u = r2 * acc;
                    binp = gv.bin_of(g, t_next, tg_next);
                    pend = true;
                }
            }
            if (!active) {
                tot_events += ev;
                max_steps = max(max_steps, (unsigned long long)ev);
            }
        }

        // ---------------- window upkeep per cohort ----------------
#pragma unroll
        for (int c = 0; c < kCohorts; ++c) {
            if (!live[c]) continue;
            const bool mine = active && coh == c;
            if (__ballot(mine) == 0) {
                flush(c, base[c], min(G, base[c] + W));       // the cohort has ended
                live[c] = false;
                continue;
            }
            if (__ballot(mine && pend && binp < G && binp >= base[c] + W)) {
                const int32_t m = wave_min(mine && pend ? binp : G);
                if (m > base[c]) {
                    flush(c, base[c], min(m, base[c] + W));
                    base[c] = m;
                }
            }
        }
    }

    // wave totals -> global statistics
    for (int off = 32; off > 0; off >>= 1) {
        tot_events += __shfl_xor(tot_events, off);
        max_steps = max(max_steps, (unsigned long long)__shfl_xor(max_steps, off));
        flags |= (uint32_t)__shfl_xor((int)flags, off);
    }
    if (lane == 0) {
        if (tot_events) atomicAdd(wl.stats + 0, tot_events);
        atomicMax(wl.stats + 1, max_steps);
        if (flags) atomicOr(wl.stats + 2, (unsigned long long)flags);
    }
}

}  // namespace ssa
