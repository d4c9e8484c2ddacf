// ssa_wave.hpp -- one trajectory per wave, for networks whose propensities are summed in
// the 64-chunk order (the wavefront-level prefix sum of the selection step, Section 2).
//
// Lane l owns the reactions l q .. l q + q - 1 (q = ceil(M / 64)) and keeps their packed
// reactant codes and rate constants in registers.  Per event every lane evaluates its
// propensities and their sequential sum inside the chunk; the 64 chunk totals go through
// a six-step inclusive Kogge-Stone scan across the wave (offsets 1, 2, 4, ..., 32), and
// S_j = (scanned total of the chunks before l) + (local sum up to j).  The selected
// reaction is the smallest j with S_j > u, found with one ballot over the lanes.  The
// species counts live in LDS, one row per wave (row 0 holds the constant 1 that stands in
// for a missing reactant, species s is row s + 1).
//
// The time bookkeeping (t, k, the grid index) is the same in every lane.  Forward events
// add their moment differences straight to the network's totals with atomic adds (one
// trajectory per wave leaves nothing to aggregate in a window).
#pragma once

#include "ssa_kernels.hpp"

namespace ssa {

__device__ __forceinline__ double wave_propensity(uint32_t code, double c, const int32_t *xl) {
    const int32_t ra = (int32_t)(code & 0xfffu), rb = (int32_t)((code >> 12) & 0xfffu);
    const int32_t d = (int32_t)(code >> 24);
    const int32_t xa = xl[ra];
    const int32_t xb = max(xl[rb] - d, 0);
    const double f = d ? 0.5 : 1.0;
    return c * (((double)xa * (double)xb) * f);
}

__device__ __forceinline__ double shfl_up_f64(double v, int d) {
    return __shfl_up(v, (unsigned)d, kWave);
}

__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int off = 32; off > 0; off >>= 1) v = v + __shfl_xor(v, off, kWave);
    return v;
}

// Backward sums alpha, beta over the crossings [ga, gb) of an interval starting at t (see
// interval_sums), one trajectory per wave: the species are spread over the lanes and summed
// across the wave.  With n.bp_quad the table carries the variance columns (weights
// quadratic in x).
__device__ __forceinline__ void wave_interval_sums(const NetDev &n, const int32_t *xl, int32_t ga, int32_t gb,
                                                   double t, uint32_t lane, double &alpha, double &beta) {
    const int32_t S = n.S;
    const int32_t ncol = n.bp_quad ? 4 * S + 2 : 2 * S + 2;
    const PrefixRow ra(n.bp, ncol, ga), rb(n.bp, ncol, gb);
    double sw = 0.0, swt = 0.0;
    for (int32_t s = lane; s < S; s += kWave) {
        const double xs = (double)xl[s + 1];
        const double dW = ra.diff_to(rb, s);
        const double dWT = ra.diff_to(rb, S + s);
        sw = sw + xs * dW;
        swt = swt + xs * (dWT - t * dW);
        if (n.bp_quad) {
            const double x2 = xs * xs;
            const double dQ = ra.diff_to(rb, 2 * S + 2 + s);
            const double dQT = ra.diff_to(rb, 3 * S + 2 + s);
            sw = sw + x2 * dQ;
            swt = swt + x2 * (dQT - t * dQ);
        }
    }
    sw = wave_sum_f64(sw);
    swt = wave_sum_f64(swt);
    const double dC = ra.diff_to(rb, 2 * S);
    const double dCT = ra.diff_to(rb, 2 * S + 1);
    alpha = sw - dC;
    beta = swt - (dCT - t * dC);
}

// Event log, one trajectory per wave: the lanes that applied a change (has) append its
// record (time bits; species, change, previous count) through one cursor bump for the wave.
// Returns true if a record did not fit (the host then runs the epoch again shorter).
__device__ __forceinline__ bool wave_log_event(const NetDev &n, bool has, double t_next, int32_t sp, int32_t dl,
                                               int32_t xo, uint32_t lane) {
    const uint64_t mk = __ballot(has);
    if (!mk) return false;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(n.ev_cursor, (unsigned long long)__popcll(mk));
    const uint32_t blo = (uint32_t)__shfl((int)(uint32_t)base, 0);
    const uint32_t bhi = (uint32_t)__shfl((int)(uint32_t)(base >> 32), 0);
    const int64_t at = (int64_t)(((unsigned long long)bhi << 32) | blo) + __popcll(mk & lanemask_lt());
    bool full = false;
    if (has && n.ev_key) {
        if (at < n.ev_cap) {
            n.ev_key[at] = (unsigned long long)__double_as_longlong(t_next);
            n.ev_val[at] = ev_pack(sp, dl, xo);
        } else {
            full = true;
        }
    }
    return __ballot(full) != 0;
}

// Event log in epochs (NetDev::rs_*, ws_*), one trajectory per wave: load the saved state
// into the LDS row, or save it (time -1 once the trajectory has ended).
__device__ __forceinline__ void wave_evt_resume(const NetDev &n, int64_t traj, int32_t *xl, uint32_t lane, double &t,
                                                uint64_t &k, uint64_t &ev, uint64_t &ev_start, bool &gone) {
    for (int32_t s = lane; s < n.S; s += kWave) xl[s + 1] = n.rs_x[(size_t)traj * n.S + s];
    t = n.rs_t[traj];
    k = n.rs_k[traj];
    ev = n.rs_ev[traj];
    ev_start = ev;
    gone = t < 0.0;
    if (gone) t = n.t_end;
}

__device__ __forceinline__ void wave_evt_save(const NetDev &n, int64_t traj, const int32_t *xl, uint32_t lane,
                                              bool pause, double t, uint64_t k, uint64_t ev) {
    for (int32_t s = lane; s < n.S; s += kWave) n.ws_x[(size_t)traj * n.S + s] = xl[s + 1];
    if (lane == 0) {
        n.ws_t[traj] = pause ? t : -1.0;
        n.ws_k[traj] = k;
        n.ws_ev[traj] = ev;
    }
}

// LDS: one row of (S + 1) int32 per wave.
template <int Q, int MODE>
__global__ void __launch_bounds__(kBlock) wave_kernel(WorkList wl) {
    extern __shared__ int32_t lds_w[];
    const uint32_t lane = __lane_id();
    const NetDev n = wl.net0;
    const int32_t S = n.S, M = n.M, G = n.G, q = n.q;
    int32_t *xl = lds_w + (threadIdx.x / kWave) * (S + 1);

    // this lane's reactions
    uint32_t code[Q];
    double c[Q];
    int32_t jr[Q];        // reaction index, or -1 for an empty slot
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int32_t j = (int32_t)lane * q + i;
        const bool real = i < q && j < M;
        jr[i] = real ? j : -1;
        code[i] = real ? n.rx[j] : 0u;
        c[i] = real ? n.rate[j] : 0.0;
    }
    const int32_t last_lane = (M - 1) / q, last_slot = (M - 1) - last_lane * q;

    const GridInfo gi = *(const SSA_CONST GridInfo *)n.ginfo;
    GridView gv;
    gv.grid = n.grid;
    gv.T = gi.T;
    gv.D = gi.D;
    gv.lo = gi.lo;
    gv.scale = gi.scale;
    gv.G = G;
    gv.uniform = gi.uniform;

    uint32_t flags = 0;
    unsigned long long tot_events = 0, max_steps = 0;

    for (;;) {
        int32_t item = 0;
        if (lane == 0) item = (int32_t)atomicAdd(wl.counter, 1u);
        item = wave_uniform(__shfl(item, 0));
        if ((int64_t)item >= wl.range_end - wl.range_begin) break;
        const int64_t traj = wl.range_begin + item;

        if (lane == 0) xl[0] = 1;
        for (int32_t s = lane; s < S; s += kWave) xl[s + 1] = n.x0[s];
        double t = 0.0;
        uint64_t k = 0, ev = 0, ev_start = 0;
        bool gone = false, pause = false;
        if (MODE == kEvt && n.rs_t) wave_evt_resume(n, traj, xl, lane, t, k, ev, ev_start, gone);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();

        int32_t g = 0;
        double tg_next = G > 0 ? gv.at(0) : 0.0;
        // record: A_j and n_j; backward: the score B_j = n_j - A_j and the accumulator
        double A[MODE == kRec ? Q : 1], nf[MODE == kRec ? Q : 1];
        double B[MODE == kBwd ? Q : 1], gacc[MODE == kBwd ? Q : 1];
        if (MODE == kRec) {
#pragma unroll
            for (int i = 0; i < Q; ++i) { A[i] = 0.0; nf[i] = 0.0; }
        }
        if (MODE == kBwd) {
#pragma unroll
            for (int i = 0; i < Q; ++i) { B[i] = 0.0; gacc[i] = 0.0; }
        }
        bool overflow = false;

        for (;;) {
            // propensities and the local sums of this lane's chunk
            double a[Q], L[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                a[i] = wave_propensity(code[i], c[i], xl);
                L[i] = i == 0 ? a[0] : L[i - 1] + a[i];       // empty slots add +0
            }
            // inclusive Kogge-Stone scan of the chunk totals, then the exclusive offsets
            double v = L[Q - 1];
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const double up = shfl_up_f64(v, d);
                if ((int)lane >= d) v = v + up;
            }
            double E = shfl_up_f64(v, 1);
            if (lane == 0) E = 0.0;
            double mine_last = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) mine_last = (i == last_slot) ? E + L[i] : mine_last;
            const double a0 = wave_uniform(__shfl(mine_last, last_lane, kWave));

            double tau = __builtin_inf(), r2 = 0.0;
            if (a0 != 0.0) {
                const u32x4 o = philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), (uint32_t)traj,
                                              (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
                const double r1 = uniform_open0(o.v0, o.v1);
                r2 = uniform_open1(o.v2, o.v3);
                tau = neg_log(r1) / a0;
                k = k + 1;
            }
            const double t_next = t + tau;

            if (MODE == kRec) {
                int32_t *rows = n.rec_states + (size_t)(traj - n.rec_begin) * G * S;
                while (g < G && gv.at(g) < t_next) {
                    for (int32_t s = lane; s < S; s += kWave) rows[(size_t)g * S + s] = xl[s + 1];
                    ++g;
                }
            } else if (MODE == kBwd) {
                // crossings [g, gb) of this interval from two prefix rows (see interval_sums);
                // the species are spread over the lanes
                if (g < G && tg_next < t_next) {
                    double tb;
                    const int32_t gb = gv.next_bin(g, t_next, tb);
                    double alpha, beta;
                    wave_interval_sums(n, xl, g, gb, t, lane, alpha, beta);
#pragma unroll
                    for (int i = 0; i < Q; ++i) gacc[i] = gacc[i] + (B[i] * alpha - a[i] * beta);
                    g = gb;
                    tg_next = tb;
                }
            }

            if (MODE == kEvt && n.ws_t) {
                // epochs: an ended trajectory stays ended; an event beyond the epoch waits for
                // the next one, which redraws the same Philox block from the same state
                if (gone) break;
                if (t_next <= n.t_end && t_next > n.t_pause) {
                    pause = true;
                    if (a0 != 0.0) k = k - 1;
                    break;
                }
            }
            if (t_next > n.t_end) break;
            if (ev >= n.max_events) {
                flags |= kFlagEventLimit;
                break;
            }
            // selection: smallest j with S_j > u, else the largest j with a_j > 0
            const double u = r2 * a0;
            int32_t first = -1, lastpos = -1;
#pragma unroll
            for (int i = Q - 1; i >= 0; --i) {
                if (jr[i] >= 0 && E + L[i] > u) first = jr[i];
                if (lastpos < 0 && jr[i] >= 0 && a[i] > 0.0) lastpos = jr[i];
            }
            int32_t sel;
            const uint64_t hit = __ballot(first >= 0);
            if (hit) {
                sel = __shfl(first, __ffsll((unsigned long long)hit) - 1, kWave);
            } else {
                const uint64_t pos = __ballot(lastpos >= 0);
                sel = pos ? __shfl(lastpos, 63 - __clzll((unsigned long long)pos), kWave) : M - 1;
            }
            sel = wave_uniform(sel);

            // grid bin of the event (forward)
            int32_t bin = G;
            if (MODE == kFwd) {
                bin = g;
                if (g < G && t_next > tg_next) bin = gv.next_bin(g, t_next, tg_next);
            }
            // apply: lanes 0 .. kChg-1 take one change slot each (distinct species)
            int32_t log_sp = 0, log_dl = 0, log_xo = 0;   // event log: this lane's change
            if ((int)lane < kChg) {
                const int32_t cv = n.chg[sel * kChg + lane];
                const int32_t r = chg_row(cv), dl = chg_delta(cv);
                if (dl != 0) {
                    const int32_t xo = xl[r];
                    const int64_t xw = (int64_t)xo + dl;
                    overflow = xw > 2147483647ll || xw < -2147483647ll - 1;
                    const int32_t xn = (int32_t)xw;
                    xl[r] = xn;
                    log_sp = r - 1;
                    log_dl = dl;
                    log_xo = xo;
                    if (MODE == kFwd && bin < G && !overflow) {
                        const int32_t sp = r - 1;
                        unsigned long long *dd = n.D + ((size_t)bin * S + sp) * 2;
                        const long long d2 = (2ll * xo + dl) * (long long)dl;
                        atomicAdd(dd, (unsigned long long)(long long)dl);
                        if (d2 > -kSmallD2 && d2 < kSmallD2) {
                            atomicAdd(dd + 1, (unsigned long long)d2);
                        } else {
                            atomicAdd(dd + 1, (unsigned long long)(d2 & ((1ll << 24) - 1)));
                            atomicAdd(n.Dhi + (size_t)bin * S + sp, (unsigned long long)(d2 >> 24));
                        }
                        if (n.Hd && sp == n.h_species) {
                            const int32_t bo = xo < n.h_lo ? 0 : min((xo - n.h_lo) / n.h_width, n.nb_hist - 1);
                            const int32_t bn = xn < n.h_lo ? 0 : min((xn - n.h_lo) / n.h_width, n.nb_hist - 1);
                            if (bo != bn) {
                                atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bo, -1);
                                atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bn, 1);
                            }
                        }
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (__ballot(overflow)) {
                flags |= kFlagOverflow;
                break;
            }
            if (MODE == kEvt) {
                const bool has = (int)lane < kChg && log_dl != 0;
                if (wave_log_event(n, has, t_next, log_sp, log_dl, log_xo, lane)) flags |= kFlagRecordsFull;
            }
            if (MODE == kRec) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    A[i] = A[i] + a[i] * tau;
                    nf[i] = nf[i] + (jr[i] == sel ? 1.0 : 0.0);
                }
            }
            if (MODE == kBwd) {
#pragma unroll
                for (int i = 0; i < Q; ++i) B[i] = B[i] + ((jr[i] == sel ? 1.0 : 0.0) - a[i] * tau);
            }
            t = t_next;
            ev = ev + 1;
            if (MODE == kFwd) g = bin;
        }

        if (MODE == kRec) {
            const int64_t r = traj - n.rec_begin;
            if (lane == 0) {
                n.rec_events[r] = ev;
                n.rec_draws[r] = k;
                n.rec_tlast[r] = t;
            }
            // final propensities for the last partial interval of A_j
            const double tail = n.t_end - t;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (jr[i] < 0) continue;
                if (n.rec_nf) n.rec_nf[r * M + jr[i]] = (int64_t)nf[i];
                if (n.rec_aint) n.rec_aint[r * M + jr[i]] = A[i] + wave_propensity(code[i], c[i], xl) * tail;
            }
        }
        if (MODE == kBwd) {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (jr[i] >= 0) n.gtraj[(size_t)traj * M + jr[i]] = gacc[i];
        }
        if (MODE == kEvt && n.ws_t) wave_evt_save(n, traj, xl, lane, pause, t, k, ev);
        tot_events += ev - ev_start;
        max_steps = max(max_steps, (unsigned long long)ev);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) {
        if (tot_events) atomicAdd(wl.stats + 0, tot_events);
        atomicMax(wl.stats + 1, max_steps);
        if (flags) atomicOr(wl.stats + 2, (unsigned long long)flags);
    }
}

// Rate constants in dependency-entry order: out[p] = rate[reaction of entry p].
__global__ void dep_rate_kernel(const int2 *dep, int32_t q, const double *rate, int64_t nnz, double *out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t slot = dep[p].x;
        out[p] = rate[(slot & (kWave - 1)) * q + (slot >> 6)];
    }
}

// Networks with more than 8 reactions per lane (q up to 64, M up to 4096), same sum order.
// One wave per block; the chunk values live in LDS, slot i of lane l at word i * 64 + l,
// so a row of slots is one conflict-free access.
//
// DEPG: the LDS slots hold the propensities themselves.  After an event only the
// propensities that read a species the event changed are evaluated again, from the
// dependency list of the fired reaction (slot and reactant code of each reaction whose
// reactants intersect the changed species, with its rate constant in a parallel array);
// every other slot keeps its value.  Without
// DEPG the slots hold the rate constants and the reactant codes, and every lane
// re-evaluates its whole chunk each event.  Both re-add the chunk's local sums in order
// from the current values, so the partial sums, the selected reaction and the trajectory
// are those of the full recomputation, bit for bit: the graph changes how much work an
// event costs (the propensity evaluations of the reactions it touches instead of M), not
// what is computed.
//
// Modes: forward (moment differences and histogram straight into the network totals, as
// above), record (per-trajectory grid states; the n_j and A_j rows accumulate in the
// caller's output arrays) and backward (the score B_j and the gradient accumulator of every
// slot in two more LDS rows each, updated as in the register kernel; the crossings'
// alpha, beta from the prefix rows with the species spread over the lanes).
template <int Q, int MODE, bool DEPG>
__global__ void __launch_bounds__(kWave) wide_kernel(WorkList wl) {
    extern __shared__ double lds_d[];
    const uint32_t lane = __lane_id();
    const NetDev n = wl.net0;
    const int32_t S = n.S, M = n.M, G = n.G, q = n.q;
    double *av = lds_d;                                             // [Q][64] propensities | rates
    double *bsc = lds_d + Q * kWave;                                // backward: [Q][64] scores B_j
    double *gac = bsc + (MODE == kBwd ? Q * kWave : 0);             // backward: [Q][64] accumulators
    double *after = gac + (MODE == kBwd ? Q * kWave : 0);
    uint32_t *cw = (uint32_t *)after;                               // [Q][64] codes (without DEPG)
    int32_t *xl = (int32_t *)after + (DEPG ? 0 : Q * kWave);
    // real slots of this lane: reactions lane q .. lane q + nreal - 1
    const int32_t nreal = max(0, min(q, M - (int32_t)lane * q));
    const int32_t last_lane = (M - 1) / q;

    if (!DEPG) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int32_t j = (int32_t)lane * q + i;
            av[i * kWave + lane] = i < nreal ? n.rate[j] : 0.0;
            cw[i * kWave + lane] = i < nreal ? n.rx[j] : 0u;
        }
    }

    const GridInfo gi = *(const SSA_CONST GridInfo *)n.ginfo;
    GridView gv;
    gv.grid = n.grid;
    gv.T = gi.T;
    gv.D = gi.D;
    gv.lo = gi.lo;
    gv.scale = gi.scale;
    gv.G = G;
    gv.uniform = gi.uniform;

    uint32_t flags = 0;
    unsigned long long tot_events = 0, max_steps = 0;

    for (;;) {
        int32_t item = 0;
        if (lane == 0) item = (int32_t)atomicAdd(wl.counter, 1u);
        item = wave_uniform(__shfl(item, 0));
        if ((int64_t)item >= wl.range_end - wl.range_begin) break;
        const int64_t traj = wl.range_begin + item;
        const int64_t r = traj - n.rec_begin;

        if (lane == 0) xl[0] = 1;
        for (int32_t s = lane; s < S; s += kWave) xl[s + 1] = n.x0[s];
        double t = 0.0;
        uint64_t k = 0, ev = 0, ev_start = 0;
        bool gone = false, pause = false;
        if (MODE == kEvt && n.rs_t) wave_evt_resume(n, traj, xl, lane, t, k, ev, ev_start, gone);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (DEPG) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int32_t j = (int32_t)lane * q + i;
                av[i * kWave + lane] = i < nreal ? wave_propensity(n.rx[j], n.rate[j], xl) : 0.0;
            }
        }
        if (MODE == kRec) {
            for (int32_t i = 0; i < nreal; ++i) {
                const int32_t j = (int32_t)lane * q + i;
                if (n.rec_nf) n.rec_nf[r * M + j] = 0;
                if (n.rec_aint) n.rec_aint[r * M + j] = 0.0;
            }
        }
        if (MODE == kBwd) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                bsc[i * kWave + lane] = 0.0;
                gac[i * kWave + lane] = 0.0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();

        int32_t g = 0;
        double tg_next = G > 0 ? gv.at(0) : 0.0;
        bool overflow = false;
        // draw k's uniforms and -ln r1, prepared one event ahead (they depend on k only;
        // an absorbing state leaves them unused)
        double r2n, nl;
        {
            const u32x4 o = philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), (uint32_t)traj,
                                          (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
            r2n = uniform_open1(o.v2, o.v3);
            nl = neg_log(uniform_open0(o.v0, o.v1));
        }

        for (;;) {
            // local sums of this lane's chunk, in slot order
            double L[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double ai = DEPG ? av[i * kWave + lane]
                                       : wave_propensity(cw[i * kWave + lane], av[i * kWave + lane], xl);
                L[i] = i == 0 ? ai : L[i - 1] + ai;    // empty slots add +0
            }
            double v = L[Q - 1];
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const double up = shfl_up_f64(v, d);
                if ((int)lane >= d) v = v + up;
            }
            double E = shfl_up_f64(v, 1);
            if (lane == 0) E = 0.0;
            const double a0 = wave_uniform(__shfl(E + L[Q - 1], last_lane, kWave));

            double tau = __builtin_inf(), r2 = 0.0;
            if (a0 != 0.0) {
                r2 = r2n;
                tau = nl / a0;
                k = k + 1;
            }
            const double t_next = t + tau;

            if (MODE == kRec) {
                int32_t *rows = n.rec_states + (size_t)r * G * S;
                while (g < G && gv.at(g) < t_next) {
                    for (int32_t s = lane; s < S; s += kWave) rows[(size_t)g * S + s] = xl[s + 1];
                    ++g;
                }
            } else if (MODE == kBwd) {
                // crossings [g, gb) of this interval from two prefix rows; the species are
                // spread over the lanes, every slot's accumulator takes B_j alpha - a_j beta
                if (g < G && tg_next < t_next) {
                    double tb;
                    const int32_t gb = gv.next_bin(g, t_next, tb);
                    double alpha, beta;
                    wave_interval_sums(n, xl, g, gb, t, lane, alpha, beta);
                    for (int32_t i = 0; i < nreal; ++i) {
                        const double ai = DEPG ? av[i * kWave + lane]
                                               : wave_propensity(cw[i * kWave + lane], av[i * kWave + lane], xl);
                        double &gi = gac[i * kWave + lane];
                        gi = gi + (bsc[i * kWave + lane] * alpha - ai * beta);
                    }
                    g = gb;
                    tg_next = tb;
                }
            }
            if (MODE == kEvt && n.ws_t) {
                // epochs: an ended trajectory stays ended; an event beyond the epoch waits for
                // the next one, which redraws the same Philox block from the same state
                if (gone) break;
                if (t_next <= n.t_end && t_next > n.t_pause) {
                    pause = true;
                    if (a0 != 0.0) k = k - 1;
                    break;
                }
            }
            if (t_next > n.t_end) break;
            if (ev >= n.max_events) {
                flags |= kFlagEventLimit;
                break;
            }

            // selection: smallest j with S_j > u (the local sums are non-decreasing, so the
            // first slot that passes is the lane's candidate), else the largest j with a_j > 0
            const double u = r2 * a0;
            int32_t first = -1;
#pragma unroll
            for (int i = Q - 1; i >= 0; --i)
                if (E + L[i] > u) first = i;
            if (nreal == 0) first = -1;
            int32_t sel, sel_lane;
            const uint64_t hit = __ballot(first >= 0);
            if (hit) {
                sel_lane = __ffsll((unsigned long long)hit) - 1;
                sel = sel_lane * q + __shfl(first, sel_lane, kWave);
            } else {
                int32_t lastpos = -1;
                for (int32_t i = 0; i < nreal; ++i) {
                    const double ai = DEPG ? av[i * kWave + lane]
                                           : wave_propensity(cw[i * kWave + lane], av[i * kWave + lane], xl);
                    if (ai > 0.0) lastpos = i;
                }
                const uint64_t pos = __ballot(lastpos >= 0);
                if (pos) {
                    sel_lane = 63 - __clzll((unsigned long long)pos);
                    sel = sel_lane * q + __shfl(lastpos, sel_lane, kWave);
                } else {
                    sel_lane = last_lane;
                    sel = M - 1;
                }
            }
            sel = wave_uniform(sel);
            sel_lane = wave_uniform(sel_lane);

            if (MODE == kBwd) {
                // B_j += [j fired] - a_j tau with the propensities before the event
                for (int32_t i = 0; i < nreal; ++i) {
                    const double ai = DEPG ? av[i * kWave + lane]
                                           : wave_propensity(cw[i * kWave + lane], av[i * kWave + lane], xl);
                    const int32_t j = (int32_t)lane * q + i;
                    double &bi = bsc[i * kWave + lane];
                    bi = bi + ((j == sel ? 1.0 : 0.0) - ai * tau);
                }
            }
            if (MODE == kRec) {
                // A_j += a_j tau with the propensities of the state before the event
                if (n.rec_aint) {
                    for (int32_t i = 0; i < nreal; ++i) {
                        const double ai = DEPG ? av[i * kWave + lane]
                                               : wave_propensity(cw[i * kWave + lane], av[i * kWave + lane], xl);
                        double *pa = n.rec_aint + r * M + (int32_t)lane * q + i;
                        *pa = *pa + ai * tau;
                    }
                }
                // the lane that owns the fired reaction counts it (it also zeroed the slot)
                if (n.rec_nf && (int32_t)lane == sel_lane) n.rec_nf[r * M + sel] += 1;
            }

            int32_t bin = G;
            if (MODE == kFwd) {
                bin = g;
                if (g < G && t_next > tg_next) bin = gv.next_bin(g, t_next, tg_next);
            }
            int32_t log_sp = 0, log_dl = 0, log_xo = 0;   // event log: this lane's change
            if ((int)lane < kChg) {
                const int32_t cv = n.chg[sel * kChg + lane];
                const int32_t rr = chg_row(cv), dl = chg_delta(cv);
                if (dl != 0) {
                    const int32_t xo = xl[rr];
                    const int64_t xw = (int64_t)xo + dl;
                    overflow = xw > 2147483647ll || xw < -2147483647ll - 1;
                    const int32_t xn = (int32_t)xw;
                    xl[rr] = xn;
                    log_sp = rr - 1;
                    log_dl = dl;
                    log_xo = xo;
                    if (MODE == kFwd && bin < G && !overflow) {
                        const int32_t sp = rr - 1;
                        unsigned long long *dd = n.D + ((size_t)bin * S + sp) * 2;
                        const long long d2 = (2ll * xo + dl) * (long long)dl;
                        atomicAdd(dd, (unsigned long long)(long long)dl);
                        if (d2 > -kSmallD2 && d2 < kSmallD2) {
                            atomicAdd(dd + 1, (unsigned long long)d2);
                        } else {
                            atomicAdd(dd + 1, (unsigned long long)(d2 & ((1ll << 24) - 1)));
                            atomicAdd(n.Dhi + (size_t)bin * S + sp, (unsigned long long)(d2 >> 24));
                        }
                        if (n.Hd && sp == n.h_species) {
                            const int32_t bo = xo < n.h_lo ? 0 : min((xo - n.h_lo) / n.h_width, n.nb_hist - 1);
                            const int32_t bn = xn < n.h_lo ? 0 : min((xn - n.h_lo) / n.h_width, n.nb_hist - 1);
                            if (bo != bn) {
                                atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bo, -1);
                                atomicAdd(n.Hd + (size_t)bin * n.nb_hist + bn, 1);
                            }
                        }
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (__ballot(overflow)) {
                flags |= kFlagOverflow;
                break;
            }
            if (MODE == kEvt) {
                const bool has = (int)lane < kChg && log_dl != 0;
                if (wave_log_event(n, has, t_next, log_sp, log_dl, log_xo, lane)) flags |= kFlagRecordsFull;
            }
            if (DEPG) {
                // re-evaluate the propensities that read a changed species; the first 64
                // entries are loaded before the next draw is prepared, so their latency
                // overlaps it
                const int32_t p0 = n.dep_ptr[sel], p1 = n.dep_ptr[sel + 1];
                const int32_t pf = p0 + (int32_t)lane;
                int2 e = make_int2(0, 0);
                double ce = 0.0;
                if (pf < p1) {
                    e = n.dep[pf];
                    ce = n.dep_rate[pf];
                }
                const u32x4 o = philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), (uint32_t)traj,
                                              (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
                r2n = uniform_open1(o.v2, o.v3);
                nl = neg_log(uniform_open0(o.v0, o.v1));
                if (pf < p1) av[e.x] = wave_propensity((uint32_t)e.y, ce, xl);
                for (int32_t p = pf + kWave; p < p1; p += kWave) {
                    const int2 e2 = n.dep[p];
                    av[e2.x] = wave_propensity((uint32_t)e2.y, n.dep_rate[p], xl);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
            } else {
                const u32x4 o = philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), (uint32_t)traj,
                                              (uint32_t)((uint64_t)traj >> 32), n.key0, n.key1);
                r2n = uniform_open1(o.v2, o.v3);
                nl = neg_log(uniform_open0(o.v0, o.v1));
            }
            t = t_next;
            ev = ev + 1;
            if (MODE == kFwd) g = bin;
        }

        if (MODE == kRec) {
            if (lane == 0) {
                n.rec_events[r] = ev;
                n.rec_draws[r] = k;
                n.rec_tlast[r] = t;
            }
            // the last partial interval of A_j, with the final state's propensities
            if (n.rec_aint) {
                const double tail = n.t_end - t;
                for (int32_t i = 0; i < nreal; ++i) {
                    const double ai = DEPG ? av[i * kWave + lane]
                                           : wave_propensity(cw[i * kWave + lane], av[i * kWave + lane], xl);
                    double *pa = n.rec_aint + r * M + (int32_t)lane * q + i;
                    *pa = *pa + ai * tail;
                }
            }
        }
        if (MODE == kBwd) {
            for (int32_t i = 0; i < nreal; ++i)
                n.gtraj[(size_t)traj * M + (int32_t)lane * q + i] = gac[i * kWave + lane];
        }
        if (MODE == kEvt && n.ws_t) wave_evt_save(n, traj, xl, lane, pause, t, k, ev);
        tot_events += ev - ev_start;
        max_steps = max(max_steps, (unsigned long long)ev);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) {
        if (tot_events) atomicAdd(wl.stats + 0, tot_events);
        atomicMax(wl.stats + 1, max_steps);
        if (flags) atomicOr(wl.stats + 2, (unsigned long long)flags);
    }
}

}  // namespace ssa
