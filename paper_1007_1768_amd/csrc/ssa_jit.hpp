// ssa_jit.hpp -- kernels specialised to one reaction network, compiled at run time.
//
// The host library generates `ssa_gen::Net` for a network (species count, reaction
// count, initial state, the propensity expressions and the stoichiometric changes as
// constants) and compiles this file with it.  Each lane then keeps its species counts in
// registers with compile-time indices, evaluates every propensity as straight-line code
// (only the rate constants are read, as scalars) and applies a reaction through per-species
// select chains, so the event loop of ssa_sim.hpp runs without tables or LDS traffic.
#pragma once

#include "ssa_sim.hpp"

namespace ssa {

struct RegPolicy {
    using Net = ssa_gen::Net;
    int32_t x[Net::S];
    double c[Net::M];     // rate constants, held in vector registers for the whole launch

    // The rates are loaded once and pinned in VGPRs: read through the scalar cache at every
    // event they put a load and its wait (which also waits for the outstanding LDS
    // atomics) on each event's critical path.
    __device__ __forceinline__ void switch_net(const NetDev &n) {
#pragma unroll
        for (int j = 0; j < Net::M; ++j) {
            c[j] = n.rate[j];
            asm volatile("" : "+v"(c[j]));
        }
    }
    __device__ __forceinline__ void reset(const NetDev &) { Net::init(x); }
    __device__ __forceinline__ void load_state(const int32_t *src) {
#pragma unroll
        for (int s = 0; s < Net::S; ++s) x[s] = src[s];
    }
    template <int MM>
    __device__ __forceinline__ void eval(const NetDev &, double (&a)[MM]) const {
        static_assert(MM == Net::M, "one propensity slot per reaction");
        Net::props(x, c, a);
    }
    __device__ double one(const NetDev &, int32_t j) const {
        double a[Net::M];
        Net::props(x, c, a);
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < Net::M; ++q) v = (q == j) ? a[q] : v;
        return v;
    }
    __device__ double total(const NetDev &) const { return 0.0; }
    __device__ int32_t select(const NetDev &, double) const { return 0; }
    template <class F>
    __device__ __forceinline__ void for_each_species(F f) const {
#pragma unroll
        for (int s = 0; s < Net::S; ++s) f(s, x[s]);
    }
    // Up to 8 species every species that some reaction changes is updated on every event
    // (f may then see x_new == x_old), so the update has no branches on the divergent
    // selection; larger networks skip the species the reaction leaves alone.
    static constexpr bool kDense = Net::S <= 8;
    template <class F>
    __device__ __forceinline__ void apply(const NetDev &, int32_t sel, F f) {
        int32_t dx[Net::S];
        Net::deltas(sel, dx);
#pragma unroll
        for (int s = 0; s < Net::S; ++s) {
            if (Net::changes(s) && (kDense || dx[s] != 0)) {
                const int32_t xo = x[s];
                const int32_t xn = xo + dx[s];
                x[s] = xn;
                f(s, xo, xn);
            }
        }
    }
    // f(s, x_old, x_new) for the species reaction sel changed, after apply(n, sel, ...)
    template <class F>
    __device__ __forceinline__ void replay(const NetDev &, int32_t sel, F f) const {
        int32_t dx[Net::S];
        Net::deltas(sel, dx);
#pragma unroll
        for (int s = 0; s < Net::S; ++s)
            if (Net::changes(s) && dx[s] != 0) f(s, x[s] - dx[s], x[s]);
    }
};

}  // namespace ssa

// Forward pass by generations: one selective-memory window of wl.win_words int64 per wave in
// dynamic LDS;
// flushes into wave-private slabs (ssa_jit_fwd) or atomically into the totals (_atomic).
extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_fwd(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, true, false>(wl, p,
                                                          ssa_win + (threadIdx.x / ssa::kWave) * wl.win_words);
}

extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_fwd_atomic(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, false>(wl, p,
                                                           ssa_win + (threadIdx.x / ssa::kWave) * wl.win_words);
}

// The same with the per-grid-point histogram of one species.
extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_fwd_hist(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, true>(wl, p,
                                                          ssa_win + (threadIdx.x / ssa::kWave) * wl.win_words);
}

extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_fwd_slab_hist(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, true, true>(wl, p,
                                                         ssa_win + (threadIdx.x / ssa::kWave) * wl.win_words);
}

// One epoch of a run in epochs of simulation time, without and with the histogram.
extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_fwd_epoch(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, false, ssa::RegPolicy, false, false, true>(
        wl, p, ssa_win + (threadIdx.x / ssa::kWave) * wl.win_words);
}

extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_fwd_hist_epoch(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, true, ssa::RegPolicy, false, false, true>(
        wl, p, ssa_win + (threadIdx.x / ssa::kWave) * wl.win_words);
}

// Forward pass with the species cross products (covariance matrices per grid point).
extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_fwd_cov(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, false, ssa::RegPolicy, true>(
        wl, p, ssa_win + (threadIdx.x / ssa::kWave) * wl.win_words);
}

// Forward pass with the likelihood-ratio Jacobian: per wave, the moment window
// (win_bins x S x 2 int64) followed by the Jacobian window (win_bins x (S+1) x M doubles);
// wl.win_words is their total in 8-byte words.
extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_fwd_jac(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    ssa::RegPolicy p;
    long long *w = ssa_win + (threadIdx.x / ssa::kWave) * wl.win_words;
    ssa::sim_fwd_jac<ssa_gen::Net::M>(wl, p, w, (double *)(w + wl.win_bins * ssa_gen::Net::S * 2));
}

extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_rec(ssa::WorkList wl) {
    ssa::RegPolicy p;
    ssa::sim_loop<ssa::kRec, ssa_gen::Net::M, false>(wl, p);
}

extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_evt(ssa::WorkList wl) {
    ssa::RegPolicy p;
    ssa::sim_loop<ssa::kEvt, ssa_gen::Net::M, false>(wl, p);
}

extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_bwd(ssa::WorkList wl) {
    ssa::RegPolicy p;
    ssa::sim_loop<ssa::kBwd, ssa_gen::Net::M, false>(wl, p);
}

// Backward with variance weights (prefix table with the quadratic columns).
extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_bwd_var(ssa::WorkList wl) {
    ssa::RegPolicy p;
    ssa::sim_loop<ssa::kBwd, ssa_gen::Net::M, false, ssa::RegPolicy, true>(wl, p);
}

// The backward in generations (lanes refilled only once the whole wave is idle), for
// launches of about one wave per SIMD.
extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_bwd_gen(ssa::WorkList wl) {
    ssa::RegPolicy p;
    ssa::sim_loop<ssa::kBwd, ssa_gen::Net::M, false, ssa::RegPolicy, false, true>(wl, p);
}

extern "C" __global__ void __launch_bounds__(ssa::kBlock) ssa_jit_bwd_var_gen(ssa::WorkList wl) {
    ssa::RegPolicy p;
    ssa::sim_loop<ssa::kBwd, ssa_gen::Net::M, false, ssa::RegPolicy, true, true>(wl, p);
}

// The backward in generations with a second wave computing the draws (blocks of two
// waves), for launches of about one block per CU.
extern "C" __global__ void __launch_bounds__(2 * ssa::kWave) ssa_jit_bwd_pc(ssa::WorkList wl) {
    __shared__ double ring[2 * 2 * ssa::kPcRows * ssa::kWave];
    __shared__ int32_t ctl[4];
    ssa::RegPolicy p;
    ssa::sim_pc<ssa::kBwd, ssa_gen::Net::M, ssa::RegPolicy>(wl, p, ring, ctl);
}

extern "C" __global__ void __launch_bounds__(2 * ssa::kWave) ssa_jit_bwd_var_pc(ssa::WorkList wl) {
    __shared__ double ring[2 * 2 * ssa::kPcRows * ssa::kWave];
    __shared__ int32_t ctl[4];
    ssa::RegPolicy p;
    ssa::sim_pc<ssa::kBwd, ssa_gen::Net::M, ssa::RegPolicy, true>(wl, p, ring, ctl);
}

// The forward in generations with a drawing wave (blocks of two waves; dynamic LDS: the
// simulating wave's window), for launches of about one block per CU.
extern "C" __global__ void __launch_bounds__(2 * ssa::kWave) ssa_jit_fwd_pc(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    __shared__ double ring[2 * 2 * ssa::kPcRows * ssa::kWave];
    __shared__ unsigned long long kl[2 * ssa::kWave];
    __shared__ int32_t ctl[4];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, false, ssa::RegPolicy, false, true>(wl, p, ssa_win, ring, kl, ctl);
}

extern "C" __global__ void __launch_bounds__(2 * ssa::kWave) ssa_jit_fwd_hist_pc(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    __shared__ double ring[2 * 2 * ssa::kPcRows * ssa::kWave];
    __shared__ unsigned long long kl[2 * ssa::kWave];
    __shared__ int32_t ctl[4];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, true, ssa::RegPolicy, false, true>(wl, p, ssa_win, ring, kl, ctl);
}

// One epoch of a run in epochs of simulation time with a drawing wave, without and with the
// histogram (launches of about one block per CU, such as long horizons over few
// trajectories).
extern "C" __global__ void __launch_bounds__(2 * ssa::kWave) ssa_jit_fwd_epoch_pc(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    __shared__ double ring[2 * 2 * ssa::kPcRows * ssa::kWave];
    __shared__ unsigned long long kl[2 * ssa::kWave];
    __shared__ int32_t ctl[4];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, false, ssa::RegPolicy, false, true, true>(wl, p, ssa_win, ring, kl,
                                                                                            ctl);
}

extern "C" __global__ void __launch_bounds__(2 * ssa::kWave) ssa_jit_fwd_hist_epoch_pc(ssa::WorkList wl) {
    extern __shared__ long long ssa_win[];
    __shared__ double ring[2 * 2 * ssa::kPcRows * ssa::kWave];
    __shared__ unsigned long long kl[2 * ssa::kWave];
    __shared__ int32_t ctl[4];
    ssa::RegPolicy p;
    ssa::sim_fwd_gen<ssa_gen::Net::M, false, false, true, ssa::RegPolicy, false, true, true>(wl, p, ssa_win, ring, kl,
                                                                                           ctl);
}

// The event log (adaptive memory) in generations with a drawing wave, for launches of about
// one block per CU.
extern "C" __global__ void __launch_bounds__(2 * ssa::kWave) ssa_jit_evt_pc(ssa::WorkList wl) {
    __shared__ double ring[2 * 2 * ssa::kPcRows * ssa::kWave];
    __shared__ int32_t ctl[4];
    ssa::RegPolicy p;
    ssa::sim_pc<ssa::kEvt, ssa_gen::Net::M, ssa::RegPolicy>(wl, p, ring, ctl);
}
