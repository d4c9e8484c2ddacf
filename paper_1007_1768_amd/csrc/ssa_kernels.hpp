// ssa_kernels.hpp -- compiled kernels for gfx950: the generic (table-driven) simulation
// kernel used for batched many-network launches, the grid description, the exact
// finalize of the grid moments (slab sum, prefix over the grid, one rounding per moment),
// the histogram prefix and the fixed-order gradient reduction.
//
// The generic policy keeps each lane's species counts in LDS columns x[row * 256 + tid]
// (row 0 is all ones, species s in row s + 1): a propensity reads one uniform row, all 64
// lanes of the wave hit consecutive words (conflict-free), and an update writes only the
// changed rows.  Reactions are evaluated branch-free from a packed encoding,
//   h = (x[a] * max(x[b] - d, 0)) * f,
// with the all-ones row standing in for missing reactants:
//   0 -> ...   a = b = 0,   d = 0, f = 1       A -> ...   a = A+1, b = 0, d = 0, f = 1
//   A + B      a = A+1, b = B+1, d = 0, f = 1  2A -> ...  a = b = A+1, d = 1, f = 1/2
// packed as a | b << 12 | d << 24.  f is 1 or 1/2 and multiplies exactly, so h is the
// integer pair count rounded once, as the contract requires.  The tables are padded with
// zero-rate entries so the unrolled loops need no per-reaction branches.
// Changes of reaction j: kChg slots chg[j * kChg + i] = row | delta << 12 (delta signed,
// |delta| < 2^19); an empty slot is 0.
#pragma once

#include "ssa_sim.hpp"

namespace ssa {

constexpr int32_t kRowBits = 12;
constexpr int kPadReactions = 32;    // generic tables are padded to a multiple of this

__host__ __device__ __forceinline__ int32_t chg_row(int32_t c) { return c & ((1 << kRowBits) - 1); }
__host__ __device__ __forceinline__ int32_t chg_delta(int32_t c) { return c >> kRowBits; }

__device__ __forceinline__ double packed_propensity(uint32_t code, double c, const int32_t *xc) {
    const int32_t ra = (int32_t)(code & 0xfffu), rb = (int32_t)((code >> 12) & 0xfffu);
    const int32_t d = (int32_t)(code >> 24);
    const int32_t xa = xc[ra * kBlock];
    const int32_t xb = max(xc[rb * kBlock] - d, 0);
    const double f = d ? 0.5 : 1.0;
    return c * (((double)xa * (double)xb) * f);
}

struct LdsPolicy {
    int32_t *xc;      // this lane's column: row r at xc[r * kBlock]
    int32_t *wchg;    // this wave's change table
    int32_t S;

    __device__ void switch_net(const NetDev &n) {
        const uint32_t lane = __lane_id();
        for (int32_t q = lane; q < n.M * kChg; q += kWave) wchg[q] = n.chg[q];
        S = wave_uniform(n.S);
    }
    __device__ void reset(const NetDev &n) {
        const SSA_CONST int32_t *x0 = (const SSA_CONST int32_t *)n.x0;
        for (int32_t s = 0; s < S; ++s) xc[(s + 1) * kBlock] = x0[s];
    }
    __device__ void load_state(const int32_t *src) {
        for (int32_t s = 0; s < S; ++s) xc[(s + 1) * kBlock] = src[s];
    }
    template <int MM>
    __device__ __forceinline__ void eval(const NetDev &n, double (&a)[MM]) const {
        const SSA_CONST uint32_t *rx = (const SSA_CONST uint32_t *)n.rx;
        const SSA_CONST double *rate = (const SSA_CONST double *)n.rate;
#pragma unroll
        for (int j = 0; j < MM; ++j) a[j] = packed_propensity(rx[j], rate[j], xc);
    }
    __device__ double one(const NetDev &n, int32_t j) const {
        return packed_propensity(((const SSA_CONST uint32_t *)n.rx)[j], ((const SSA_CONST double *)n.rate)[j], xc);
    }
    __device__ double total(const NetDev &n) const {
        const SSA_CONST uint32_t *rx = (const SSA_CONST uint32_t *)n.rx;
        const SSA_CONST double *rate = (const SSA_CONST double *)n.rate;
        double acc = packed_propensity(rx[0], rate[0], xc);
        for (int32_t j = 1; j < n.M; ++j) acc = acc + packed_propensity(rx[j], rate[j], xc);
        return acc;
    }
    // count of partial sums S_j <= u, recomputing S_j exactly as total() did
    __device__ int32_t select(const NetDev &n, double u) const {
        const SSA_CONST uint32_t *rx = (const SSA_CONST uint32_t *)n.rx;
        const SSA_CONST double *rate = (const SSA_CONST double *)n.rate;
        double acc = packed_propensity(rx[0], rate[0], xc);
        int32_t cnt = acc <= u ? 1 : 0;
        for (int32_t j = 1; j < n.M; ++j) {
            acc = acc + packed_propensity(rx[j], rate[j], xc);
            cnt += acc <= u ? 1 : 0;
        }
        return cnt;
    }
    template <class F>
    __device__ __forceinline__ void for_each_species(F f) const {
        for (int32_t s = 0; s < S; ++s) f(s, xc[(s + 1) * kBlock]);
    }
    template <class F>
    __device__ __forceinline__ void apply(const NetDev &, int32_t sel, F f) {
        const int4 cq = *(const int4 *)(wchg + sel * kChg);
        const int32_t cs[kChg] = {cq.x, cq.y, cq.z, cq.w};
#pragma unroll
        for (int q = 0; q < kChg; ++q) {
            const int32_t r = chg_row(cs[q]), dl = chg_delta(cs[q]);
            if (dl == 0) continue;
            const int32_t xo = xc[r * kBlock];
            const int32_t xn = xo + dl;
            xc[r * kBlock] = xn;
            f(r - 1, xo, xn);
        }
    }
};

// LDS per block: rows [s_rows + 1][kBlock] int32 (row 0 all ones, species s in row s + 1),
// then one change table per wave of m_rows * kChg int32, then (forward) kCohorts selective-
// memory windows per wave of win_words int64 each.
__device__ __forceinline__ void generic_setup(const WorkList &wl, int32_t *lds, LdsPolicy &p) {
    p.xc = lds + threadIdx.x;
    p.wchg = lds + (wl.s_rows + 1) * kBlock + (threadIdx.x / kWave) * wl.m_rows * kChg;
    p.S = 0;
    p.xc[0] = 1;
}

__host__ __device__ __forceinline__ size_t generic_int_words(int32_t s_rows, int32_t m_rows) {
    const size_t w = (size_t)(s_rows + 1) * kBlock + (size_t)(kBlock / kWave) * m_rows * kChg;
    return (w + 1) & ~(size_t)1;   // 8-byte alignment of the windows that follow
}

template <int MODE, int MM, bool BATCH, bool QUAD = false>
__global__ void __launch_bounds__(kBlock) sim_kernel(WorkList wl) {
    extern __shared__ int32_t lds_x[];
    LdsPolicy p;
    generic_setup(wl, lds_x, p);
    sim_loop<MODE, MM, BATCH, LdsPolicy, QUAD>(wl, p);
}

template <int MM, bool BATCH, bool SLAB>
__global__ void __launch_bounds__(kBlock) fwd_kernel(WorkList wl) {
    extern __shared__ int32_t lds_x[];
    LdsPolicy p;
    generic_setup(wl, lds_x, p);
    long long *win = (long long *)(lds_x + generic_int_words(wl.s_rows, wl.m_rows)) +
                     (size_t)(threadIdx.x / kWave) * kCohorts * wl.win_words;
    sim_fwd<MM, BATCH, SLAB>(wl, p, win);
}

// Backward prefix table.  With c_g = sum_s w_gs mhat_gs the per-crossing weight is
// phi_g = sum_s w_gs x_s - c_g, so the sums a backward interval needs over its crossings
// g in [ga, gb),
//   alpha = sum phi_g = sum_s x_s dW_s - dC,
//   beta  = sum phi_g (t_g - t) = sum_s x_s (dWT_s - t dW_s) - (dCT - t dC),
// come from differences of prefix sums (over g' < g) of the 2S + 2 columns
//   W_s = w_gs,  WT_s = w_gs t_g,  C = c_g,  CT = c_g t_g.
// With variance weights wv and centring vhat the weight is quadratic in x,
//   phi_g = sum_s [w (x - mhat) + wv ((x - mhat)^2 - vhat)]
//         = sum_s [(w - 2 wv mhat) x + wv x^2] - sum_s [w mhat + wv (vhat - mhat^2)],
// so W_s becomes w - 2 wv mhat, c_g the second sum, and 2S more columns follow:
//   Q_s = wv_gs,  QT_s = wv_gs t_g   (4S + 2 in all).
// The prefixes are kept as unevaluated double-double sums (hi + lo), so a difference of
// two rows loses nothing to cancellation.  Row g (0 <= g <= G) holds the hi parts of the
// columns (binary64) followed by their lo parts (binary32), see PrefixRow.
__device__ __forceinline__ double bwd_column(const double *w, const double *mhat, const double *wv,
                                             const double *vhat, const double *grid, int32_t S, int32_t g,
                                             int32_t k) {
    if (k < 2 * S) {
        const int32_t s = k < S ? k : k - S;
        double v = w[(size_t)g * S + s];
        if (wv) v = v - 2.0 * wv[(size_t)g * S + s] * mhat[(size_t)g * S + s];
        return k < S ? v : v * grid[g];
    }
    if (k >= 2 * S + 2) {
        const int32_t s = k < 3 * S + 2 ? k - (2 * S + 2) : k - (3 * S + 2);
        const double v = wv[(size_t)g * S + s];
        return k < 3 * S + 2 ? v : v * grid[g];
    }
    double c = 0.0;
    for (int32_t s = 0; s < S; ++s) {
        const double m = mhat[(size_t)g * S + s];
        c = c + w[(size_t)g * S + s] * m;
        if (wv) c = c + wv[(size_t)g * S + s] * (vhat[(size_t)g * S + s] - m * m);
    }
    return k == 2 * S ? c : c * grid[g];
}

// One block of 256 threads per column: chunked double-double sums, a scan of the chunk
// totals, then the prefix rows.
__global__ void __launch_bounds__(256) bwd_prefix_kernel(const double *__restrict__ w,
                                                         const double *__restrict__ mhat,
                                                         const double *__restrict__ wv,
                                                         const double *__restrict__ vhat,
                                                         const double *__restrict__ grid, int32_t G, int32_t S,
                                                         void *__restrict__ P, double *__restrict__ PT) {
    const int32_t k = blockIdx.x, ncol = wv ? 4 * S + 2 : 2 * S + 2;
    auto hi = [&](int32_t g) { return (double *)((char *)P + (size_t)g * 12 * ncol); };
    auto lo = [&](int32_t g) { return (float *)((char *)P + (size_t)g * 12 * ncol + 8 * (size_t)ncol); };
    const int32_t nt = blockDim.x, per = (G + nt - 1) / nt;
    const int32_t g0 = min(G, (int32_t)threadIdx.x * per), g1 = min(G, g0 + per);
    double h = 0.0, l = 0.0;
    for (int32_t g = g0; g < g1; ++g) dd_add(h, l, bwd_column(w, mhat, wv, vhat, grid, S, g, k), 0.0);
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = h;
    sh[1][threadIdx.x] = l;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        double ph = 0.0, pl = 0.0;
        if ((int)threadIdx.x >= off) {
            ph = sh[0][threadIdx.x - off];
            pl = sh[1][threadIdx.x - off];
        }
        __syncthreads();
        if ((int)threadIdx.x >= off) {
            double a = sh[0][threadIdx.x], b = sh[1][threadIdx.x];
            dd_add(a, b, ph, pl);
            sh[0][threadIdx.x] = a;
            sh[1][threadIdx.x] = b;
        }
        __syncthreads();
    }
    // exclusive start of this chunk
    h = threadIdx.x ? sh[0][threadIdx.x - 1] : 0.0;
    l = threadIdx.x ? sh[1][threadIdx.x - 1] : 0.0;
    if (threadIdx.x == 0) {
        hi(0)[k] = 0.0;
        lo(0)[k] = 0.0f;
    }
    for (int32_t g = g0; g < g1; ++g) {
        const double v = bwd_column(w, mhat, wv, vhat, grid, S, g, k);
        if (PT) PT[(size_t)g * ncol + k] = v;    // the point's own row, for one-crossing intervals
        dd_add(h, l, v, 0.0);
        hi(g + 1)[k] = h;
        lo(g + 1)[k] = (float)l;
    }
}

// A run whose inputs fail the device-side checks (grid or log rates) is refused on the
// device: the check sets this bit in the run's status word and moves the work counter to
// kRefusedItem, so every simulation kernel finds no work item and exits through its normal
// path, and the finalize kernels write NaN (all-ones histogram counts) instead of results.
// The host reports SSA_E_INVALID when it reads the status word.
constexpr uint32_t kFlagRefused = 8u;
constexpr unsigned int kRefusedItem = 0x7f000000u;   // above any work-item count the library accepts

__device__ __forceinline__ bool refused(const unsigned long long *flags) {
    return flags && (*(const volatile unsigned long long *)flags & kFlagRefused);
}

// The exact integer sums hold every event's change of x and its low part of (2x + nu) nu
// (below 2^24) in int64 words and running prefixes, exact up to 2^39 events per run; a run
// with more events is refused at its finalize (NaN moments, this bit in the status word).
constexpr uint32_t kFlagTooManyEvents = 16u;
constexpr unsigned long long kMaxExactEvents = 1ull << 39;

// status: the run's words (events, largest step count, flags).  True when the finalize must
// write NaN: the run was refused, or it applied too many events for exact sums (flagged here).
__device__ __forceinline__ bool finalize_refused(const unsigned long long *status) {
    if (!status) return false;
    if (refused(status + 2)) return true;
    if (*(const volatile unsigned long long *)status >= kMaxExactEvents) {
        if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr((unsigned long long *)status + 2, (unsigned long long)kFlagTooManyEvents);
        return true;
    }
    return false;
}

__device__ __forceinline__ void refuse(unsigned int *counter, unsigned long long *flags) {
    atomicOr(flags, (unsigned long long)kFlagRefused);
    atomicMax(counter, kRefusedItem);
}

// Grid description of a device grid: uniform if t_g == fl(fl(T g) / D) for all g with
// D = G - 1 and T either t_end or t_{G-1} (first that fits), else general; plus the affine
// guess.  The grid must be non-decreasing inside [0, t_end] (Section 3.2.1's time
// alignment is on increasing simulation times): any other grid, NaN included, refuses the
// run (counter and flags: the run's work counter and status word).  One block of 256
// threads.
__global__ void __launch_bounds__(256) grid_info_kernel(const double *__restrict__ grid, int32_t G, double t_end,
                                                        GridInfo *__restrict__ out, unsigned int *__restrict__ counter,
                                                        unsigned long long *__restrict__ flags) {
    __shared__ int bad[3];
    if (threadIdx.x < 3) bad[threadIdx.x] = 0;
    __syncthreads();
    const double D = (double)(G - 1);
    const double Tc[2] = {t_end, grid[G - 1]};
    for (int c = 0; c < 2; ++c) {
        int mine = (G < 2 || !(Tc[c] > 0.0)) ? 1 : 0;
        for (int32_t g = threadIdx.x; g < G && !mine; g += blockDim.x)
            if (grid[g] != (Tc[c] * (double)g) / D) mine = 1;
        if (mine) atomicOr(&bad[c], 1);
    }
    int invalid = 0;
    for (int32_t g = threadIdx.x; g < G && !invalid; g += blockDim.x) {
        const double v = grid[g];
        if (!(v >= 0.0 && v <= t_end) || (g > 0 && !(v >= grid[g - 1]))) invalid = 1;
    }
    if (invalid) atomicOr(&bad[2], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        GridInfo gi;
        gi.uniform = (!bad[0] || !bad[1]) ? 1 : 0;
        gi.T = !bad[0] ? Tc[0] : Tc[1];
        gi.D = D;
        gi.lo = grid[0];
        const double span = grid[G - 1] - grid[0];
        gi.scale = (G > 1 && span > 0.0) ? (double)(G - 1) / span : 0.0;
        gi.pad = 0;
        if (bad[2]) {
            gi.uniform = 1;            // harmless values; no work item runs
            gi.T = 0.0;
            gi.lo = 0.0;
            gi.scale = 0.0;
            if (counter && flags) refuse(counter, flags);
        }
        *out = gi;
    }
}

// Rate constants from log rate constants (the parameters theta_j = ln c_j of the
// likelihood-ratio gradient), c = e^theta with fixed roundings so that the CPU oracle can
// form the same binary64 values:
//   theta < -708 (also -inf): c = 0;  theta > 709 or NaN: invalid;
//   otherwise k = rint(fl(theta * INV_LN2)) (ties to even), r = fma(-k, LN2_LO, fma(-k, LN2_HI, theta)),
//   p = Horner with fma over the Taylor coefficients E_n = fl(1/n!), n = 13 down to 0
//   (p = E_13, then p = fma(p, r, E_n)), and c = p 2^k (exact: k >= -1021, p > 0.7).
// |r| <= ln 2 / 2 + 2^-40, so the degree-13 remainder is below 2^-57 of e^r.
// LN2_HI keeps 32 significant bits (k LN2_HI is exact for |k| < 2^21).
__device__ __forceinline__ double exp_contract(double theta, bool &invalid) {
    invalid = false;
    if (theta < -708.0) return 0.0;
    if (!(theta <= 709.0)) {
        invalid = true;
        return __builtin_nan("");
    }
    constexpr double kInvLn2 = 0x1.71547652b82fep0;
    constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
    constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
    const double k = rint(theta * kInvLn2);
    const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, theta));
    constexpr double E[14] = {1.0,
                              1.0,
                              1.0 / 2.0,
                              1.0 / 6.0,
                              1.0 / 24.0,
                              1.0 / 120.0,
                              1.0 / 720.0,
                              1.0 / 5040.0,
                              1.0 / 40320.0,
                              1.0 / 362880.0,
                              1.0 / 3628800.0,
                              1.0 / 39916800.0,
                              1.0 / 479001600.0,
                              1.0 / 6227020800.0};
    double p = E[13];
#pragma unroll
    for (int n = 12; n >= 0; --n) p = fma(p, r, E[n]);
    return ldexp(p, (int)k);
}

// c[j] = exp_contract(theta[j]) for j < M and 0 for M <= j < m_pad (the table-driven kernels
// read zero-padded rate tables); an invalid theta refuses the run.
__global__ void rates_from_log_kernel(const double *__restrict__ theta, int32_t M, int32_t m_pad,
                                      double *__restrict__ c, unsigned int *__restrict__ counter,
                                      unsigned long long *__restrict__ flags) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_pad) return;
    bool invalid = false;
    c[j] = j < M ? exp_contract(theta[j], invalid) : 0.0;
    if (invalid && counter && flags) refuse(counter, flags);
    if (invalid && flags && !counter) atomicOr(flags, (unsigned long long)kFlagRefused);
}

// ---------------------------------------------------------------------------------------
// Finalize: exact integer totals of sum x and sum x^2 at every grid point, then the
// moments.
// ---------------------------------------------------------------------------------------

// 128-bit two's-complement helpers (hi:lo).
struct i128s { uint64_t lo; int64_t hi; };

__device__ __forceinline__ i128s i128_from(int64_t v) { return i128s{(uint64_t)v, v < 0 ? -1 : 0}; }
__device__ __forceinline__ i128s i128_add(i128s x, i128s y) {
    i128s r;
    r.lo = x.lo + y.lo;
    r.hi = x.hi + y.hi + (r.lo < x.lo ? 1 : 0);
    return r;
}
__device__ __forceinline__ i128s i128_neg(i128s x) {
    i128s r;
    r.lo = ~x.lo + 1;
    r.hi = ~x.hi + (r.lo == 0 ? 1 : 0);
    return r;
}
// unsigned 64 x signed 128 -> signed 128 (low 128 bits; callers stay in range)
__device__ __forceinline__ i128s i128_mul_u64(i128s x, uint64_t m) {
    i128s r;
    r.lo = x.lo * m;
    r.hi = (int64_t)(__umul64hi(x.lo, m) + (uint64_t)x.hi * m);
    return r;
}
__device__ __forceinline__ i128s i128_sq(int64_t v) {
    const uint64_t a = (uint64_t)(v < 0 ? -v : v);
    i128s r;
    r.lo = a * a;
    r.hi = (int64_t)__umul64hi(a, a);
    return r;
}
// round-to-nearest conversion of a signed 128-bit integer to binary64
__device__ __forceinline__ double i128_to_double(i128s x) {
    bool neg = x.hi < 0;
    if (neg) x = i128_neg(x);
    const uint64_t hi = (uint64_t)x.hi, lo = x.lo;
    double r;
    if (hi == 0) {
        r = (double)lo;
    } else {
        // keep 64 significant bits with a sticky bit, then one rounding by the conversion
        if ((int64_t)hi < 0) {           // 2^127 and above: out of the range used here
            r = __builtin_ldexp((double)hi, 64);
            return neg ? -r : r;
        }
        const int lz = __clzll(hi);
        const int sh = 64 - lz;                       // bits of hi that are used
        const uint64_t top = (hi << lz) | (lo >> sh);
        const uint64_t sticky = (lo << lz) != 0 ? 1u : 0u;
        // top has 64 bits; fold the sticky bit into its lowest bit (below the 53 kept)
        r = __builtin_ldexp((double)(top | sticky), sh);
    }
    return neg ? -r : r;
}

// Sum of the wave-private slabs: out[q] = sum over slabs of slabs[slab * words + q].
__global__ void slab_reduce_kernel(const unsigned long long *__restrict__ slabs, int64_t n_slabs, int64_t words,
                                   unsigned long long *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= words) return;
    unsigned long long acc = 0;
    for (int64_t k = 0; k < n_slabs; ++k) acc += slabs[k * words + q];
    out[q] = acc;
}

// One block per species: inclusive prefix over the grid of the difference sums
// D[g][s] = (sum nu, low sum (2x+nu)nu) and Dhi[g][s] (high parts, scaled by 2^24), giving
// the exact totals
//   Sx = N x0 + prefix(nu),   Sx2 = N x0^2 + prefix(low) + 2^24 prefix(high)
// and from them the moments with one rounding each:
//   mean = Sx / N,   var = (N Sx2 - Sx^2) / (N (N - 1))  (0 when N == 1).
// Optionally also writes the totals as (Sx hi, Sx lo, Sx2 hi, Sx2 lo) 128-bit pairs.
// Mean and variance of one (point, species) from its exact totals, one rounding each.
__device__ __forceinline__ void moment_point(int64_t sx, const i128s &sx2, int64_t n_traj, double dn, double dd,
                                             double *mean, double *var) {
    *mean = (double)sx / dn;
    if (n_traj == 1) {
        *var = 0.0;
    } else {
        const i128s num = i128_add(i128_mul_u64(sx2, (uint64_t)n_traj), i128_neg(i128_sq(sx)));
        *var = i128_to_double(num) / dd;
    }
}

__device__ __forceinline__ void moment_final_body(const unsigned long long *__restrict__ D,
                                                  const unsigned long long *__restrict__ Dhi, int32_t G, int32_t S,
                                                  int32_t s, const int32_t *__restrict__ x0, int64_t n_traj,
                                                  double *__restrict__ mean, double *__restrict__ var,
                                                  int64_t *__restrict__ sums) {
    const int32_t nt = blockDim.x;
    const int32_t per = (G + nt - 1) / nt;
    const int32_t g0 = min(G, (int32_t)threadIdx.x * per), g1 = min(G, g0 + per);
    int64_t s1 = 0, s2 = 0, s3 = 0;
    for (int32_t g = g0; g < g1; ++g) {
        s1 += (int64_t)D[((size_t)g * S + s) * 2];
        s2 += (int64_t)D[((size_t)g * S + s) * 2 + 1];
        s3 += (int64_t)Dhi[(size_t)g * S + s];
    }
    __shared__ int64_t sh[3][1024];
    sh[0][threadIdx.x] = s1;
    sh[1][threadIdx.x] = s2;
    sh[2][threadIdx.x] = s3;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        int64_t v1 = 0, v2 = 0, v3 = 0;
        if ((int)threadIdx.x >= off) {
            v1 = sh[0][threadIdx.x - off];
            v2 = sh[1][threadIdx.x - off];
            v3 = sh[2][threadIdx.x - off];
        }
        __syncthreads();
        sh[0][threadIdx.x] += v1;
        sh[1][threadIdx.x] += v2;
        sh[2][threadIdx.x] += v3;
        __syncthreads();
    }
    int64_t c1 = sh[0][threadIdx.x] - s1, c2 = sh[1][threadIdx.x] - s2, c3 = sh[2][threadIdx.x] - s3;
    const int64_t xs = x0[s];
    const int64_t base1 = n_traj * xs;
    const i128s base2 = i128_mul_u64(i128_sq(xs), (uint64_t)n_traj);
    const double dn = (double)n_traj;
    const double dd = dn * (double)(n_traj - 1);
    for (int32_t g = g0; g < g1; ++g) {
        c1 += (int64_t)D[((size_t)g * S + s) * 2];
        c2 += (int64_t)D[((size_t)g * S + s) * 2 + 1];
        c3 += (int64_t)Dhi[(size_t)g * S + s];
        const int64_t sx = base1 + c1;
        const i128s sx2 = i128_add(i128_add(base2, i128_from(c2)), i128_mul_u64(i128_from(c3), 1ull << 24));
        const size_t q = (size_t)g * S + s;
        moment_point(sx, sx2, n_traj, dn, dd, mean + q, var + q);
        if (sums) {
            sums[4 * q + 0] = sx < 0 ? -1 : 0;
            sums[4 * q + 1] = sx;
            sums[4 * q + 2] = sx2.hi;
            sums[4 * q + 3] = (int64_t)sx2.lo;
        }
    }
}

// One block of 1024 threads per species.
__global__ void __launch_bounds__(1024) moment_final_kernel(const unsigned long long *__restrict__ D,
                                                            const unsigned long long *__restrict__ Dhi, int32_t G,
                                                            int32_t S, const int32_t *__restrict__ x0,
                                                            int64_t n_traj, double *__restrict__ mean,
                                                            double *__restrict__ var, int64_t *__restrict__ sums,
                                                            const unsigned long long *__restrict__ status) {
    if (finalize_refused(status)) {
        const int32_t s = blockIdx.x;
        for (int32_t g = threadIdx.x; g < G; g += blockDim.x) {
            mean[(size_t)g * S + s] = __builtin_nan("");
            var[(size_t)g * S + s] = __builtin_nan("");
        }
        return;
    }
    moment_final_body(D, Dhi, G, S, blockIdx.x, x0, n_traj, mean, var, sums);
}

// The same finalize for long point sequences (the adaptive selective memory's Avg-Y), over
// many blocks: chunks of kFinChunk points per block.  A block takes up to kFinGroup species
// per pass over its chunk, reading each point's slice of those species at once: a point's
// S entries share cache lines, and a chunk (96 KB at four species) does not stay in L2 from
// one species to the next while every CU streams its own chunks.
// Step 1: the chunk totals of the three difference sums.
constexpr int kFinChunk = 1024;
constexpr int kFinGroup = 4;

__device__ __forceinline__ void chunk_total_group(const unsigned long long *__restrict__ D,
                                                  const unsigned long long *__restrict__ Dhi, int64_t G, int32_t S,
                                                  long long *__restrict__ T, int64_t c, int32_t s0, int32_t ns) {
    const int64_t g0 = c * kFinChunk, g1 = min(g0 + kFinChunk, G);
    int64_t a[3][kFinGroup];
#pragma unroll
    for (int q = 0; q < kFinGroup; ++q) a[0][q] = a[1][q] = a[2][q] = 0;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
        const unsigned long long *d = D + ((size_t)g * S + s0) * 2;
        const unsigned long long *h = Dhi + (size_t)g * S + s0;
#pragma unroll
        for (int q = 0; q < kFinGroup; ++q) {
            if (q < ns) {
                a[0][q] += (int64_t)d[2 * q];
                a[1][q] += (int64_t)d[2 * q + 1];
                a[2][q] += (int64_t)h[q];
            }
        }
    }
    __shared__ int64_t sh[3 * kFinGroup][256];
#pragma unroll
    for (int q = 0; q < kFinGroup; ++q)
        for (int i = 0; i < 3; ++i) sh[i * kFinGroup + q][threadIdx.x] = a[i][q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int v = 0; v < 3 * kFinGroup; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + off];
        __syncthreads();
    }
    if ((int)threadIdx.x < 3 * ns) {
        const int32_t i = threadIdx.x / ns, q = threadIdx.x - i * ns;
        T[((size_t)c * S + s0 + q) * 3 + i] = sh[i * kFinGroup + q][0];
    }
}

__global__ void __launch_bounds__(256) chunk_total_kernel(const unsigned long long *__restrict__ D,
                                                          const unsigned long long *__restrict__ Dhi, int64_t G,
                                                          int32_t S, long long *__restrict__ T) {
    for (int32_t s0 = 0; s0 < S; s0 += kFinGroup) {
        chunk_total_group(D, Dhi, G, S, T, blockIdx.x, s0, min(kFinGroup, S - s0));
        __syncthreads();                // the shared sums are reused by the next group
    }
}

// Step 2: exclusive prefix of the chunk totals per species (one block per species),
// starting from carry[s][3] (the sums of earlier epochs; NULL = 0), whose entries are then
// advanced to include this call's totals.
__global__ void __launch_bounds__(1024) chunk_scan_kernel(long long *__restrict__ T, int64_t n_chunks, int32_t S,
                                                          long long *__restrict__ carry) {
    const int32_t s = blockIdx.x;
    const int64_t per = (n_chunks + blockDim.x - 1) / blockDim.x;
    const int64_t c0 = min(n_chunks, (int64_t)threadIdx.x * per), c1 = min(n_chunks, c0 + per);
    int64_t a[3] = {0, 0, 0};
    for (int64_t c = c0; c < c1; ++c)
        for (int i = 0; i < 3; ++i) a[i] += T[((size_t)c * S + s) * 3 + i];
    __shared__ int64_t sh[3][1024];
    for (int i = 0; i < 3; ++i) sh[i][threadIdx.x] = a[i];
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        int64_t v[3] = {0, 0, 0};
        if ((int)threadIdx.x >= off)
            for (int i = 0; i < 3; ++i) v[i] = sh[i][threadIdx.x - off];
        __syncthreads();
        for (int i = 0; i < 3; ++i) sh[i][threadIdx.x] += v[i];
        __syncthreads();
    }
    int64_t base[3] = {0, 0, 0};
    if (carry)
        for (int i = 0; i < 3; ++i) base[i] = carry[(size_t)s * 3 + i];
    int64_t run[3];
    for (int i = 0; i < 3; ++i) run[i] = base[i] + sh[i][threadIdx.x] - a[i];
    for (int64_t c = c0; c < c1; ++c)
        for (int i = 0; i < 3; ++i) {
            const int64_t v = T[((size_t)c * S + s) * 3 + i];
            T[((size_t)c * S + s) * 3 + i] = run[i];
            run[i] += v;
        }
    __syncthreads();   // every thread has read base before the carry moves on
    if (carry && threadIdx.x == blockDim.x - 1)
        for (int i = 0; i < 3; ++i) carry[(size_t)s * 3 + i] = base[i] + sh[i][threadIdx.x];
}

// Step 3: within each chunk, the inclusive prefix (4 points per thread, then a block scan)
// plus the chunk's offset and the initial-state terms, then the moments per point, for up
// to kFinGroup species per pass.
__device__ __forceinline__ void chunk_final_group(const unsigned long long *__restrict__ D,
                                                  const unsigned long long *__restrict__ Dhi, int64_t G, int32_t S,
                                                  const long long *__restrict__ T, const int32_t *__restrict__ x0,
                                                  int64_t n_traj, double *__restrict__ mean, double *__restrict__ var,
                                                  int64_t c, int32_t s0, int32_t ns) {
    static_assert(kFinChunk == 4 * 256, "four points per thread");
    const int64_t g0 = c * kFinChunk + 4 * (int64_t)threadIdx.x;
    int64_t v[4][3][kFinGroup];
    int64_t a[3][kFinGroup];
#pragma unroll
    for (int q = 0; q < kFinGroup; ++q) a[0][q] = a[1][q] = a[2][q] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t g = g0 + k;
        const unsigned long long *d = D + ((size_t)g * S + s0) * 2;
        const unsigned long long *h = Dhi + (size_t)g * S + s0;
#pragma unroll
        for (int q = 0; q < kFinGroup; ++q) {
            const bool in = g < G && q < ns;
            v[k][0][q] = in ? (int64_t)d[2 * q] : 0;
            v[k][1][q] = in ? (int64_t)d[2 * q + 1] : 0;
            v[k][2][q] = in ? (int64_t)h[q] : 0;
            a[0][q] += v[k][0][q];
            a[1][q] += v[k][1][q];
            a[2][q] += v[k][2][q];
        }
    }
    // inclusive block scan of the per-thread sums (3 per species)
    __shared__ int64_t sh[3 * kFinGroup][256];
#pragma unroll
    for (int q = 0; q < kFinGroup; ++q)
        for (int i = 0; i < 3; ++i) sh[i * kFinGroup + q][threadIdx.x] = a[i][q];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int64_t u[3 * kFinGroup];
#pragma unroll
        for (int x = 0; x < 3 * kFinGroup; ++x) u[x] = (int)threadIdx.x >= off ? sh[x][threadIdx.x - off] : 0;
        __syncthreads();
#pragma unroll
        for (int x = 0; x < 3 * kFinGroup; ++x) sh[x][threadIdx.x] += u[x];
        __syncthreads();
    }
    const double dn = (double)n_traj;
    const double dd = dn * (double)(n_traj - 1);
#pragma unroll
    for (int q = 0; q < kFinGroup; ++q) {
        if (q >= ns) continue;
        const int32_t s = s0 + q;
        int64_t c1 = T[((size_t)c * S + s) * 3 + 0] + sh[0 * kFinGroup + q][threadIdx.x] - a[0][q];
        int64_t c2 = T[((size_t)c * S + s) * 3 + 1] + sh[1 * kFinGroup + q][threadIdx.x] - a[1][q];
        int64_t c3 = T[((size_t)c * S + s) * 3 + 2] + sh[2 * kFinGroup + q][threadIdx.x] - a[2][q];
        const int64_t xs = x0[s];
        const int64_t base1 = n_traj * xs;
        const i128s base2 = i128_mul_u64(i128_sq(xs), (uint64_t)n_traj);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t g = g0 + k;
            c1 += v[k][0][q];
            c2 += v[k][1][q];
            c3 += v[k][2][q];
            if (g < G) {
                const int64_t sx = base1 + c1;
                const i128s sx2 = i128_add(i128_add(base2, i128_from(c2)), i128_mul_u64(i128_from(c3), 1ull << 24));
                moment_point(sx, sx2, n_traj, dn, dd, mean + (size_t)g * S + s, var + (size_t)g * S + s);
            }
        }
    }
}

__global__ void __launch_bounds__(256) chunk_final_kernel(const unsigned long long *__restrict__ D,
                                                          const unsigned long long *__restrict__ Dhi, int64_t G,
                                                          int32_t S, const long long *__restrict__ T,
                                                          const int32_t *__restrict__ x0, int64_t n_traj,
                                                          double *__restrict__ mean, double *__restrict__ var) {
    for (int32_t s0 = 0; s0 < S; s0 += kFinGroup) {
        chunk_final_group(D, Dhi, G, S, T, x0, n_traj, mean, var, blockIdx.x, s0, min(kFinGroup, S - s0));
        __syncthreads();                // the shared scan is reused by the next group
    }
}

// Covariance finalize, step 1: one block per column c of the cross-product rows
// (c < S: species c, its sum of nu, low and high parts of (2x+nu)nu; c >= S: pair c - S,
// low and high parts of the x_s x_r differences); exact inclusive prefixes over the grid
// plus the initial-state terms give sx[g][s] (int64) and sxx[g][c] (128-bit).
__global__ void __launch_bounds__(1024) cov_prefix_kernel(const unsigned long long *__restrict__ D,
                                                          const unsigned long long *__restrict__ Dhi, int32_t G,
                                                          int32_t S, const int32_t *__restrict__ x0, int64_t n_traj,
                                                          int64_t *__restrict__ sx, i128s *__restrict__ sxx) {
    const int32_t c = blockIdx.x, npairs = S * (S - 1) / 2, row = 2 * S + npairs, hrow = S + npairs;
    int32_t ps = c, pr = c;             // the pair's species (for the initial-state term)
    if (c >= S) {
        int32_t q = c - S, a = 0;
        while (q >= S - a - 1) { q -= S - a - 1; ++a; }
        ps = a;
        pr = a + 1 + q;
    }
    const int32_t lo_col = c < S ? 2 * c + 1 : 2 * S + (c - S);
    const int32_t nt = blockDim.x, per = (G + nt - 1) / nt;
    const int32_t g0 = min(G, (int32_t)threadIdx.x * per), g1 = min(G, g0 + per);
    int64_t s1 = 0, s2 = 0, s3 = 0;
    for (int32_t g = g0; g < g1; ++g) {
        if (c < S) s1 += (int64_t)D[(size_t)g * row + 2 * c];
        s2 += (int64_t)D[(size_t)g * row + lo_col];
        s3 += (int64_t)Dhi[(size_t)g * hrow + c];
    }
    __shared__ int64_t sh[3][1024];
    sh[0][threadIdx.x] = s1;
    sh[1][threadIdx.x] = s2;
    sh[2][threadIdx.x] = s3;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        int64_t v1 = 0, v2 = 0, v3 = 0;
        if ((int)threadIdx.x >= off) {
            v1 = sh[0][threadIdx.x - off];
            v2 = sh[1][threadIdx.x - off];
            v3 = sh[2][threadIdx.x - off];
        }
        __syncthreads();
        sh[0][threadIdx.x] += v1;
        sh[1][threadIdx.x] += v2;
        sh[2][threadIdx.x] += v3;
        __syncthreads();
    }
    int64_t c1 = sh[0][threadIdx.x] - s1, c2 = sh[1][threadIdx.x] - s2, c3 = sh[2][threadIdx.x] - s3;
    const int64_t xs = x0[ps], xr = x0[pr];
    i128s init = i128_from(xs * xr);                     // |x0| < 2^31: the product fits int64
    init = i128_mul_u64(init, (uint64_t)n_traj);
    for (int32_t g = g0; g < g1; ++g) {
        if (c < S) c1 += (int64_t)D[(size_t)g * row + 2 * c];
        c2 += (int64_t)D[(size_t)g * row + lo_col];
        c3 += (int64_t)Dhi[(size_t)g * hrow + c];
        if (c < S) sx[(size_t)g * S + c] = n_traj * xs + c1;
        sxx[(size_t)g * hrow + c] = i128_add(i128_add(init, i128_from(c2)), i128_mul_u64(i128_from(c3), 1ull << 24));
    }
}

// Covariance finalize, step 2: one thread per (g, s, r):
//   cov = fl(N sxx - sx_s sx_r) / (N (N - 1)),  0 when N == 1; mean[g][s] from sx.
__global__ void cov_final_kernel(const int64_t *__restrict__ sx, const i128s *__restrict__ sxx, int32_t G, int32_t S,
                                 int64_t n_traj, double *__restrict__ mean, double *__restrict__ cov,
                                 const unsigned long long *__restrict__ status) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)G * S * S) return;
    const int32_t r = (int32_t)(idx % S), s = (int32_t)((idx / S) % S);
    const int64_t g = idx / ((int64_t)S * S);
    if (finalize_refused(status)) {
        if (s == r) mean[g * S + s] = __builtin_nan("");
        cov[idx] = __builtin_nan("");
        return;
    }
    const int32_t npairs = S * (S - 1) / 2, hrow = S + npairs;
    int32_t c = s;
    if (s != r) {
        const int32_t lo = min(s, r), hi = max(s, r);
        c = S + lo * (2 * S - lo - 1) / 2 + (hi - lo - 1);
    }
    const int64_t a = sx[g * S + s], b = sx[g * S + r];
    if (s == r) mean[g * S + s] = (double)a / (double)n_traj;
    if (n_traj == 1) {
        cov[idx] = 0.0;
        return;
    }
    // N sxx - a b in 128 bits: a b as a signed 128-bit product
    const bool neg = (a < 0) != (b < 0);
    const uint64_t ua = (uint64_t)(a < 0 ? -a : a), ub = (uint64_t)(b < 0 ? -b : b);
    i128s ab;
    ab.lo = ua * ub;
    ab.hi = (int64_t)__umul64hi(ua, ub);
    if (neg) ab = i128_neg(ab);
    const i128s num = i128_add(i128_mul_u64(sxx[g * hrow + c], (uint64_t)n_traj), i128_neg(ab));
    cov[idx] = i128_to_double(num) / ((double)n_traj * (double)(n_traj - 1));
}

// Finalize of every network of a batch in one launch: block i handles species
// block_species[i] of network block_net[i].
struct FinalNet {
    const unsigned long long *D, *Dhi;
    const int32_t *x0;
    double *mean, *var;
    int64_t n_traj;
    int32_t G, S;
};

__global__ void __launch_bounds__(1024) moment_final_batched_kernel(const FinalNet *__restrict__ nets,
                                                                    const int32_t *__restrict__ block_net,
                                                                    const int32_t *__restrict__ block_species) {
    const FinalNet f = nets[block_net[blockIdx.x]];
    moment_final_body(f.D, f.Dhi, f.G, f.S, block_species[blockIdx.x], f.x0, f.n_traj, f.mean, f.var, nullptr);
}

// Likelihood-ratio Jacobian from the per-item slabs [items][G][S+1][M] (row S holds the
// score sums): J[g][s][j] = F/N - mean[g][s] Z/N with F and Z summed over the items in
// order.  One thread per (g, s, j).
__global__ void jacobian_final_kernel(const double *__restrict__ slabs, int64_t n_items, int32_t G, int32_t S,
                                      int32_t M, int64_t n_traj, const double *__restrict__ mean,
                                      double *__restrict__ jac, const unsigned long long *__restrict__ flags) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)G * S * M) return;
    if (refused(flags)) {
        jac[idx] = __builtin_nan("");
        return;
    }
    const int32_t j = (int32_t)(idx % M);
    const int64_t gs = idx / M;
    const int32_t s = (int32_t)(gs % S);
    const int32_t g = (int32_t)(gs / S);
    const size_t item_words = (size_t)G * (S + 1) * M;
    const size_t fo = ((size_t)g * (S + 1) + s) * M + j, zo = ((size_t)g * (S + 1) + S) * M + j;
    double F = 0.0, Z = 0.0;
    for (int64_t it = 0; it < n_items; ++it) {
        F = F + slabs[it * item_words + fo];
        Z = Z + slabs[it * item_words + zo];
    }
    const double dn = (double)n_traj;
    jac[idx] = F / dn - mean[gs] * (Z / dn);
}

// grad_j = sum_{g,s} w[g][s] jac[g][s][j]: one block of 256 threads per j, strided partial
// sums and a fixed tree, so the result does not depend on scheduling.
__global__ void __launch_bounds__(256) jacobian_vjp_kernel(const double *__restrict__ jac,
                                                           const double *__restrict__ w, int64_t cells, int32_t M,
                                                           double *__restrict__ grad) {
    const int32_t j = blockIdx.x;
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < cells; q += blockDim.x) acc = acc + w[q] * jac[q * M + j];
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[j] = sh[0];
}

// Histogram: inclusive prefix over g of the bin differences plus N in the initial bin.
__global__ void hist_prefix_kernel(const int32_t *__restrict__ Hd, int32_t G, int32_t nb, int32_t init_bin,
                                   int64_t n_traj, uint32_t *__restrict__ out,
                                   const unsigned long long *__restrict__ flags) {
    const int32_t bin = blockIdx.x;
    if (refused(flags)) {
        for (int32_t g = threadIdx.x; g < G; g += blockDim.x) out[(size_t)g * nb + bin] = 0xffffffffu;
        return;
    }
    const int32_t nt = blockDim.x;
    const int32_t per = (G + nt - 1) / nt;
    const int32_t g0 = min(G, (int32_t)threadIdx.x * per), g1 = min(G, g0 + per);
    int64_t s = 0;
    for (int32_t g = g0; g < g1; ++g) s += Hd[(size_t)g * nb + bin];
    __shared__ int64_t sh[1024];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        int64_t v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t c = sh[threadIdx.x] - s + (bin == init_bin ? n_traj : 0);
    for (int32_t g = g0; g < g1; ++g) {
        c += Hd[(size_t)g * nb + bin];
        out[(size_t)g * nb + bin] = (uint32_t)c;
    }
}

// Quantiles of the binned distribution at every grid point: for q in (0, 1] the rank is
// k = max(1, ceil(q N)) and the result is the lower edge lo + b width of the first bin b
// whose cumulative count reaches k (with width 1 and no clamping in the top bin, the k-th
// smallest count).  One thread per (grid point, quantile).
__global__ void hist_quantile_kernel(const uint32_t *__restrict__ hist, int32_t G, int32_t nb, int32_t lo,
                                     int32_t width, int64_t n_traj, const double *__restrict__ qs, int32_t nq,
                                     int32_t *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)G * nq) return;
    const int64_t g = idx / nq;
    const double q = qs[idx % nq];
    int64_t k = (int64_t)ceil(q * (double)n_traj);
    k = max(k, (int64_t)1);
    int64_t cum = 0;
    int32_t b = nb - 1;
    for (int32_t i = 0; i < nb; ++i) {
        cum += hist[g * nb + i];
        if (cum >= k) {
            b = i;
            break;
        }
    }
    out[idx] = lo + b * width;
}

// Fixed-order pairwise sum of the per-trajectory gradient rows, then the 1/N scale.  One
// level: out[r][j] = in[2r][j] + in[2r+1][j], an odd last row copied.  A launch applies L
// such levels at once to tiles of 2^L rows in LDS (block (tile, column)): tiles start at
// multiples of 2^L, so no pair crosses a tile and only the last tile sees the odd tails,
// which gives the same sums, in the same order, as L one-level passes.
__global__ void __launch_bounds__(256) pair_sum_kernel(const double *__restrict__ in, int64_t rows, int32_t M,
                                                       int32_t L, double *__restrict__ out) {
    __shared__ double v[256];
    const int64_t t = blockIdx.x;
    const int32_t j = (int32_t)blockIdx.y;
    const int32_t i = (int32_t)threadIdx.x;
    const int64_t r0 = t << L;
    int64_t valid = min((int64_t)1 << L, rows - r0);
    if (i < valid) v[i] = in[(r0 + i) * M + j];
    __syncthreads();
    for (int32_t l = 0; l < L; ++l) {
        const int64_t ov = (valid + 1) / 2;
        double x = 0.0;
        if (i < ov) x = (2 * i + 1 < valid) ? v[2 * i] + v[2 * i + 1] : v[2 * i];
        __syncthreads();
        if (i < ov) v[i] = x;
        __syncthreads();
        valid = ov;
    }
    if (i == 0) out[t * M + j] = v[0];
}

__global__ void scale_kernel(const double *__restrict__ in, int32_t M, double scale, double *__restrict__ out,
                             const unsigned long long *__restrict__ flags) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < M) out[j] = refused(flags) ? __builtin_nan("") : in[j] * scale;
}

// Zero fill with plain stores (kept out of hipMemsetAsync so the launch sequence can be
// captured in a graph).
__global__ void zero_kernel(unsigned long long *__restrict__ p, size_t n_words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void fill_kernel(unsigned long long *__restrict__ p, size_t n_words, unsigned long long v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}


// ---------------------------------------------------------------------------------------
// Inclusive prefix sum of int32 values (n < 2^31, totals below 2^31), in place or not:
// tiles of kScanTile values (16 per thread), the tile totals scanned by one block, then
// every tile scanned with its offset.
// ---------------------------------------------------------------------------------------
constexpr int kScanPer = 16;
constexpr int kScanTile = 256 * kScanPer;

__device__ __forceinline__ int32_t block_excl_scan256(int32_t v, int32_t *sh, int32_t &total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t a = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[255];
    const int32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(256) scan_tile_sums_kernel(const int32_t *__restrict__ in, int64_t n,
                                                             int32_t *__restrict__ sums) {
    __shared__ int32_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) acc += in[base + i];
    int32_t total = 0;
    block_excl_scan256(acc, sh, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the tile totals in place (one block).
__global__ void __launch_bounds__(256) scan_sums_kernel(int32_t *__restrict__ sums, int64_t n_tiles) {
    __shared__ int32_t sh[256];
    int32_t carry = 0;
    for (int64_t base = 0; base < n_tiles; base += 256) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = i < n_tiles ? sums[i] : 0;
        int32_t total = 0;
        const int32_t ex = block_excl_scan256(v, sh, total);
        if (i < n_tiles) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(256) scan_apply_kernel(const int32_t *in, int64_t n,
                                                         const int32_t *__restrict__ sums, int32_t *out) {
    __shared__ int32_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        acc += v[i];
    }
    int32_t total = 0;
    int32_t run = sums[blockIdx.x] + block_excl_scan256(acc, sh, total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        run += v[i];
        if (base + i < n) out[base + i] = run;
    }
}

// ---------------------------------------------------------------------------------------
// Trajectory order of a backward pass.  The backward re-simulates the forward's
// trajectories; a forward in generations records each trajectory's event count, and the
// backward then takes its trajectories longest first, in buckets of similar length
// (len >> shift, shift the smallest that brings the longest below kLenBuckets), so that the
// 64 trajectories of one generation end close together.  Any order gives the same results,
// so the counts are only a hint: a stale one costs time, never bits.
// ---------------------------------------------------------------------------------------
constexpr int32_t kLenBuckets = 4096;

// Copies the counts (the order is built from this private copy, so that a forward writing
// the recorded counts at the same time cannot make it anything but a permutation) and takes
// their maximum.
__global__ void __launch_bounds__(256) len_max_kernel(const uint32_t *__restrict__ len, int64_t n,
                                                      uint32_t *__restrict__ snap, unsigned int *__restrict__ mx) {
    uint32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = len[i];
        snap[i] = v;
        m = max(m, v);
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    __shared__ uint32_t wm[4];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(mx, max(max(wm[0], wm[1]), max(wm[2], wm[3])));   // one atomic per block
}

// Bucket of a length: longest first (bucket 0 holds the longest).
__device__ __forceinline__ int32_t len_bucket(uint32_t v, int32_t shift) {
    return kLenBuckets - 1 - (int32_t)min(v >> shift, (uint32_t)(kLenBuckets - 1));
}

__device__ __forceinline__ int32_t len_shift(uint32_t mx) {
    int32_t s = 0;
    while ((mx >> s) >= (uint32_t)kLenBuckets) ++s;
    return s;
}

// Counting sort by bucket without global atomics: block t takes positions
// [t * tile, (t + 1) * tile) and counts them per bucket in LDS; the counts are stored
// bucket-major (cnt[b * n_tiles + t]), so that their inclusive prefix sum less the count
// is where tile t's positions of bucket b start; the scatter counts again in LDS, each
// position taking the next rank of its bucket in its tile.
__global__ void __launch_bounds__(256) len_count_kernel(const uint32_t *__restrict__ len, int64_t n, int64_t tile,
                                                        const unsigned int *__restrict__ mx,
                                                        int32_t *__restrict__ cnt, int32_t n_tiles) {
    __shared__ int32_t loc[kLenBuckets];
    for (int32_t b = threadIdx.x; b < kLenBuckets; b += blockDim.x) loc[b] = 0;
    __syncthreads();
    const int32_t sh = len_shift(*mx);
    const int64_t lo = (int64_t)blockIdx.x * tile, hi = min(n, lo + tile);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&loc[len_bucket(len[i], sh)], 1);
    __syncthreads();
    for (int32_t b = threadIdx.x; b < kLenBuckets; b += blockDim.x) cnt[(int64_t)b * n_tiles + blockIdx.x] = loc[b];
}

__global__ void __launch_bounds__(256) len_scatter_kernel(const uint32_t *__restrict__ len, int64_t n, int64_t tile,
                                                          const unsigned int *__restrict__ mx,
                                                          const int32_t *__restrict__ cnt,
                                                          const int32_t *__restrict__ incl, int32_t n_tiles,
                                                          uint32_t *__restrict__ perm) {
    __shared__ int32_t loc[kLenBuckets];
    for (int32_t b = threadIdx.x; b < kLenBuckets; b += blockDim.x) loc[b] = 0;
    __syncthreads();
    const int32_t sh = len_shift(*mx);
    const int64_t lo = (int64_t)blockIdx.x * tile, hi = min(n, lo + tile);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const int32_t b = len_bucket(len[i], sh);
        const int64_t j = (int64_t)b * n_tiles + blockIdx.x;
        perm[incl[j] - cnt[j] + atomicAdd(&loc[b], 1)] = (uint32_t)i;
    }
}

// ---------------------------------------------------------------------------------------
// Time order of the event log (adaptive selective memory, Section 3.2.1: the points of all
// trajectories merged by simulation time).  The keys are the bit patterns of the event
// times of one epoch, in [t0, t1] (non-negative binary64 values order like their bits), or
// ~0 for a slot no record took.  A bucket sort by time: bin(t) = floor((t - t0) * scale),
// clamped to [0, B - 1], is monotone in t, so every key of bin b is at most every key of
// bin b + 1; the records are put in bin order (slots without a record last), each bin's
// first position is marked, and then every bin is sorted by key -- by one wave (rank by
// counting) up to 64 records, else by one block (bitonic network with ascending
// comparators only, in LDS up to kBinLds records, in global memory beyond).  Records with
// equal keys end in any order: only the distinct times and the integer sums of their
// records are used.
// ---------------------------------------------------------------------------------------
struct TimeBins {
    double t0, scale;
    int32_t B, pad;
};

constexpr unsigned long long kNoRecord = ~0ull;
constexpr int kBinLds = 2048;

__device__ __forceinline__ int32_t time_bin(const TimeBins &tb, unsigned long long key) {
    const double f = (__longlong_as_double((long long)key) - tb.t0) * tb.scale;
    return f > 0.0 ? (f < (double)tb.B ? (int32_t)f : tb.B - 1) : 0;
}

// The records are first put in bin order by a stable least-significant-digit radix sort on
// the bin index (a slot without a record has bin B, after every bin), kRdxTile records per
// block and pass: rdx_count_kernel counts each tile's digits, their prefix sum in digit-major
// order gives every (digit, tile) its first output position, and rdx_scatter_kernel ranks
// each record within its tile (chunks of 256 in slot order; lanes of one digit matched by
// ballots, so equal digits keep their order), stages the tile in LDS in digit order and
// writes each digit's run contiguously.  No global atomic is taken.
constexpr int kRdxTile = 4096;

__device__ __forceinline__ uint32_t rdx_digit(const TimeBins &tb, unsigned long long k, int32_t shift,
                                              uint32_t mask) {
    const uint32_t b = k == kNoRecord ? (uint32_t)tb.B : (uint32_t)time_bin(tb, k);
    return (b >> shift) & mask;
}

// cnt[d * n_tiles + t]: records of tile t whose digit is d (256 digits; those above the
// pass's width count 0).
__global__ void __launch_bounds__(256) rdx_count_kernel(const unsigned long long *__restrict__ key, int64_t n,
                                                        TimeBins tb, int32_t shift, uint32_t mask, int32_t n_tiles,
                                                        int32_t *__restrict__ cnt) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kRdxTile, t1 = min(t0 + (int64_t)kRdxTile, n);
    for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) atomicAdd(&h[rdx_digit(tb, key[i], shift, mask)], 1);
    __syncthreads();
    cnt[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// incl: the inclusive prefix sum of cnt.  Moves tile blockIdx.x of (key, val) to its place
// in (okey, oval) for this pass's digit.
__global__ void __launch_bounds__(256) rdx_scatter_kernel(const unsigned long long *__restrict__ key,
                                                          const unsigned long long *__restrict__ val, int64_t n,
                                                          TimeBins tb, int32_t shift, uint32_t mask, int32_t bits,
                                                          int32_t n_tiles, const int32_t *__restrict__ cnt,
                                                          const int32_t *__restrict__ incl,
                                                          unsigned long long *__restrict__ okey,
                                                          unsigned long long *__restrict__ oval) {
    __shared__ unsigned long long sk[kRdxTile], sv[kRdxTile];
    __shared__ int32_t first[256];      // the tile's first local position of each digit
    __shared__ int32_t run[256];        // the next local position of each digit
    __shared__ int32_t wcnt[4][256];    // per wave: records of each digit in the chunk, then offsets
    const int32_t t = threadIdx.x, w = t / kWave;
    const uint32_t lane = __lane_id();
    const int64_t t0 = (int64_t)blockIdx.x * kRdxTile, t1 = min(t0 + (int64_t)kRdxTile, n);
    // exclusive prefix of this tile's digit counts (Hillis-Steele over 256 digits)
    const int32_t mine = cnt[(int64_t)t * n_tiles + blockIdx.x];
    first[t] = mine;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t x = t >= off ? first[t - off] : 0;
        __syncthreads();
        first[t] += x;
        __syncthreads();
    }
    const int32_t excl = first[t] - mine;
    __syncthreads();
    first[t] = excl;
    run[t] = excl;
    __syncthreads();
    for (int64_t c = t0; c < t1; c += 256) {
        for (int q = t; q < 4 * 256; q += 256) wcnt[q / 256][q % 256] = 0;
        __syncthreads();
        const int64_t i = c + t;
        const bool in = i < t1;
        const unsigned long long k = in ? key[i] : kNoRecord;
        const unsigned long long v = in ? val[i] : 0ull;
        const uint32_t d = in ? rdx_digit(tb, k, shift, mask) : 0u;
        uint64_t same = __ballot(in);
        for (int32_t b = 0; b < bits; ++b) {
            const bool one = ((d >> b) & 1u) != 0u;
            const uint64_t bb = __ballot(one);
            same &= one ? bb : ~bb;
        }
        const int32_t rank = __popcll(same & lanemask_lt());
        if (in && rank == 0) wcnt[w][d] = __popcll(same);
        __syncthreads();
        {
            // digit t: the waves' first positions in this chunk, in wave order
            int32_t r = run[t];
            for (int q = 0; q < 4; ++q) {
                const int32_t m = wcnt[q][t];
                wcnt[q][t] = r;
                r += m;
            }
            run[t] = r;
        }
        __syncthreads();
        if (in) {
            const int32_t lp = wcnt[w][d] + rank;
            sk[lp] = k;
            sv[lp] = v;
        }
        __syncthreads();
    }
    // the staged tile in digit order: position j of digit d goes to the digit's first output
    // position for this tile plus (j - first[d])
    const int32_t tn = (int32_t)(t1 - t0);
    for (int32_t j = t; j < tn; j += blockDim.x) {
        const unsigned long long k = sk[j];
        const uint32_t d = rdx_digit(tb, k, shift, mask);
        const int64_t q = (int64_t)d * n_tiles + blockIdx.x;
        const int64_t dst = (int64_t)incl[q] - cnt[q] + (j - first[d]);
        if (dst >= 0 && dst < n) {
            okey[dst] = k;
            oval[dst] = sv[j];
        }
    }
}

// start[b]: the first position of bin b among the R records sorted by bin (R for the bins
// after the last record); every bin is written once, by the record that starts it or the
// sentinel position R.
__global__ void __launch_bounds__(256) bin_start_kernel(const unsigned long long *__restrict__ key, int64_t R,
                                                        TimeBins tb, int32_t *__restrict__ start) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= R; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = i < R ? time_bin(tb, key[i]) : tb.B;
        const int32_t bp = i > 0 ? time_bin(tb, key[i - 1]) : -1;
        const int32_t hi = min(b, tb.B - 1);
        for (int32_t x = bp + 1; x <= hi; ++x) start[x] = (int32_t)i;
    }
}

// Bins of at most 64 records, one wave each: lane i takes record i, its place is the number
// of smaller keys plus the number of equal keys at lower lanes.  Larger bins are listed in
// big[] for bin_sort_big_kernel.
__global__ void __launch_bounds__(256) bin_sort_small_kernel(unsigned long long *__restrict__ key,
                                                             unsigned long long *__restrict__ val,
                                                             const int32_t *__restrict__ start, int32_t B, int64_t R,
                                                             int32_t *__restrict__ big, int32_t *__restrict__ n_big) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; b < B; b += waves) {
        const int64_t s = start[b], e = b + 1 < B ? (int64_t)start[b + 1] : R;
        const int32_t n = (int32_t)(e - s);
        if (n <= 1) continue;
        if (n > kWave) {
            if (lane == 0) big[atomicAdd(n_big, 1)] = (int32_t)b;
            continue;
        }
        const unsigned long long k = lane < n ? key[s + lane] : kNoRecord;
        const unsigned long long v = lane < n ? val[s + lane] : 0ull;
        int32_t rank = 0;
        for (int32_t j = 0; j < n; ++j) {
            const unsigned long long kj = __shfl(k, j);
            rank += (kj < k || (kj == k && j < lane)) ? 1 : 0;
        }
        if (lane < n) {
            key[s + rank] = k;
            val[s + rank] = v;
        }
    }
}

// Ascending bitonic network over n elements at positions [0, P) (P = n rounded up to a power
// of two; positions >= n act as +infinity and are never touched): for every merge size k,
// first i against i ^ (k - 1), then i against i ^ d for d = k/4 .. 1, every comparator
// putting the smaller key at the lower position.  ACC(i) is a reference to key i, SWP(i, j)
// exchanges records i and j.
template <class KeyAt, class Swap>
__device__ __forceinline__ void bitonic_ascending(int64_t n, KeyAt key_at, Swap swp, bool lds) {
    int64_t P = 1;
    while (P < n) P <<= 1;
    auto stage = [&](int64_t d, bool flip) {
        for (int64_t q = threadIdx.x; q < P / 2; q += blockDim.x) {
            // q-th pair: i has bit log2(d) clear (flip: the lower half of its k-block)
            const int64_t i = ((q / d) * 2 * d) + (q % d);
            const int64_t j = flip ? (i ^ (2 * d - 1)) : (i + d);
            if (j < n && key_at(j) < key_at(i)) swp(i, j);
        }
        if (!lds) __threadfence_block();
        __syncthreads();
    };
    for (int64_t k = 2; k <= P; k <<= 1) {
        stage(k / 2, true);
        for (int64_t d = k / 4; d >= 1; d >>= 1) stage(d, false);
    }
}

__global__ void __launch_bounds__(256) bin_sort_big_kernel(unsigned long long *__restrict__ key,
                                                           unsigned long long *__restrict__ val,
                                                           const int32_t *__restrict__ start, int32_t B, int64_t R,
                                                           const int32_t *__restrict__ big,
                                                           const int32_t *__restrict__ n_big) {
    __shared__ unsigned long long sk[kBinLds], sv[kBinLds];
    const int32_t nb = *n_big;
    for (int32_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int64_t b = big[i];
        const int64_t s = start[b], e = b + 1 < B ? (int64_t)start[b + 1] : R;
        const int64_t n = e - s;
        if (n <= kBinLds) {
            for (int64_t q = threadIdx.x; q < n; q += blockDim.x) {
                sk[q] = key[s + q];
                sv[q] = val[s + q];
            }
            __syncthreads();
            bitonic_ascending(
                n, [&](int64_t q) { return sk[q]; },
                [&](int64_t a, int64_t c) {
                    const unsigned long long tk = sk[a], tv = sv[a];
                    sk[a] = sk[c];
                    sv[a] = sv[c];
                    sk[c] = tk;
                    sv[c] = tv;
                },
                true);
            for (int64_t q = threadIdx.x; q < n; q += blockDim.x) {
                key[s + q] = sk[q];
                val[s + q] = sv[q];
            }
        } else {
            unsigned long long *gk = key + s, *gv = val + s;
            bitonic_ascending(
                n, [&](int64_t q) { return gk[q]; },
                [&](int64_t a, int64_t c) {
                    const unsigned long long tk = gk[a], tv = gv[a];
                    gk[a] = gk[c];
                    gv[a] = gv[c];
                    gk[c] = tk;
                    gv[c] = tv;
                },
                false);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// Adaptive selective memory (Section 3.2.1, Figure 3) from the time-sorted event log:
// Avg-Y's points are time 0 and the distinct event times; a record starts a point when its
// time differs from the previous record's.
// ---------------------------------------------------------------------------------------
__global__ void evt_start_kernel(const unsigned long long *__restrict__ key, int64_t R, int32_t *__restrict__ start) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x)
        start[r] = (r == 0 || key[r] != key[r - 1]) ? 1 : 0;
}

// Each record's moment differences at its point u = (rank of its time among the distinct
// times, from 1) - 1 + off (off = 1 when no event happens at time 0, whose point then
// holds the initial state), in the forward kernels' split (whole (2x+nu)nu below 2^24,
// else its low 24 bits and the rest >> 24); the first record of a point writes its time.
// D and Dhi are zero on entry.  A record alone at its point (no other record has its time:
// an event that changed one species) is the only contribution to its words and stores
// them; the records of a point with several (several species changed, or equal times) add
// theirs atomically.
__global__ void evt_diff_kernel(const unsigned long long *__restrict__ key, const unsigned long long *__restrict__ val,
                                const int32_t *__restrict__ start, const int32_t *__restrict__ rank1, int64_t R,
                                int32_t off, int32_t S, unsigned long long *__restrict__ D,
                                unsigned long long *__restrict__ Dhi, double *__restrict__ y_time) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = (int64_t)rank1[r] - 1 + off;
        const unsigned long long v = val[r];
        const int32_t s = (int32_t)(v & 0xfffu);
        const int32_t dl = ((int32_t)(((uint32_t)(v >> 12) & 0xfffffu) << 12)) >> 12;
        const int32_t xo = (int32_t)(uint32_t)(v >> 32);
        unsigned long long *dd = D + ((size_t)u * S + s) * 2;
        const long long d2 = (2ll * xo + dl) * (long long)dl;
        const bool small = d2 > -kSmallD2 && d2 < kSmallD2;
        const unsigned long long lo = (unsigned long long)(small ? d2 : (d2 & ((1ll << 24) - 1)));
        const bool first = start[r] != 0;
        const bool alone = first && (r + 1 == R || start[r + 1] != 0);
        if (alone) {
            dd[0] = (unsigned long long)(long long)dl;
            dd[1] = lo;
            if (!small) Dhi[(size_t)u * S + s] = (unsigned long long)(d2 >> 24);
        } else {
            atomicAdd(dd, (unsigned long long)(long long)dl);
            atomicAdd(dd + 1, lo);
            if (!small) atomicAdd(Dhi + (size_t)u * S + s, (unsigned long long)(d2 >> 24));
        }
        if (first) y_time[u] = __longlong_as_double((long long)key[r]);
    }
}

// Avg-XY: groups of k successive Avg-Y points (the last one may be shorter).  A group has
// C = 2S + 1 chains -- the time, S means and S variances -- each summed left to right in
// binary64 and then divided once by the group's size.  One block of four waves per group
// (and per 64 chains): the block copies the group's points tile by tile into LDS with
// coalesced loads of whole rows, and lane j of the first wave adds chain j of the tile in
// order while the loads of the next tile are in flight (four waves keep more bytes in
// flight than one wave's loads alone could behind the adds).  A wave per chain, adding 64
// lane broadcasts in a row, spent most of the adaptive run at k = 10^6 on that serial
// chain.
constexpr int kXyRegs = 16;                 // doubles per thread staged for the next tile
constexpr int kXyThreads = 4 * kWave;       // threads per block: all load, the first wave adds
constexpr int kXyTile = kXyRegs * kXyThreads;   // doubles per tile: T points of C values
constexpr int kXyBatch = 16;                // LDS reads of a chain in flight together

__global__ void __launch_bounds__(kXyThreads) xy_kernel(const double *__restrict__ y_time, const double *__restrict__ y_mean,
                                                const double *__restrict__ y_var, int64_t U, int32_t S, int64_t k,
                                                int64_t P, double *__restrict__ xy_time,
                                                double *__restrict__ xy_mean, double *__restrict__ xy_var) {
    __shared__ double tile[kXyTile];
    const int64_t p = blockIdx.x;
    const int32_t tid = (int32_t)threadIdx.x, lane = tid % kWave;
    if (p >= P) return;
    const int32_t C = 2 * S + 1;
    const int32_t T = kXyTile / C;          // points per tile, >= 1 for S <= 2047
    const int32_t TS = T * S;
    const int64_t u0 = p * k, u1 = min(u0 + k, U);
    // tile layout: times at [0, T), means at [T, T + T*S), variances at [T + T*S, T*C),
    // each in the row-major order of the source arrays
    // staged slot r of this thread: its source (time row, or a mean or variance entry) is
    // the same for every tile; only the tile's first point and its point count change
    const double *pb[kXyRegs];
    int32_t po[kXyRegs];
    bool pt[kXyRegs];
#pragma unroll
    for (int32_t r = 0; r < kXyRegs; ++r) {
        const int32_t f = tid + r * kXyThreads;
        pt[r] = f < T;
        if (f < T) {
            pb[r] = y_time + f;
            po[r] = f;
        } else if (f < T + TS) {
            pb[r] = y_mean + (f - T);
            po[r] = f - T;
        } else if (f < T * C) {
            pb[r] = y_var + (f - T - TS);
            po[r] = f - T - TS;
        } else {
            pb[r] = y_time;
            po[r] = INT32_MAX;   // never loaded
        }
    }
    double nx[kXyRegs];
    // every thread loads (slots past the tile's points read y_time[0] and keep 0), so the
    // loads stay unconditional and all of them are in flight together
    auto fetch = [&](int64_t base) {
        const int32_t n = (int32_t)min((int64_t)T, u1 - base), nS = n * S;
        const int64_t bS = base * S;
#pragma unroll
        for (int32_t r = 0; r < kXyRegs; ++r) {
            const bool ok = po[r] < (pt[r] ? n : nS);
            const double v = *(ok ? pb[r] + (pt[r] ? base : bS) : y_time);
            nx[r] = ok ? v : 0.0;
        }
    };
    const int32_t j = (int32_t)blockIdx.y * kWave + lane;   // this lane's chain (first wave)
    const bool act = tid < kWave && j < C;
    int32_t off = 0, stride = 1;
    if (j >= 1 && j <= S) {
        off = T + (j - 1);
        stride = S;
    } else if (j > S) {
        off = T + TS + (j - S - 1);
        stride = S;
    }
    double s = 0.0;
    fetch(u0);
    for (int64_t base = u0; base < u1; base += T) {
        __syncthreads();                    // every chain is done with the previous tile
#pragma unroll
        for (int32_t r = 0; r < kXyRegs; ++r) tile[tid + r * kXyThreads] = nx[r];
        __syncthreads();
        if (base + T < u1) fetch(base + T);
        const int32_t n = (int32_t)min((int64_t)T, u1 - base);
        if (act) {
            // reads issued kXyBatch at a time, so one LDS latency covers kXyBatch adds
            const double *c = tile + off;
            int32_t i = 0;
            for (; i + kXyBatch <= n; i += kXyBatch) {
                double v[kXyBatch];
#pragma unroll
                for (int32_t q = 0; q < kXyBatch; ++q) v[q] = c[(i + q) * stride];
#pragma unroll
                for (int32_t q = 0; q < kXyBatch; ++q) s = s + v[q];
            }
            for (; i < n; ++i) s = s + c[i * stride];
        }
    }
    if (act) {
        const double kk = (double)(u1 - u0);
        if (j == 0) {
            xy_time[p] = s / kk;
        } else if (j <= S) {
            xy_mean[(size_t)p * S + (j - 1)] = s / kk;
        } else {
            xy_var[(size_t)p * S + (j - S - 1)] = s / kk;
        }
    }
}

}  // namespace ssa
