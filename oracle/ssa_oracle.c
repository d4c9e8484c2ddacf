/*
 * ssa_oracle.c -- plain serial CPU oracle for the Gillespie direct-method SSA with
 * grid-aligned ("selective memory") reduction and the likelihood-ratio gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  The product path never calls it, and it
 * shares no source with the HIP kernels: every constant and every step below is written
 * out here from the paper's semantics and the published definitions it relies on.
 *
 * What the paper fixes (StochKit-FF, Aldinucci et al. 2010):
 *   - Section 2: the system is a CTMC; Gillespie's algorithm picks the next transition and
 *     its firing time exactly according to the memoryless (negative-exponential)
 *     distributions, one trajectory per realisation.
 *   - Section 3.2 (model format): integer state vector, integer stoichiometric matrix
 *     (entries such as -1 or +200), mass-action propensities built from reactant amounts
 *     and rates, and a simulated duration.
 *   - Section 3.2.1 (selective memory): trajectory points are aligned by simulation time
 *     and reduced across simulations with associative, commutative functions (average,
 *     variance).
 * Everything the paper leaves open (which random stream, the exact float operations of
 * the exponential draw, the sum order, the alignment convention, the variance estimator,
 * the gradient estimator) is a documented reading; each is stated where it is used.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math, no -march).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

/* Status codes (same meaning as the library's, numbered independently here). */
enum { ORC_OK = 0, ORC_INVALID = 1, ORC_NOMEM = 2, ORC_OVERFLOW = 4, ORC_EVENT_LIMIT = 5 };

/* A reaction network: S species, M reactions, reactant / product coefficient matrices
 * (row j = reaction j, column s = species s), stochastic rate constants c_j, the initial
 * integer state and the order in which the propensities are summed (see partial_sums). */
enum { ORC_SUM_SEQ = 0, ORC_SUM_BLOCK64 = 1 };

typedef struct {
    int32_t S, M;
    const int32_t *reac;  /* [M*S] */
    const int32_t *prod;  /* [M*S] */
    const double *rate;   /* [M]   */
    const int32_t *x0;    /* [S]   */
    int32_t sum_order;    /* ORC_SUM_SEQ or ORC_SUM_BLOCK64 */
    /* Optional rate laws (NULL: mass action throughout).  For reaction j with
     * law_species[j] = m >= 0 the rate constant is not c_j but
     *   c_j(x) = min(max(c_j + law_slope[j] * x_m, law_lo[j]), law_hi[j])
     * -- the infectivities of Section 2.1, beta -/+ K F clamped to [0, beta] -- evaluated as
     * one product, one sum (binary64) and the two exact bounds, before the one product with
     * the mass-action count. */
    const int32_t *law_species;  /* [M] or NULL */
    const double *law_slope, *law_lo, *law_hi;  /* [M] */
} orc_net;

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11).  Ten rounds of the 4x32 Philox S-box; the key is bumped by the Weyl constants
 * between rounds.  Multipliers and Weyl increments are the published ones.
 * ---------------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;   /* golden ratio */
            k1 += 0xBB67AE85u;   /* sqrt(3) - 1  */
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The draw for step k of trajectory i: key = (seed low word, seed high word),
 * counter = (k low, k high, i low, i high).  One block per drawn step. */
static void draw_block(uint64_t seed, uint64_t traj, uint64_t k, uint32_t o[4])
{
    uint32_t ctr[4] = { (uint32_t)k, (uint32_t)(k >> 32), (uint32_t)traj, (uint32_t)(traj >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, o);
}

/* 53-bit uniforms: words (o0,o1) give r1 in (0,1], words (o2,o3) give r2 in [0,1).
 * The 64-bit word is (hi << 32) | lo; its top 53 bits are taken and scaled by 2^-53,
 * which is exact in binary64. */
static double u01_open_low(uint32_t lo, uint32_t hi)
{
    uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
    return (double)(v + 1u) * 0x1p-53;
}
static double u01_open_high(uint32_t lo, uint32_t hi)
{
    uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
    return (double)v * 0x1p-53;
}

void orc_uniforms(uint64_t seed, uint64_t traj, uint64_t k, double *r1, double *r2)
{
    uint32_t o[4];
    draw_block(seed, traj, k, o);
    *r1 = u01_open_low(o[0], o[1]);
    *r2 = u01_open_high(o[2], o[3]);
}

/* ------------------------------------------------------------------------------------
 * -ln(r) for r in [2^-53, 1]: the exponential waiting time of the direct method needs
 * -ln(U).  Written from the mathematics so that a second implementation can reproduce
 * every rounding:
 *   r = m * 2^E with m in (sqrt(2)/2, sqrt(2)]
 *   ln m = 2 atanh(f), f = (m-1)/(m+1), 2 atanh(f) = 2f + f * s * sum_{n>=1} C_n s^(n-1),
 *   s = f^2, C_n = 2/(2n+1)   (series truncated after n = 10; |f| <= 0.1716)
 *   ln r = E*LN2_HI + (ln m + E*LN2_LO)
 * Each operation is one IEEE binary64 operation rounded to nearest-even; fma() is the
 * single-rounding fused multiply-add.  LN2_HI is ln 2 rounded to binary64 with its low
 * 21 significand bits cleared (so E*LN2_HI is exact for |E| < 2^21); LN2_LO is the
 * binary64 nearest to ln 2 - LN2_HI.
 * ---------------------------------------------------------------------------------- */
static const double ORC_LN2_HI = 0x1.62e42fee00000p-1;
static const double ORC_LN2_LO = 0x1.a39ef35793c76p-33;
static const double ORC_SQRT2 = 0x1.6a09e667f3bcdp+0;

double orc_neglog(double r)
{
    uint64_t b;
    memcpy(&b, &r, 8);
    int E = (int)((b >> 52) & 0x7ff) - 1023;
    uint64_t mb = (b & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &mb, 8);
    if (m > ORC_SQRT2) {
        m = m * 0.5;
        E = E + 1;
    }
    double f = (m - 1.0) / (m + 1.0);
    double s = f * f;
    double P = 2.0 / 21.0;                    /* C_10 */
    for (int n = 9; n >= 1; --n)
        P = fma(P, s, 2.0 / (double)(2 * n + 1));
    double t = s * P;
    double lnm = fma(f, t, f + f);
    double Ed = (double)E;
    double lnr = fma(Ed, ORC_LN2_HI, fma(Ed, ORC_LN2_LO, lnm));
    return -lnr;
}

/* ------------------------------------------------------------------------------------
 * e^theta for the log rate constants theta = ln c (the parameters of the gradient; Section
 * 4's sensitivity analysis varies rate parameters).  The paper fixes no arithmetic, so the
 * reading is a plain argument reduction and a Taylor polynomial with stated roundings:
 *   theta < -708 (below the normal range of c): 0;  theta > 709 or NaN: invalid (NaN);
 *   k = nearest integer (ties to even) to fl(theta * (1/ln 2)), 1/ln 2 rounded to binary64;
 *   r = theta - k ln 2 in two fused steps, first with LN2_HI, then with LN2_LO;
 *   e^r by Horner over the Taylor coefficients 1/n!, n = 13 down to 0, each step one
 *   fused multiply-add, the coefficients being the binary64 quotients 1/n! (n! is an exact
 *   integer in binary64 up to 13!);
 *   c = e^r * 2^k (a power-of-two scaling, exact for k >= -1021).
 * |r| <= ln2/2 + |k| 2^-60, so the Taylor remainder |r|^14/14! < 2^-57 relative.
 * ---------------------------------------------------------------------------------- */
static const double ORC_INV_LN2 = 0x1.71547652b82fep+0;

double orc_exp(double theta)
{
    if (theta < -708.0)
        return 0.0;
    if (!(theta <= 709.0))
        return NAN;
    double k = nearbyint(theta * ORC_INV_LN2);
    double r = fma(-k, ORC_LN2_HI, theta);
    r = fma(-k, ORC_LN2_LO, r);
    double coef[14];
    double fact = 1.0;
    for (int n = 0; n < 14; ++n) {
        if (n > 0)
            fact = fact * (double)n;
        coef[n] = 1.0 / fact;
    }
    double p = coef[13];
    for (int n = 12; n >= 0; --n)
        p = fma(p, r, coef[n]);
    return ldexp(p, (int)k);
}

/* ------------------------------------------------------------------------------------
 * Model checks and mass-action propensities (Section 3.2: integer state, integer
 * stoichiometry, propensity from reactant amounts and the rate).
 *   order 0:           h = 1
 *   one reactant A:    h = x_A
 *   A + B (A != B):    h = x_A * x_B
 *   2A:                h = x_A (x_A - 1) / 2     (distinct unordered pairs)
 * h is formed exactly in 64-bit integers, converted to binary64 (round to nearest even),
 * and a_j = c_j * h with one rounding.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int32_t order, sa, sb;   /* sa/sb: reactant species (-1 if unused); sb == sa for 2A */
} rxn_info;

static int check_net(const orc_net *n)
{
    if (!n || n->S <= 0 || n->M <= 0 || !n->reac || !n->prod || !n->rate || !n->x0) return ORC_INVALID;
    if (n->sum_order != ORC_SUM_SEQ && n->sum_order != ORC_SUM_BLOCK64) return ORC_INVALID;
    for (int j = 0; j < n->M; ++j) {
        int order = 0;
        for (int s = 0; s < n->S; ++s) {
            int32_t r = n->reac[j * n->S + s], p = n->prod[j * n->S + s];
            if (r < 0 || p < 0) return ORC_INVALID;
            order += r;
            if (order > 2) return ORC_INVALID;
        }
        if (!(n->rate[j] >= 0.0) || !isfinite(n->rate[j])) return ORC_INVALID;
        if (n->law_species && n->law_species[j] >= 0) {
            if (n->law_species[j] >= n->S || !isfinite(n->law_slope[j]) || !(n->law_lo[j] >= 0.0) ||
                !(n->law_hi[j] >= n->law_lo[j]))
                return ORC_INVALID;
        }
    }
    for (int s = 0; s < n->S; ++s)
        if (n->x0[s] < 0) return ORC_INVALID;
    return ORC_OK;
}

static void build_info(const orc_net *n, rxn_info *info)
{
    for (int j = 0; j < n->M; ++j) {
        info[j].order = 0; info[j].sa = -1; info[j].sb = -1;
        for (int s = 0; s < n->S; ++s) {
            int32_t r = n->reac[j * n->S + s];
            for (int q = 0; q < r; ++q) {
                if (info[j].sa < 0) info[j].sa = s; else info[j].sb = s;
            }
            info[j].order += r;
        }
    }
}

static double propensity(const orc_net *n, const rxn_info *ri, int j, const int32_t *x)
{
    int64_t h;
    if (ri->order == 0) {
        h = 1;
    } else if (ri->order == 1) {
        h = x[ri->sa];
    } else if (ri->sa == ri->sb) {
        int64_t v = x[ri->sa];
        h = v * (v - 1) / 2;
    } else {
        h = (int64_t)x[ri->sa] * (int64_t)x[ri->sb];
    }
    double c = n->rate[j];
    if (n->law_species && n->law_species[j] >= 0) {
        double v = c + n->law_slope[j] * (double)x[n->law_species[j]];
        c = fmin(fmax(v, n->law_lo[j]), n->law_hi[j]);
    }
    return c * (double)h;
}

/* ------------------------------------------------------------------------------------
 * Partial sums S_j of the propensities (Section 2's cumulative sums for the selection).
 * The paper leaves the summation order open; it is a model attribute:
 *   sequential: S_0 = a_0, S_j = S_{j-1} + a_j.
 *   block64:    the reactions are cut into 64 consecutive chunks of q = ceil(M / 64)
 *               (chunk l holds indices l q .. l q + q - 1 that are below M).  L_j is the
 *               sequential sum inside the chunk, T_l the chunk total (0 for an empty
 *               chunk).  The totals are scanned inclusively in six steps d = 1, 2, 4, ..., 32,
 *               each step replacing v_l by v_l + v_{l-d} for l >= d from the previous
 *               step's values; E_l is the scanned value of chunk l - 1 (E_0 = 0) and
 *               S_j = E_l + L_j for j in chunk l.
 * In both orders a0 = S_{M-1}.
 * ---------------------------------------------------------------------------------- */
static void partial_sums(int order, int M, const double *a, double *S)
{
    if (order == ORC_SUM_SEQ) {
        S[0] = a[0];
        for (int j = 1; j < M; ++j) S[j] = S[j - 1] + a[j];
        return;
    }
    const int q = (M + 63) / 64;
    double v[64], prev[64], E[64];
    for (int l = 0; l < 64; ++l) {
        v[l] = 0.0;
        double L = 0.0;
        for (int i = 0; i < q; ++i) {
            int j = l * q + i;
            if (j >= M) break;
            L = (i == 0) ? a[j] : L + a[j];
            S[j] = L;                       /* local sum for now */
        }
        if (l * q < M) v[l] = L;
    }
    for (int d = 1; d < 64; d *= 2) {
        for (int l = 0; l < 64; ++l) prev[l] = v[l];
        for (int l = d; l < 64; ++l) v[l] = prev[l] + prev[l - d];
    }
    E[0] = 0.0;
    for (int l = 1; l < 64; ++l) E[l] = v[l - 1];
    for (int j = 0; j < M; ++j) S[j] = E[j / q] + S[j];
}

static int check_grid(const double *grid, int32_t G, double t_end)
{
    if (!(t_end >= 0.0) || !isfinite(t_end)) return ORC_INVALID;
    if (G <= 0 || !grid) return ORC_INVALID;
    for (int g = 0; g < G; ++g) {
        if (!(grid[g] >= 0.0) || !(grid[g] <= t_end)) return ORC_INVALID;
        if (g > 0 && !(grid[g] >= grid[g - 1])) return ORC_INVALID;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------
 * One trajectory of the direct method (Section 2), with the grid alignment of
 * Section 3.2.1 and optional bookkeeping for the likelihood-ratio gradient.
 *
 * Readings:
 *   - Propensities are recomputed in full at every step; a0 and the partial sums S_j
 *     follow the network's sum order (partial_sums); a0 = S_{M-1}.
 *   - If a0 == 0 the state is absorbing: no draw is made and the state holds to t_end.
 *   - Otherwise draw k gives (r1, r2); tau = neglog(r1) / a0 (IEEE division);
 *     t_next = t + tau; k counts draws made, the last (overshooting) draw included.
 *   - Grid alignment is right-continuous: the value at grid time t_g contains every event
 *     with t_e <= t_g.  All grid points with t_g < t_next are given the current state
 *     before the event is applied.
 *   - An event with t_next > t_end is not applied; one with t_next == t_end is.
 *   - Selection: u = r2 * a0; j = smallest index with S_j > u; if rounding leaves no
 *     such j, the largest j with a_j > 0.
 *   - Update: x += nu_j in 32-bit integers; leaving the int32 range is an error.
 *   - Gradient bookkeeping per applied event: n_j of the fired reaction += 1, and for
 *     every reaction A_j += a_j * tau (one product, one sum, in index order), before t
 *     is advanced.  At a grid crossing the integral up to t_g is A_j + a_j * (t_g - t).
 *
 * visit(g) is called at each grid crossing with the current state.
 * ---------------------------------------------------------------------------------- */
typedef struct traj_state_ {
    const orc_net *net;
    const rxn_info *info;
    int32_t *x;      /* [S] */
    double *a;       /* [M] */
    double *Ssum;    /* [M] */
    int64_t *nf;     /* [M] fired counts */
    double *A;       /* [M] integrated propensities */
    double t;
    /* called after every applied event (t and x already updated), or NULL */
    void (*on_event)(void *ctx, const struct traj_state_ *st);
    void *ev_ctx;
} traj_state;

typedef void (*visit_fn)(void *ctx, int g, const traj_state *st, double tg);

static int run_trajectory(const orc_net *net, const rxn_info *info, uint64_t seed, uint64_t traj,
                          double t_end, const double *grid, int32_t G, uint64_t max_events,
                          traj_state *st, uint64_t *events_out, uint64_t *draws_out,
                          visit_fn visit, void *ctx)
{
    const int S = net->S, M = net->M;
    for (int s = 0; s < S; ++s) st->x[s] = net->x0[s];
    for (int j = 0; j < M; ++j) { st->nf[j] = 0; st->A[j] = 0.0; }
    st->t = 0.0;
    uint64_t k = 0, events = 0;
    int g = 0;
    int status = ORC_OK;
    for (;;) {
        for (int j = 0; j < M; ++j) st->a[j] = propensity(net, &info[j], j, st->x);
        partial_sums(net->sum_order, M, st->a, st->Ssum);
        const double a0 = st->Ssum[M - 1];
        double tau, r2 = 0.0;
        if (a0 == 0.0) {
            tau = INFINITY;
        } else {
            double r1;
            orc_uniforms(seed, traj, k, &r1, &r2);
            tau = orc_neglog(r1) / a0;
            k = k + 1;
        }
        double t_next = st->t + tau;
        while (g < G && grid[g] < t_next) {
            if (visit) visit(ctx, g, st, grid[g]);
            g = g + 1;
        }
        if (t_next > t_end) break;
        if (events >= max_events) { status = ORC_EVENT_LIMIT; break; }
        double u = r2 * a0;
        int sel = -1;
        for (int j = 0; j < M; ++j)
            if (st->Ssum[j] > u) { sel = j; break; }
        if (sel < 0)
            for (int j = M - 1; j >= 0; --j)
                if (st->a[j] > 0.0) { sel = j; break; }
        for (int s = 0; s < S; ++s) {
            int64_t nx = (int64_t)st->x[s] + (int64_t)net->prod[sel * S + s] - (int64_t)net->reac[sel * S + s];
            if (nx > INT32_MAX || nx < INT32_MIN) { status = ORC_OVERFLOW; break; }
            st->x[s] = (int32_t)nx;
        }
        if (status != ORC_OK) break;
        st->nf[sel] += 1;
        for (int j = 0; j < M; ++j) st->A[j] = st->A[j] + st->a[j] * tau;
        st->t = t_next;
        events = events + 1;
        if (st->on_event) st->on_event(st->ev_ctx, st);
    }
    if (events_out) *events_out = events;
    if (draws_out) *draws_out = k;
    return status;
}

static int alloc_state(const orc_net *net, traj_state *st, const rxn_info *info)
{
    st->net = net; st->info = info;
    st->on_event = NULL; st->ev_ctx = NULL;
    st->x = (int32_t *)malloc(sizeof(int32_t) * net->S);
    st->a = (double *)malloc(sizeof(double) * net->M);
    st->Ssum = (double *)malloc(sizeof(double) * net->M);
    st->nf = (int64_t *)malloc(sizeof(int64_t) * net->M);
    st->A = (double *)malloc(sizeof(double) * net->M);
    if (!st->x || !st->a || !st->Ssum || !st->nf || !st->A) return ORC_NOMEM;
    return ORC_OK;
}

static void free_state(traj_state *st)
{
    free(st->x); free(st->a); free(st->Ssum); free(st->nf); free(st->A);
}

/* ---------------------------------------------------------------------------------- */
/* Record one trajectory: states at every grid point, events applied, draws made, time of */
/* the last applied event, and per-reaction n_j and A_j over [0, t_end].                  */
/* A_j over [0, t_end] adds the final partial interval a_j * (t_end - t_last).            */
/* ---------------------------------------------------------------------------------- */
typedef struct { int32_t *states; int S; } rec_ctx;

static void rec_visit(void *c, int g, const traj_state *st, double tg)
{
    (void)tg;
    rec_ctx *rc = (rec_ctx *)c;
    if (rc->states)
        for (int s = 0; s < rc->S; ++s) rc->states[(size_t)g * rc->S + s] = st->x[s];
}

int orc_trajectory(const orc_net *net, uint64_t seed, uint64_t traj, double t_end,
                   const double *grid, int32_t G, uint64_t max_events,
                   int32_t *states, uint64_t *events, uint64_t *draws, double *t_last,
                   int64_t *n_fired, double *a_int)
{
    int st_ok = check_net(net);
    if (st_ok) return st_ok;
    if (check_grid(grid, G, t_end)) return ORC_INVALID;
    rxn_info *info = (rxn_info *)malloc(sizeof(rxn_info) * net->M);
    traj_state st;
    if (!info) return ORC_NOMEM;
    build_info(net, info);
    if (alloc_state(net, &st, info)) { free_state(&st); free(info); return ORC_NOMEM; }
    rec_ctx rc = { states, net->S };
    int status = run_trajectory(net, info, seed, traj, t_end, grid, G, max_events, &st, events, draws,
                                rec_visit, &rc);
    if (t_last) *t_last = st.t;
    if (n_fired) for (int j = 0; j < net->M; ++j) n_fired[j] = st.nf[j];
    if (a_int) {
        /* propensities at the final state, then the last partial interval */
        double tail = t_end - st.t;
        for (int j = 0; j < net->M; ++j) {
            double aj = propensity(net, &info[j], j, st.x);
            a_int[j] = st.A[j] + aj * tail;
        }
    }
    free_state(&st);
    free(info);
    return status;
}

/* ------------------------------------------------------------------------------------
 * Cross-trajectory reduction (Section 3.2.1 with average and variance as combining
 * functions, Section 4's mean/variance plots).  Exact: sums of X and X^2 per (grid point,
 * species) in 128-bit integers over all N trajectories, then
 *   mean = fl(sum X) / N
 *   var  = fl(N * sum X^2 - (sum X)^2) / (N (N - 1))     (unbiased; var = 0 when N = 1)
 * Optional histogram of one species per grid point: bin = (x - lo) div width, clamped
 * to [0, nbins - 1].
 * Requires N <= 2^30 so that N * sum X^2 stays within 127 bits.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int S, G;
    i128 *sx, *sx2;       /* [G*S] */
    uint32_t *hist;       /* [G*nb] or NULL */
    int hs, hlo, hw, hnb;
} mom_ctx;

static void mom_visit(void *c, int g, const traj_state *st, double tg)
{
    (void)tg;
    mom_ctx *mc = (mom_ctx *)c;
    for (int s = 0; s < mc->S; ++s) {
        i128 v = st->x[s];
        mc->sx[(size_t)g * mc->S + s] += v;
        mc->sx2[(size_t)g * mc->S + s] += v * v;
    }
    if (mc->hist) {
        int32_t v = st->x[mc->hs];
        int64_t b = (v < mc->hlo) ? 0 : ((int64_t)v - mc->hlo) / mc->hw;
        if (b > mc->hnb - 1) b = mc->hnb - 1;
        mc->hist[(size_t)g * mc->hnb + b] += 1u;
    }
}

int orc_run(const orc_net *net, int64_t N, double t_end, const double *grid, int32_t G,
            uint64_t seed, uint64_t max_events,
            int32_t hist_species, int32_t hist_lo, int32_t hist_width, int32_t hist_nbins,
            double *mean, double *var, uint32_t *hist, int64_t *sum_x_hi_lo /* [G*S*4] or NULL */,
            uint64_t *total_events, int nthreads)
{
    int st0 = check_net(net);
    if (st0) return st0;
    if (check_grid(grid, G, t_end)) return ORC_INVALID;
    if (N <= 0 || N > ((int64_t)1 << 30)) return ORC_INVALID;
    if (hist && (hist_species < 0 || hist_species >= net->S || hist_width <= 0 || hist_nbins <= 0))
        return ORC_INVALID;
    const int S = net->S, M = net->M;
    const size_t GS = (size_t)G * S;
    rxn_info *info = (rxn_info *)malloc(sizeof(rxn_info) * M);
    i128 *sx = (i128 *)calloc(GS, sizeof(i128));
    i128 *sx2 = (i128 *)calloc(GS, sizeof(i128));
    uint32_t *h = hist ? (uint32_t *)calloc((size_t)G * hist_nbins, sizeof(uint32_t)) : NULL;
    if (!info || !sx || !sx2 || (hist && !h)) { free(info); free(sx); free(sx2); free(h); return ORC_NOMEM; }
    build_info(net, info);
    int status = ORC_OK;
    uint64_t events_all = 0;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        mom_ctx mc;
        mc.S = S; mc.G = G;
        mc.sx = (i128 *)calloc(GS, sizeof(i128));
        mc.sx2 = (i128 *)calloc(GS, sizeof(i128));
        mc.hist = hist ? (uint32_t *)calloc((size_t)G * hist_nbins, sizeof(uint32_t)) : NULL;
        mc.hs = hist_species; mc.hlo = hist_lo; mc.hw = hist_width; mc.hnb = hist_nbins;
        traj_state st;
        int ok = (mc.sx && mc.sx2 && (!hist || mc.hist) && alloc_state(net, &st, info) == ORC_OK);
        int my_status = ok ? ORC_OK : ORC_NOMEM;
        uint64_t my_events = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < N; ++i) {
            if (my_status != ORC_OK) continue;
            uint64_t ev = 0;
            int r = run_trajectory(net, info, seed, (uint64_t)i, t_end, grid, G, max_events, &st, &ev, NULL,
                                   mom_visit, &mc);
            my_events += ev;
            if (r != ORC_OK) my_status = r;
        }
#pragma omp critical
        {
            if (my_status != ORC_OK && status == ORC_OK) status = my_status;
            events_all += my_events;
            if (ok) {
                for (size_t q = 0; q < GS; ++q) { sx[q] += mc.sx[q]; sx2[q] += mc.sx2[q]; }
                if (hist)
                    for (size_t q = 0; q < (size_t)G * hist_nbins; ++q) h[q] += mc.hist[q];
            }
        }
        if (ok) free_state(&st);
        free(mc.sx); free(mc.sx2); free(mc.hist);
    }
    if (status == ORC_OK) {
        for (size_t q = 0; q < GS; ++q) {
            mean[q] = (double)sx[q] / (double)N;
            if (N == 1) {
                var[q] = 0.0;
            } else {
                i128 num = (i128)N * sx2[q] - sx[q] * sx[q];
                var[q] = (double)num / ((double)N * (double)(N - 1));
            }
            if (sum_x_hi_lo) {
                /* sum X and sum X^2 as two's-complement 128-bit values (hi, lo) */
                sum_x_hi_lo[4 * q + 0] = (int64_t)(sx[q] >> 64);
                sum_x_hi_lo[4 * q + 1] = (int64_t)(uint64_t)sx[q];
                sum_x_hi_lo[4 * q + 2] = (int64_t)(sx2[q] >> 64);
                sum_x_hi_lo[4 * q + 3] = (int64_t)(uint64_t)sx2[q];
            }
        }
        if (hist) memcpy(hist, h, sizeof(uint32_t) * (size_t)G * hist_nbins);
    }
    if (total_events) *total_events = events_all;
    free(info); free(sx); free(sx2); free(h);
    return status;
}

/* ------------------------------------------------------------------------------------
 * Likelihood-ratio gradient of a loss on the grid means with respect to theta_j = ln c_j.
 * The paper gives no estimator (it motivates sensitivity analysis in Section 4); the
 * reading used here is the standard score-function identity for a CTMC path density:
 *   d/d theta_j log p(path on [0,t]) = n_j(t) - A_j(t),  A_j(t) = int_0^t a_j(x(s)) ds,
 * so d m_{g,s} / d theta_j = E[ X_s(t_g) z_j(t_g) ],  z_j = n_j - A_j.  With the centring
 * m_hat (E[z_j] = 0 makes it consistent):
 *   D_{g,s,j} = (1/N) sum_i (X^i_s(t_g) - m_hat_{g,s}) z^i_j(t_g)
 *   grad_j    = sum_{g,s} w_{g,s} D_{g,s,j}
 * l1_j returns (1/N) sum_i sum_{g,s} |w_{g,s} (X - m_hat) z_j|, the scale for tolerances.
 * Sums run in long double, per trajectory and then across trajectories.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int S, M;
    const double *w, *mhat;
    const double *wv, *vhat; /* variance weights and centring, or NULL */
    long double *acc, *l1;   /* [M] for the current trajectory */
    double *z;               /* [M] scratch */
} grad_ctx;

static void grad_visit(void *c, int g, const traj_state *st, double tg)
{
    grad_ctx *gc = (grad_ctx *)c;
    for (int j = 0; j < gc->M; ++j) {
        double Atg = st->A[j] + st->a[j] * (tg - st->t);
        gc->z[j] = (double)st->nf[j] - Atg;
    }
    for (int s = 0; s < gc->S; ++s) {
        double d = (double)st->x[s] - gc->mhat[(size_t)g * gc->S + s];
        double wd = gc->w[(size_t)g * gc->S + s] * d;
        for (int j = 0; j < gc->M; ++j) {
            double term = wd * gc->z[j];
            gc->acc[j] += (long double)term;
            gc->l1[j] += (long double)fabs(term);
        }
        if (gc->wv) {
            /* variance term: wv ((X - mhat)^2 - vhat) z_j, in long double; its scale is the
             * size of the expanded terms wv (X^2 + 2|X mhat| + mhat^2 + |vhat|) |z_j| */
            const long double x = (long double)st->x[s], m = (long double)gc->mhat[(size_t)g * gc->S + s];
            const long double v = (long double)gc->vhat[(size_t)g * gc->S + s];
            const long double wv = (long double)gc->wv[(size_t)g * gc->S + s];
            const long double q = wv * ((x - m) * (x - m) - v);
            const long double qs = fabsl(wv) * (x * x + 2.0L * fabsl(x * m) + m * m + fabsl(v));
            for (int j = 0; j < gc->M; ++j) {
                gc->acc[j] += q * (long double)gc->z[j];
                gc->l1[j] += qs * fabsl((long double)gc->z[j]);
            }
        }
    }
}

int orc_grad_moments(const orc_net *net, int64_t N, double t_end, const double *grid, int32_t G,
                     uint64_t seed, uint64_t max_events, const double *w, const double *mhat, const double *wv,
                     const double *vhat, double *grad, double *l1, int nthreads);

int orc_grad(const orc_net *net, int64_t N, double t_end, const double *grid, int32_t G,
             uint64_t seed, uint64_t max_events, const double *w, const double *mhat,
             double *grad, double *l1, int nthreads)
{
    return orc_grad_moments(net, N, t_end, grid, G, seed, max_events, w, mhat, NULL, NULL, grad, l1, nthreads);
}

/* The same gradient for a loss on the grid means and variances: with wv = dL/dvar and the
 * centring vhat (usually the forward variance) each crossing adds
 *   wv_{g,s} ((X_s(t_g) - mhat_{g,s})^2 - vhat_{g,s}) z_j(t_g),
 * the score-function derivative of the variance: d/dtheta E[(X - mu)^2] = E[(X - mu)^2 z]
 * because E[X - mu] = 0, and E[z] = 0 makes the centring by vhat unbiased. */
int orc_grad_moments(const orc_net *net, int64_t N, double t_end, const double *grid, int32_t G,
                     uint64_t seed, uint64_t max_events, const double *w, const double *mhat, const double *wv,
                     const double *vhat, double *grad, double *l1, int nthreads)
{
    if (wv && !vhat) return ORC_INVALID;
    int st0 = check_net(net);
    if (st0) return st0;
    if (check_grid(grid, G, t_end)) return ORC_INVALID;
    if (N <= 0 || !w || !mhat || !grad) return ORC_INVALID;
    const int S = net->S, M = net->M;
    rxn_info *info = (rxn_info *)malloc(sizeof(rxn_info) * M);
    long double *tot = (long double *)calloc(M, sizeof(long double));
    long double *totl1 = (long double *)calloc(M, sizeof(long double));
    if (!info || !tot || !totl1) { free(info); free(tot); free(totl1); return ORC_NOMEM; }
    build_info(net, info);
    int status = ORC_OK;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        grad_ctx gc;
        gc.S = S; gc.M = M; gc.w = w; gc.mhat = mhat; gc.wv = wv; gc.vhat = vhat;
        gc.acc = (long double *)calloc(M, sizeof(long double));
        gc.l1 = (long double *)calloc(M, sizeof(long double));
        gc.z = (double *)calloc(M, sizeof(double));
        long double *mine = (long double *)calloc(M, sizeof(long double));
        long double *minel1 = (long double *)calloc(M, sizeof(long double));
        traj_state st;
        int ok = gc.acc && gc.l1 && gc.z && mine && minel1 && alloc_state(net, &st, info) == ORC_OK;
        int my_status = ok ? ORC_OK : ORC_NOMEM;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < N; ++i) {
            if (my_status != ORC_OK) continue;
            for (int j = 0; j < M; ++j) { gc.acc[j] = 0.0L; gc.l1[j] = 0.0L; }
            int r = run_trajectory(net, info, seed, (uint64_t)i, t_end, grid, G, max_events, &st, NULL, NULL,
                                   grad_visit, &gc);
            if (r != ORC_OK) { my_status = r; continue; }
            for (int j = 0; j < M; ++j) { mine[j] += gc.acc[j]; minel1[j] += gc.l1[j]; }
        }
#pragma omp critical
        {
            if (my_status != ORC_OK && status == ORC_OK) status = my_status;
            if (ok) for (int j = 0; j < M; ++j) { tot[j] += mine[j]; totl1[j] += minel1[j]; }
        }
        if (ok) free_state(&st);
        free(gc.acc); free(gc.l1); free(gc.z); free(mine); free(minel1);
    }
    if (status == ORC_OK) {
        for (int j = 0; j < M; ++j) {
            grad[j] = (double)(tot[j] / (long double)N);
            if (l1) l1[j] = (double)(totl1[j] / (long double)N);
        }
    }
    free(info); free(tot); free(totl1);
    return status;
}

/* ------------------------------------------------------------------------------------
 * The whole likelihood-ratio Jacobian of the grid means (the same estimator as orc_grad,
 * before it is contracted with w):
 *   J_{g,s,j} = (1/N) sum_i (X^i_s(t_g) - m_hat_{g,s}) z^i_j(t_g),   z_j = n_j - A_j,
 * with l1_{g,s,j} = (1/N) sum_i |(X - m_hat) z_j| as the tolerance scale.  Layout
 * [G][S][M].  Sums run in long double.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int S, M;
    const double *mhat;
    long double *acc, *l1;   /* [G*S*M] of this thread */
    double *z;               /* [M] scratch */
} jac_ctx;

static void jac_visit(void *c, int g, const traj_state *st, double tg)
{
    jac_ctx *jc = (jac_ctx *)c;
    for (int j = 0; j < jc->M; ++j) {
        double Atg = st->A[j] + st->a[j] * (tg - st->t);
        jc->z[j] = (double)st->nf[j] - Atg;
    }
    for (int s = 0; s < jc->S; ++s) {
        double d = (double)st->x[s] - jc->mhat[(size_t)g * jc->S + s];
        size_t base = ((size_t)g * jc->S + s) * jc->M;
        for (int j = 0; j < jc->M; ++j) {
            double term = d * jc->z[j];
            jc->acc[base + j] += (long double)term;
            jc->l1[base + j] += (long double)fabs(term);
        }
    }
}

int orc_jacobian(const orc_net *net, int64_t N, double t_end, const double *grid, int32_t G,
                 uint64_t seed, uint64_t max_events, const double *mhat, double *jac, double *l1,
                 int nthreads)
{
    int st0 = check_net(net);
    if (st0) return st0;
    if (check_grid(grid, G, t_end)) return ORC_INVALID;
    if (N <= 0 || !mhat || !jac) return ORC_INVALID;
    const int S = net->S, M = net->M;
    const size_t cells = (size_t)G * S * M;
    rxn_info *info = (rxn_info *)malloc(sizeof(rxn_info) * M);
    long double *tot = (long double *)calloc(cells, sizeof(long double));
    long double *totl1 = (long double *)calloc(cells, sizeof(long double));
    if (!info || !tot || !totl1) { free(info); free(tot); free(totl1); return ORC_NOMEM; }
    build_info(net, info);
    int status = ORC_OK;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        jac_ctx jc;
        jc.S = S; jc.M = M; jc.mhat = mhat;
        jc.acc = (long double *)calloc(cells, sizeof(long double));
        jc.l1 = (long double *)calloc(cells, sizeof(long double));
        jc.z = (double *)calloc(M, sizeof(double));
        traj_state st;
        int ok = jc.acc && jc.l1 && jc.z && alloc_state(net, &st, info) == ORC_OK;
        int my_status = ok ? ORC_OK : ORC_NOMEM;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < N; ++i) {
            if (my_status != ORC_OK) continue;
            int r = run_trajectory(net, info, seed, (uint64_t)i, t_end, grid, G, max_events, &st, NULL, NULL,
                                   jac_visit, &jc);
            if (r != ORC_OK) my_status = r;
        }
#pragma omp critical
        {
            if (my_status != ORC_OK && status == ORC_OK) status = my_status;
            if (ok) for (size_t q = 0; q < cells; ++q) { tot[q] += jc.acc[q]; totl1[q] += jc.l1[q]; }
        }
        if (ok) free_state(&st);
        free(jc.acc); free(jc.l1); free(jc.z);
    }
    if (status == ORC_OK) {
        for (size_t q = 0; q < cells; ++q) {
            jac[q] = (double)(tot[q] / (long double)N);
            if (l1) l1[q] = (double)(totl1[q] / (long double)N);
        }
    }
    free(info); free(tot); free(totl1);
    return status;
}

/* ------------------------------------------------------------------------------------
 * Covariance between species at every grid point (a further associative, commutative
 * recombining function over the time-aligned states): exact 128-bit sums of X_s and
 * X_s X_r over the N trajectories, then
 *   cov_{g,s,r} = fl(N sum X_s X_r - sum X_s sum X_r) / (N (N - 1))   (0 when N = 1),
 * the variance formula with two species; cov_{g,s,s} is the variance.  Layout [G][S][S].
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int S;
    i128 *sx, *sxx;   /* [G*S], [G*S*S] */
} cov_ctx;

static void cov_visit(void *c, int g, const traj_state *st, double tg)
{
    (void)tg;
    cov_ctx *cc = (cov_ctx *)c;
    const int S = cc->S;
    for (int s = 0; s < S; ++s) {
        cc->sx[(size_t)g * S + s] += (i128)st->x[s];
        for (int r = 0; r < S; ++r)
            cc->sxx[((size_t)g * S + s) * S + r] += (i128)st->x[s] * (i128)st->x[r];
    }
}

int orc_covariance(const orc_net *net, int64_t N, double t_end, const double *grid, int32_t G,
                   uint64_t seed, uint64_t max_events, double *mean, double *cov, int nthreads)
{
    int st0 = check_net(net);
    if (st0) return st0;
    if (check_grid(grid, G, t_end)) return ORC_INVALID;
    if (N <= 0 || N > ((int64_t)1 << 30) || !mean || !cov) return ORC_INVALID;
    const int S = net->S, M = net->M;
    const size_t GS = (size_t)G * S, GSS = GS * S;
    rxn_info *info = (rxn_info *)malloc(sizeof(rxn_info) * M);
    i128 *sx = (i128 *)calloc(GS, sizeof(i128));
    i128 *sxx = (i128 *)calloc(GSS, sizeof(i128));
    if (!info || !sx || !sxx) { free(info); free(sx); free(sxx); return ORC_NOMEM; }
    build_info(net, info);
    int status = ORC_OK;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        cov_ctx cc;
        cc.S = S;
        cc.sx = (i128 *)calloc(GS, sizeof(i128));
        cc.sxx = (i128 *)calloc(GSS, sizeof(i128));
        traj_state st;
        int ok = cc.sx && cc.sxx && alloc_state(net, &st, info) == ORC_OK;
        int my_status = ok ? ORC_OK : ORC_NOMEM;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < N; ++i) {
            if (my_status != ORC_OK) continue;
            int r = run_trajectory(net, info, seed, (uint64_t)i, t_end, grid, G, max_events, &st, NULL, NULL,
                                   cov_visit, &cc);
            if (r != ORC_OK) my_status = r;
        }
#pragma omp critical
        {
            if (my_status != ORC_OK && status == ORC_OK) status = my_status;
            if (ok) {
                for (size_t q = 0; q < GS; ++q) sx[q] += cc.sx[q];
                for (size_t q = 0; q < GSS; ++q) sxx[q] += cc.sxx[q];
            }
        }
        if (ok) free_state(&st);
        free(cc.sx); free(cc.sxx);
    }
    if (status == ORC_OK) {
        for (int g = 0; g < G; ++g)
            for (int s = 0; s < S; ++s) {
                const size_t q = (size_t)g * S + s;
                mean[q] = (double)sx[q] / (double)N;
                for (int r = 0; r < S; ++r) {
                    const size_t qq = q * S + r;
                    if (N == 1) {
                        cov[qq] = 0.0;
                    } else {
                        i128 num = (i128)N * sxx[qq] - sx[q] * sx[(size_t)g * S + r];
                        cov[qq] = (double)num / ((double)N * (double)(N - 1));
                    }
                }
            }
    }
    free(info); free(sx); free(sxx);
    return status;
}

/* ------------------------------------------------------------------------------------
 * Adaptive selective memory (Section 3.2.1, Figure 3): the two curves of the figure,
 * computed for N trajectories without a caller grid.
 *   Avg-Y, the oversampled time-aligned average: its points are time 0 and every distinct
 *     time at which some trajectory applies an event (t <= t_end).  At a point every
 *     trajectory contributes its state after all of its own events up to and including
 *     that time (sample and hold), so the values are exactly orc_run's on a grid made of
 *     the point times -- and orc_run computes them.
 *   Avg-XY, the average along time: consecutive groups of k Avg-Y points, the last group
 *     possibly shorter (k' points), each give one point
 *       time = (t_1 + ... + t_k') / k',  mean = (m_1 + ... + m_k') / k',
 *       var  = (v_1 + ... + v_k') / k',
 *     every sum taken left to right in binary64, then one division.
 * The figure fixes the idea, not the arithmetic; the definitions above are this oracle's
 * reading.  Output sizes: U Avg-Y points, P = ceil(U / k) Avg-XY points; when a capacity is
 * too small the sizes are still returned, with ORC_INVALID.
 * ---------------------------------------------------------------------------------- */
typedef struct { double *t; int64_t n, cap; int fail; } time_log;

static void log_event_time(void *c, const traj_state *st)
{
    time_log *lg = (time_log *)c;
    if (lg->fail) return;
    if (lg->n == lg->cap) {
        int64_t nc = lg->cap ? 2 * lg->cap : 4096;
        double *nt = (double *)realloc(lg->t, sizeof(double) * (size_t)nc);
        if (!nt) { lg->fail = 1; return; }
        lg->t = nt;
        lg->cap = nc;
    }
    lg->t[lg->n++] = st->t;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* The Avg-Y points of N trajectories: {0} and every distinct applied-event time, ascending.
 * *pts is malloc'ed (caller frees); *U its length. */
static int union_times(const orc_net *net, const rxn_info *info, int64_t N, double t_end, uint64_t seed,
                       uint64_t max_events, int nthreads, double **pts_out, int64_t *U_out)
{
    time_log all = { NULL, 0, 0, 0 };
    int status = ORC_OK;
#pragma omp parallel num_threads(nthreads)
    {
        time_log lg = { NULL, 0, 0, 0 };
        traj_state st;
        int ok = alloc_state(net, &st, info) == ORC_OK;
        int my_status = ok ? ORC_OK : ORC_NOMEM;
        if (ok) { st.on_event = log_event_time; st.ev_ctx = &lg; }
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < N; ++i) {
            if (my_status != ORC_OK) continue;
            int r = run_trajectory(net, info, seed, (uint64_t)i, t_end, NULL, 0, max_events, &st, NULL, NULL,
                                   NULL, NULL);
            if (r != ORC_OK) my_status = r;
            if (lg.fail) my_status = ORC_NOMEM;
        }
#pragma omp critical
        {
            if (my_status != ORC_OK && status == ORC_OK) status = my_status;
            if (status == ORC_OK && lg.n > 0) {
                double *nt = (double *)realloc(all.t, sizeof(double) * (size_t)(all.n + lg.n + 1));
                if (!nt) {
                    status = ORC_NOMEM;
                } else {
                    all.t = nt;
                    memcpy(all.t + all.n, lg.t, sizeof(double) * (size_t)lg.n);
                    all.n += lg.n;
                }
            }
        }
        if (ok) free_state(&st);
        free(lg.t);
    }
    if (status != ORC_OK) { free(all.t); return status; }
    double *pts = (double *)malloc(sizeof(double) * (size_t)(all.n + 1));
    if (!pts) { free(all.t); return ORC_NOMEM; }
    if (all.n > 0) qsort(all.t, (size_t)all.n, sizeof(double), cmp_double);
    int64_t U = 0;
    pts[U++] = 0.0;
    for (int64_t e = 0; e < all.n; ++e)
        if (all.t[e] != pts[U - 1]) pts[U++] = all.t[e];
    free(all.t);
    *pts_out = pts;
    *U_out = U;
    return ORC_OK;
}

/* One Avg-XY point from the Avg-Y values of its group (m, v: [k'][S], t: [k']). */
static void xy_point(const double *t, const double *m, const double *v, int64_t kk, int S,
                     double *xt, double *xm, double *xv)
{
    double ts = 0.0;
    for (int64_t u = 0; u < kk; ++u) ts = ts + t[u];
    *xt = ts / (double)kk;
    for (int s = 0; s < S; ++s) {
        double ms = 0.0, vs = 0.0;
        for (int64_t u = 0; u < kk; ++u) {
            ms = ms + m[(size_t)u * S + s];
            vs = vs + v[(size_t)u * S + s];
        }
        xm[s] = ms / (double)kk;
        xv[s] = vs / (double)kk;
    }
}

int orc_adaptive(const orc_net *net, int64_t N, double t_end, uint64_t seed, uint64_t max_events, int64_t k,
                 int64_t cap_y, int64_t *n_y, double *y_time, double *y_mean, double *y_var,
                 int64_t cap_xy, int64_t *n_xy, double *xy_time, double *xy_mean, double *xy_var, int nthreads)
{
    int st0 = check_net(net);
    if (st0) return st0;
    if (N <= 0 || N > ((int64_t)1 << 30) || k <= 0 || !(t_end >= 0.0) || !isfinite(t_end)) return ORC_INVALID;
    const int S = net->S, M = net->M;
    rxn_info *info = (rxn_info *)malloc(sizeof(rxn_info) * M);
    if (!info) return ORC_NOMEM;
    build_info(net, info);
    if (nthreads <= 0) nthreads = 1;
    double *pts = NULL;
    int64_t U = 0;
    int status = union_times(net, info, N, t_end, seed, max_events, nthreads, &pts, &U);
    if (status != ORC_OK) { free(info); return status; }
    const int64_t P = (U + k - 1) / k;
    if (n_y) *n_y = U;
    if (n_xy) *n_xy = P;
    if (U > cap_y || P > cap_xy || U > INT32_MAX) { free(pts); free(info); return ORC_INVALID; }
    /* Avg-Y: the grid reduction at the point times */
    status = orc_run(net, N, t_end, pts, (int32_t)U, seed, max_events, 0, 0, 1, 1, y_mean, y_var, NULL, NULL, NULL,
                     nthreads);
    if (status == ORC_OK) {
        memcpy(y_time, pts, sizeof(double) * (size_t)U);
        for (int64_t p = 0; p < P; ++p) {
            const int64_t u0 = p * k, u1 = (u0 + k < U) ? u0 + k : U;
            xy_point(pts + u0, y_mean + (size_t)u0 * S, y_var + (size_t)u0 * S, u1 - u0, S, xy_time + p,
                     xy_mean + (size_t)p * S, xy_var + (size_t)p * S);
        }
    }
    free(pts);
    free(info);
    return status;
}

/* The same reduction for chosen Avg-XY groups only (for runs whose Avg-Y is too long to
 * evaluate whole): all Avg-Y point times (times [cap], U), and for each group in groups
 * [n_groups] its Avg-XY point (g_time [n], g_mean / g_var [n][S]) from the grid reduction
 * at that group's points alone. */
int orc_adaptive_groups(const orc_net *net, int64_t N, double t_end, uint64_t seed, uint64_t max_events, int64_t k,
                        int64_t n_groups, const int64_t *groups, int64_t cap, int64_t *n_y, double *times,
                        double *g_time, double *g_mean, double *g_var, int nthreads)
{
    int st0 = check_net(net);
    if (st0) return st0;
    if (N <= 0 || N > ((int64_t)1 << 30) || k <= 0 || !(t_end >= 0.0) || !isfinite(t_end)) return ORC_INVALID;
    const int S = net->S, M = net->M;
    rxn_info *info = (rxn_info *)malloc(sizeof(rxn_info) * M);
    if (!info) return ORC_NOMEM;
    build_info(net, info);
    if (nthreads <= 0) nthreads = 1;
    double *pts = NULL;
    int64_t U = 0;
    int status = union_times(net, info, N, t_end, seed, max_events, nthreads, &pts, &U);
    if (status != ORC_OK) { free(info); return status; }
    if (n_y) *n_y = U;
    const int64_t P = (U + k - 1) / k;
    if (U > cap) { free(pts); free(info); return ORC_INVALID; }
    memcpy(times, pts, sizeof(double) * (size_t)U);
    for (int64_t q = 0; q < n_groups && status == ORC_OK; ++q) {
        const int64_t p = groups[q];
        if (p < 0 || p >= P || k > INT32_MAX) { status = ORC_INVALID; break; }
        const int64_t u0 = p * k, u1 = (u0 + k < U) ? u0 + k : U;
        const int64_t kk = u1 - u0;
        double *m = (double *)malloc(sizeof(double) * (size_t)kk * S);
        double *v = (double *)malloc(sizeof(double) * (size_t)kk * S);
        if (!m || !v) { free(m); free(v); status = ORC_NOMEM; break; }
        status = orc_run(net, N, t_end, pts + u0, (int32_t)kk, seed, max_events, 0, 0, 1, 1, m, v, NULL, NULL, NULL,
                         nthreads);
        if (status == ORC_OK)
            xy_point(pts + u0, m, v, kk, S, g_time + q, g_mean + (size_t)q * S, g_var + (size_t)q * S);
        free(m);
        free(v);
    }
    free(pts);
    free(info);
    return status;
}
