// ssa_api.hip -- host runtime behind include/ssa.h: validation, device layout of a model,
// per-network kernel specialisation (run-time compilation), work lists, launches,
// finalize and error reporting.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ssa.h"
#include "ssa_wave.hpp"

using namespace ssa;

// The scratch area of ssa_run_device_static: every GPU the library runs on holds its own
// copy until the process ends.  Host code never uses the symbol itself (on the host it is
// a stand-in, not a device address): it takes each device's address once, with that device
// current, from hipGetSymbolAddress (static_scratch below).
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Device sources of the run-time specialised kernels, embedded at build time.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wc23-extensions"
const char kSrcDevice[] = {
#embed "ssa_device.hpp"
    , 0};
const char kSrcSim[] = {
#embed "ssa_sim.hpp"
    , 0};
const char kSrcJit[] = {
#embed "ssa_jit.hpp"
    , 0};
#pragma clang diagnostic pop

thread_local std::string g_err;

ssa_status fail(ssa_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? SSA_E_NOMEM : SSA_E_DEVICE, "%s: %s (%s:%d)",  \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                         \
    } while (0)

constexpr int32_t kMaxSpecies = 1024;
static_assert(2 * kMaxSpecies + 1 <= kXyTile, "an Avg-XY tile must hold one point of every chain");
constexpr int32_t kMaxReactions = 4096;
constexpr int32_t kMaxProduct = (1 << 19) - 4;
constexpr uint64_t kDefaultMaxEvents = 1ull << 62;
constexpr int32_t kJitMaxReactions = 32;     // specialised kernels keep a_j, S_j in registers
constexpr int32_t kJitMaxSpecies = 64;
constexpr int32_t kWaveMaxQ = 8;            // 64-chunk order: reactions per lane held in registers
constexpr int64_t kMaxDepEntries = (int64_t)1 << 24;   // dependency lists beyond this: full re-evaluation

// Device memory one call needs beyond its inputs and outputs.
struct Scratch {
    virtual ~Scratch() = default;
    virtual hipError_t alloc(void **p, size_t bytes) = 0;
};

// Stream-ordered allocations of one call, released on the stream in reverse order.
struct StreamScratch : Scratch {
    hipStream_t stream;
    std::vector<void *> ptrs;
    explicit StreamScratch(hipStream_t s) : stream(s) {}
    hipError_t alloc(void **p, size_t bytes) override {
        hipError_t e = hipMallocAsync(p, std::max<size_t>(bytes, 256), stream);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    ~StreamScratch() override {
        for (auto it = ptrs.rbegin(); it != ptrs.rend(); ++it) (void)hipFreeAsync(*it, stream);
    }
};

// Consecutive 256-byte aligned pieces of a fixed device area (no allocation call).
struct FixedScratch : Scratch {
    char *base;
    size_t cap, used = 0;
    FixedScratch(void *b, size_t c) : base((char *)b), cap(c) {}
    static size_t piece(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255; }
    hipError_t alloc(void **p, size_t bytes) override {
        const size_t b = piece(bytes);
        if (used + b > cap) return hipErrorOutOfMemory;
        *p = base + used;
        used += b;
        return hipSuccess;
    }
};

// Scratch of a call made while its stream is captured into a graph: each piece is a
// hipMalloc of its own (taken with this thread's capture mode relaxed, since the caller may
// capture in global mode), which the model keeps until ssa_model_destroy, so that every
// replay of the graph finds its scratch in place and allocates nothing.
struct CaptureScratch : Scratch {
    const ssa_model *m;
    explicit CaptureScratch(const ssa_model *model);
    hipError_t alloc(void **p, size_t bytes) override;
};

std::mutex g_static_mu;
void *g_static_ptr[64] = {};

// The current device's address of the scratch area (looked up at the first call on the device).
ssa_status static_scratch(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (dev < 0 || dev >= 64) return fail(SSA_E_UNSUPPORTED, "device index %d beyond 63", dev);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SSA_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return SSA_OK;
}

// Keep freed stream-ordered memory in the pool between calls instead of returning it.
void keep_pool(int dev) {
    static std::once_flag once[64];
    if (dev < 0 || dev >= 64) return;
    std::call_once(once[dev], [dev] {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = ~0ull;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    });
}

int cu_count(int dev) {
    static int cache[64] = {0};
    if (dev >= 0 && dev < 64 && cache[dev]) return cache[dev];
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    if (dev >= 0 && dev < 64) cache[dev] = n;
    return n;
}

// LDS one block may use (bytes).
size_t lds_max(int dev) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || n <= 0)
        n = 64 * 1024;
    return (size_t)n;
}

// Launch form and grid size of the last simulation kernel this thread launched (copied into
// ssa_stats.form / ssa_stats.blocks).
struct LaunchRec {
    uint32_t form = SSA_FORM_NONE;
    uint32_t blocks = 0;
    uint32_t ordered = 0;
};
thread_local LaunchRec g_launch;

void note_launch(uint32_t form, int64_t blocks, bool ordered = false) {
    g_launch.form = form;
    g_launch.blocks = (uint32_t)blocks;
    g_launch.ordered = ordered ? 1u : 0u;
}

// Launch form requested for the specialised kernels by SSA_LAUNCH_FORM (two_wave,
// generations or refill; SSA_FORM_NONE when unset).  Forms a kernel kind does not have are
// ignored there (the forward has no refill form).  Every form gives the same bits.
uint32_t forced_form() {
    const char *e = std::getenv("SSA_LAUNCH_FORM");
    if (!e) return SSA_FORM_NONE;
    if (std::strcmp(e, "two_wave") == 0) return SSA_FORM_TWO_WAVE;
    if (std::strcmp(e, "generations") == 0) return SSA_FORM_GENERATIONS;
    if (std::strcmp(e, "refill") == 0) return SSA_FORM_REFILL;
    return SSA_FORM_NONE;
}

// Kernel choice for single-network launches: the kernel specialised to the network
// (default) or the compiled table-driven one (SSA_KERNEL=generic).  Both give bit-identical
// results; the variable only selects the implementation.
bool prefer_generic() {
    const char *e = std::getenv("SSA_KERNEL");
    return e && std::strcmp(e, "generic") == 0;
}

// ---------------------------------------------------------------------------------------
// Run-time specialisation
// ---------------------------------------------------------------------------------------
struct JitKernels {
    hipModule_t module = nullptr;
    hipFunction_t fwd = nullptr, fwd_atomic = nullptr, fwd_hist = nullptr, fwd_slab_hist = nullptr, fwd_jac = nullptr,
                  fwd_cov = nullptr,
                  rec = nullptr, bwd = nullptr, bwd_var = nullptr, evt = nullptr, bwd_gen = nullptr,
                  bwd_var_gen = nullptr, bwd_pc = nullptr, bwd_var_pc = nullptr, fwd_pc = nullptr,
                  fwd_hist_pc = nullptr, evt_pc = nullptr, fwd_epoch = nullptr, fwd_hist_epoch = nullptr,
                  fwd_epoch_pc = nullptr, fwd_hist_epoch_pc = nullptr;
};

std::mutex g_jit_mu;
std::map<std::tuple<int, std::string, bool>, std::shared_ptr<JitKernels>> g_jit_cache;

std::string device_arch(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "gfx950";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

}  // namespace

struct ssa_model {
    int32_t S = 0, M = 0, device = 0;
    std::vector<int32_t> reac, prod;  // [M*S] as given
    std::vector<double> rate;         // [M]
    std::vector<int32_t> x0;          // [S]
    int32_t m_pad = 0;                // generic tables padded to this many reactions
    int32_t max_changes = 0;          // largest number of species one reaction changes
    int32_t order = SSA_SUM_SEQ;      // propensity sum order
    int32_t q = 1;                    // 64-chunk order: reactions per lane (ceil(M / 64))
    uint32_t *d_rx = nullptr;         // [m_pad] packed reactant encoding
    double *d_rate = nullptr;         // [m_pad] zero-padded rates
    int32_t *d_chg = nullptr;         // [M * kChg] packed changes
    int32_t *d_x0 = nullptr;          // [S]
    int2 *d_dep = nullptr;            // 64-chunk order above kWaveMaxQ per lane: dependency lists
    double *d_dep_rate = nullptr;     // [dep_nnz] the model's rate of each entry's reaction
    int32_t *d_dep_ptr = nullptr;     // [M + 1]
    int64_t dep_nnz = 0;
    std::string jit_src;              // generated network description for specialisation
    bool has_laws = false;            // some rate constant depends on a species (ssa_rate_law)
    std::vector<ssa_rate_law> laws;   // [M] when has_laws
    mutable std::mutex cap_mu;
    mutable std::vector<void *> cap_mem;   // scratch of calls captured into graphs (freed with the model)
    // the event count of every trajectory of the last forward in generations, and that
    // run's identity: a backward over the same trajectories orders them by length
    mutable std::mutex hint_mu;
    mutable uint32_t *hint_len = nullptr;
    mutable int64_t hint_cap = 0;
    mutable bool hint_valid = false;
    mutable int64_t hint_n = 0;
    mutable double hint_t_end = 0.0;
    mutable uint64_t hint_seed = 0, hint_max_events = 0;
    mutable const double *hint_grid = nullptr, *hint_rates = nullptr, *hint_log_rates = nullptr;
    mutable int32_t hint_G = 0;
    mutable int hint_dev = -1;
    mutable std::vector<void *> hint_old;  // replaced buffers (a launch may still read one)
};

namespace {

CaptureScratch::CaptureScratch(const ssa_model *model) : m(model) {}

hipError_t CaptureScratch::alloc(void **p, size_t bytes) {
    hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
    hipError_t e = hipThreadExchangeStreamCaptureMode(&mode);
    if (e != hipSuccess) return e;
    e = hipMalloc(p, std::max<size_t>(bytes, 256));
    (void)hipThreadExchangeStreamCaptureMode(&mode);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(m->cap_mu);
    m->cap_mem.push_back(*p);
    return hipSuccess;
}

}  // namespace

struct ssa_batch {
    int32_t B = 0, device = 0, s_rows = 0, m_rows = 0, mm = 0;
    std::vector<const ssa_model *> models;
    std::vector<int64_t> n_traj;
    std::vector<int32_t> G;
    NetDev *d_nets = nullptr;
    int32_t *d_item_net = nullptr;
    int64_t *d_item_begin = nullptr;
    int32_t *d_item_count = nullptr;
    int32_t n_items = 0;
    std::vector<double *> d_grids;
    unsigned long long *d_D = nullptr;      // per network [G][S][2] sums then [G][S] high parts
    size_t D_words = 0;
    std::vector<size_t> D_off;
    unsigned int *d_counter = nullptr;
    unsigned long long *d_stats = nullptr;
    GridInfo *d_ginfo = nullptr;
    // finalize table (one entry per network; the output pointers of the last run)
    std::vector<FinalNet> fin;
    FinalNet *d_fin = nullptr;
    int32_t *d_block_net = nullptr, *d_block_species = nullptr;
    int32_t n_fin_blocks = 0;
    // the launch sequence captured as a graph on first use, replayed afterwards
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t win_bytes = 0;            // LDS window bytes per cohort (0: built-in default), see ssa_batch_autotune
    LaunchRec launch;                 // form and grid of the captured simulation launch
};

// A run taken in epochs of simulation time (ssa_run_begin / advance / finish): the device
// copies of the grid and rates, the exact sums so far, the trajectories' saved states
// (double-buffered: read one, write the other) and the host totals.
struct ssa_run_state {
    const ssa_model *m = nullptr;
    int device = 0;
    int64_t n_traj = 0;
    double t_end = 0.0, t_done = 0.0;
    int32_t G = 0;
    uint64_t seed = 0, max_events = 0;
    bool has_hist = false, started = false;
    ssa_hist_spec hist{};
    double *d_grid = nullptr, *d_rates = nullptr;
    unsigned long long *D = nullptr, *Dhi = nullptr;
    int32_t *Hd = nullptr;
    void *ctl = nullptr;
    int32_t *sx[2] = {nullptr, nullptr};
    double *st[2] = {nullptr, nullptr};
    uint64_t *sk[2] = {nullptr, nullptr}, *sev[2] = {nullptr, nullptr};
    int cur = -1;                      // buffer holding the saved states (-1: none yet)
    unsigned long long events = 0, max_steps = 0;
    uint32_t flags = 0;
    float kernel_ms = 0.f;
};

namespace {

// FNV-1a over the embedded kernel sources.  Stamped into every generated program so a
// compilation cache keyed on the main source text can never return code built from
// different headers.
uint64_t kernel_sources_hash() {
    uint64_t h = 1469598103934665603ull;
    for (const char *src : {kSrcDevice, kSrcSim, kSrcJit})
        for (const char *c = src; *c; ++c) h = (h ^ (unsigned char)*c) * 1099511628211ull;
    return h;
}

// Generated description of one network for ssa_jit.hpp.
std::string generate_net_source(const ssa_model *m) {
    const int32_t S = m->S, M = m->M;
    std::string s;
    char buf[512];
    snprintf(buf, sizeof buf, "// kernel sources %016llx\n", (unsigned long long)kernel_sources_hash());
    s += buf;
    s += "#include \"ssa_device.hpp\"\nnamespace ssa_gen {\nstruct Net {\n";
    snprintf(buf, sizeof buf, "    static constexpr int S = %d, M = %d;\n", S, M);
    s += buf;
    s += "    __device__ static __forceinline__ void init(int32_t (&x)[S]) {\n";
    for (int32_t q = 0; q < S; ++q) {
        snprintf(buf, sizeof buf, "        x[%d] = %d;\n", q, m->x0[q]);
        s += buf;
    }
    s += "    }\n";
    s += "    template <class R>\n    __device__ static __forceinline__ void props(const int32_t (&x)[S], R c, "
         "double (&a)[M]) {\n";
    for (int32_t j = 0; j < M; ++j) {
        int32_t order = 0, sa = -1, sb = -1;
        for (int32_t q = 0; q < S; ++q) {
            const int32_t r = m->reac[(size_t)j * S + q];
            for (int32_t t = 0; t < r; ++t) (sa < 0 ? sa : sb) = q;
            order += r;
        }
        // the rate constant: c_j, or its rate law min(max(c_j + slope x_m, lo), hi)
        std::string cj = "c[" + std::to_string(j) + "]";
        if (m->has_laws && m->laws[j].species >= 0) {
            const ssa_rate_law &L = m->laws[j];
            snprintf(buf, sizeof buf, "(%s + %a * (double)x[%d])", cj.c_str(), L.slope, L.species);
            cj = buf;
            snprintf(buf, sizeof buf, "fmax(%s, %a)", cj.c_str(), L.lo);
            cj = buf;
            if (std::isfinite(L.hi)) {
                snprintf(buf, sizeof buf, "fmin(%s, %a)", cj.c_str(), L.hi);
                cj = buf;
            }
        }
        if (order == 0)
            snprintf(buf, sizeof buf, "        a[%d] = %s * 1.0;\n", j, cj.c_str());
        else if (order == 1)
            snprintf(buf, sizeof buf, "        a[%d] = %s * (double)x[%d];\n", j, cj.c_str(), sa);
        else if (sa != sb)
            snprintf(buf, sizeof buf, "        a[%d] = %s * ((double)x[%d] * (double)x[%d]);\n", j, cj.c_str(), sa, sb);
        else
            snprintf(buf, sizeof buf, "        a[%d] = %s * (((double)x[%d] * (double)max(x[%d] - 1, 0)) * 0.5);\n", j,
                     cj.c_str(), sa, sa);
        s += buf;
    }
    s += "    }\n";
    // the change of species q by reaction j: a 4-bit field (delta + 8) of one or two
    // 64-bit constants when every delta lies in [-8, 7] (no branches on the divergent j),
    // else a select chain
    std::string changed;
    s += "    __device__ static __forceinline__ void deltas(int32_t j, int32_t (&d)[S]) {\n";
    for (int32_t q = 0; q < S; ++q) {
        bool any = false, small = M <= 32;
        uint64_t K[2] = {0, 0};
        for (int32_t j = 0; j < M; ++j) {
            const int32_t dl = m->prod[(size_t)j * S + q] - m->reac[(size_t)j * S + q];
            any = any || dl != 0;
            small = small && dl >= -8 && dl <= 7;
            if (small) K[j / 16] |= (uint64_t)(dl + 8) << (4 * (j % 16));
        }
        for (int32_t j = M; j < 32; ++j) K[j / 16] |= (uint64_t)8 << (4 * (j % 16));
        changed += any ? (q ? ", true" : "true") : (q ? ", false" : "false");
        std::string e;
        if (!any) {
            e = "0";
        } else if (small && M <= 16) {
            snprintf(buf, sizeof buf, "(int32_t)((0x%016llxull >> (4 * j)) & 15ull) - 8", (unsigned long long)K[0]);
            e = buf;
        } else if (small) {
            snprintf(buf, sizeof buf,
                     "(int32_t)(((j < 16 ? 0x%016llxull : 0x%016llxull) >> (4 * (j & 15))) & 15ull) - 8",
                     (unsigned long long)K[0], (unsigned long long)K[1]);
            e = buf;
        } else {
            e = "0";
            for (int32_t j = M - 1; j >= 0; --j) {
                const int32_t dl = m->prod[(size_t)j * S + q] - m->reac[(size_t)j * S + q];
                if (!dl) continue;
                snprintf(buf, sizeof buf, "(j == %d ? %d : %s)", j, dl, e.c_str());
                e = buf;
            }
        }
        s += "        d[" + std::to_string(q) + "] = " + e + ";\n";
    }
    s += "    }\n";
    // species that some reaction changes (the others are never touched)
    s += "    __device__ static constexpr bool changes(int q) {\n";
    s += "        constexpr bool c[S] = {" + changed + "};\n";
    s += "        return c[q];\n    }\n";
    s += "};\n}  // namespace ssa_gen\n#include \"ssa_jit.hpp\"\n";
    return s;
}

// A launch of n_items work items (64 trajectories each, one wave apiece) that leaves most
// SIMDs with at most two waves runs at the latency of a wave's dependency chains rather
// than at the chip's issue rate.
bool latency_bound(int64_t n_items, int dev) { return n_items <= (int64_t)2 * 4 * cu_count(dev); }

// Launches of at most two work items per CU run the specialised forward and backward in
// blocks of two waves, one simulating and one computing the draws (each wave on its own
// SIMD); SSA_DRAW_WAVE=0 turns this off.
bool pc_launch(int64_t n_items, int dev) {
    const char *e = std::getenv("SSA_DRAW_WAVE");
    if (e && std::strcmp(e, "0") == 0) return false;
    return n_items <= (int64_t)2 * cu_count(dev);
}

// The network's kernels compiled at run time; ilp: scheduled for latency-bound launches
// (independent chains interleaved), else for throughput (the default scheduler, which
// measured faster once several waves share a SIMD).
bool jit_cached(const ssa_model *m, int dev, bool ilp) {
    std::lock_guard<std::mutex> lk(g_jit_mu);
    return g_jit_cache.count(std::make_tuple(dev, m->jit_src, ilp)) != 0;
}

ssa_status get_jit(const ssa_model *m, int dev, std::shared_ptr<JitKernels> &out, bool ilp = false) {
    const auto key = std::make_tuple(dev, m->jit_src, ilp);
    {
        std::lock_guard<std::mutex> lk(g_jit_mu);
        auto it = g_jit_cache.find(key);
        if (it != g_jit_cache.end()) {
            out = it->second;
            return SSA_OK;
        }
    }
    hiprtcProgram prog;
    const char *hdrs[] = {kSrcDevice, kSrcSim, kSrcJit};
    const char *names[] = {"ssa_device.hpp", "ssa_sim.hpp", "ssa_jit.hpp"};
    if (hiprtcCreateProgram(&prog, m->jit_src.c_str(), "ssa_net.hip", 3, hdrs, names) != HIPRTC_SUCCESS)
        return fail(SSA_E_DEVICE, "hiprtcCreateProgram failed");
    const std::string arch = "--offload-arch=" + device_arch(dev);
    // ilp: the instruction scheduler that interleaves independent chains.  A lone wave per
    // SIMD runs the event loop at the latency of its dependency chains, and the loop carries
    // two of them (the next draw's variates; the propensities and the division).
    const char *opts[] = {arch.c_str(), "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                          "-mllvm", "-amdgpu-sched-strategy=max-ilp"};
    const int n_opts = (int)(sizeof opts / sizeof opts[0]) - (ilp ? 0 : 2);
    const hiprtcResult rc = hiprtcCompileProgram(prog, n_opts, opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(SSA_E_DEVICE, "run-time compilation failed: %s", log.substr(0, 800).c_str());
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    std::vector<char> code(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    auto k = std::make_shared<JitKernels>();
    HIP_TRY(hipModuleLoadData(&k->module, code.data()));
    HIP_TRY(hipModuleGetFunction(&k->fwd, k->module, "ssa_jit_fwd"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_atomic, k->module, "ssa_jit_fwd_atomic"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_hist, k->module, "ssa_jit_fwd_hist"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_slab_hist, k->module, "ssa_jit_fwd_slab_hist"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_jac, k->module, "ssa_jit_fwd_jac"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_cov, k->module, "ssa_jit_fwd_cov"));
    HIP_TRY(hipModuleGetFunction(&k->rec, k->module, "ssa_jit_rec"));
    HIP_TRY(hipModuleGetFunction(&k->evt, k->module, "ssa_jit_evt"));
    HIP_TRY(hipModuleGetFunction(&k->bwd_var, k->module, "ssa_jit_bwd_var"));
    HIP_TRY(hipModuleGetFunction(&k->bwd, k->module, "ssa_jit_bwd"));
    HIP_TRY(hipModuleGetFunction(&k->bwd_gen, k->module, "ssa_jit_bwd_gen"));
    HIP_TRY(hipModuleGetFunction(&k->bwd_var_gen, k->module, "ssa_jit_bwd_var_gen"));
    HIP_TRY(hipModuleGetFunction(&k->bwd_pc, k->module, "ssa_jit_bwd_pc"));
    HIP_TRY(hipModuleGetFunction(&k->bwd_var_pc, k->module, "ssa_jit_bwd_var_pc"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_pc, k->module, "ssa_jit_fwd_pc"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_hist_pc, k->module, "ssa_jit_fwd_hist_pc"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_epoch, k->module, "ssa_jit_fwd_epoch"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_hist_epoch, k->module, "ssa_jit_fwd_hist_epoch"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_epoch_pc, k->module, "ssa_jit_fwd_epoch_pc"));
    HIP_TRY(hipModuleGetFunction(&k->fwd_hist_epoch_pc, k->module, "ssa_jit_fwd_hist_epoch_pc"));
    HIP_TRY(hipModuleGetFunction(&k->evt_pc, k->module, "ssa_jit_evt_pc"));
    std::lock_guard<std::mutex> lk(g_jit_mu);
    auto ins = g_jit_cache.emplace(key, k);
    out = ins.first->second;
    return SSA_OK;
}

bool jit_eligible(const ssa_model *m) {
    // networks with rate laws exist only in specialised form
    return (m->has_laws || !prefer_generic()) && m->M <= kJitMaxReactions && m->S <= kJitMaxSpecies;
}

// Whether the caller's stream is being captured into a graph.  A captured call takes its
// scratch from CaptureScratch, compiles nothing (specialised: the call runs the network's
// specialised kernels, whose form ilp must exist from an earlier call on this device) and
// synchronises nothing (no statistics); every check comes before the call's first stream
// operation, so a refused call leaves the capture as it was.
ssa_status capture_check(const ssa_model *m, hipStream_t st, int dev, const ssa_stats *stats, bool specialised,
                         bool ilp, bool *capturing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return fail(SSA_E_DEVICE, "hipStreamIsCapturing: %s", hipGetErrorString(e));
    if (cs == hipStreamCaptureStatusInvalidated) return fail(SSA_E_INVALID, "the stream's capture is invalidated");
    *capturing = cs == hipStreamCaptureStatusActive;
    if (!*capturing) return SSA_OK;
    if (stats)
        return fail(SSA_E_INVALID, "statistics are read back with a synchronisation: pass none while the stream is "
                                   "captured");
    if (specialised && !jit_cached(m, dev, ilp))
        return fail(SSA_E_INVALID, "the network's kernels are compiled by its first call on a device: make one "
                                   "call of the same size before capturing");
    return SSA_OK;
}

ssa_status validate_grid_host(const double *grid, int32_t G, double t_end) {
    if (!(t_end >= 0.0) || !std::isfinite(t_end)) return fail(SSA_E_INVALID, "t_end must be finite and >= 0");
    if (G <= 0 || !grid) return fail(SSA_E_INVALID, "grid must have at least one point");
    for (int32_t g = 0; g < G; ++g) {
        if (!(grid[g] >= 0.0) || !(grid[g] <= t_end))
            return fail(SSA_E_INVALID, "grid[%d] = %g outside [0, t_end]", g, grid[g]);
        if (g && !(grid[g] >= grid[g - 1])) return fail(SSA_E_INVALID, "grid decreases at %d", g);
    }
    return SSA_OK;
}

NetDev base_net(const ssa_model *m, const double *rates, int64_t n_traj, double t_end, const double *grid,
                int32_t G, uint64_t seed, uint64_t max_events) {
    NetDev n;
    std::memset(&n, 0, sizeof n);
    n.S = m->S;
    n.M = m->M;
    n.G = G;
    n.n_traj = n_traj;
    n.t_end = t_end;
    n.key0 = (uint32_t)seed;
    n.key1 = (uint32_t)(seed >> 32);
    n.max_events = max_events ? max_events : kDefaultMaxEvents;
    n.rx = m->d_rx;
    n.rate = rates ? rates : m->d_rate;
    n.chg = m->d_chg;
    n.x0 = m->d_x0;
    n.grid = grid;
    n.q = m->q;
    n.dep = m->d_dep;
    n.dep_rate = m->d_dep_rate;
    n.dep_ptr = m->d_dep_ptr;
    return n;
}

// generic kernel: register slots for a_j and S_j (0 = two-pass variant for large M)
int generic_mm(int32_t M) { return M <= 8 ? 8 : (M <= 16 ? 16 : (M <= 32 ? 32 : 0)); }

int64_t grid_blocks(int per_cu, int dev, int64_t n_items) {
    per_cu = std::max(per_cu, 1);
    int64_t blocks = std::min<int64_t>((int64_t)per_cu * cu_count(dev), (n_items + 3) / 4);
    return std::max<int64_t>(blocks, 1);
}

size_t generic_lds(const WorkList &wl) {
    return (size_t)(wl.s_rows + 1) * kBlock * sizeof(int32_t) +
           (size_t)(kBlock / kWave) * wl.m_rows * kChg * sizeof(int32_t);
}

template <int MODE, int MM, bool BATCH, bool QUAD = false>
hipError_t launch_generic_mm(const WorkList &wl, int64_t n_items, int dev, hipStream_t st) {
    auto kern = sim_kernel<MODE, MM, BATCH, QUAD>;
    const size_t lds = generic_lds(wl);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, lds);
    if (e != hipSuccess) return e;
    const int64_t blocks = grid_blocks(per_cu, dev, n_items);
    note_launch(SSA_FORM_TABLE, blocks);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), lds, st, wl);
    return hipGetLastError();
}

template <int MODE, bool BATCH, bool QUAD = false>
hipError_t launch_generic(int mm, const WorkList &wl, int64_t n_items, int dev, hipStream_t st) {
    if (mm == 8) return launch_generic_mm<MODE, 8, BATCH, QUAD>(wl, n_items, dev, st);
    if (mm == 16) return launch_generic_mm<MODE, 16, BATCH, QUAD>(wl, n_items, dev, st);
    if (mm == 32) return launch_generic_mm<MODE, 32, BATCH, QUAD>(wl, n_items, dev, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------
// Forward launches (selective-memory windows, see ssa_sim.hpp)
// ---------------------------------------------------------------------------------------

// Bytes of LDS per window (SSA_WIN_BYTES overrides; 512 .. 16384).  The specialised
// kernels (one window per wave, state in registers) do best with 8 KB on the 4-species
// network (4 KB: +5 % forward time, 2 KB: +20 % on the 10^4-point grid); the table-driven
// kernel holds two windows next to its LDS state columns, where 4 KB keeps two blocks per
// CU (8 KB slowed the batched workload by half).
size_t window_budget(bool generic, int32_t tuned = 0) {
    size_t b = generic ? 4096 : 8192;
    if (const char *e = std::getenv("SSA_WIN_BYTES")) b = (size_t)std::strtoull(e, nullptr, 10);
    if (tuned > 0) b = (size_t)tuned;
    return std::min<size_t>(std::max<size_t>(b, 512), 16384);
}

// Window length in bins: the largest power of two whose S x 2 int64 words per bin fit the
// budget, capped at 1024 and at the grid length rounded up to a power of two.
int32_t window_bins(int32_t S, int32_t G, bool generic, int32_t tuned = 0) {
    const size_t per_bin = (size_t)S * 2 * sizeof(long long);
    int32_t W = 1;
    while (W < 1024 && (size_t)(2 * W) * per_bin <= window_budget(generic, tuned) && W < G) W *= 2;
    return W;
}

// Flush target of the forward windows: atomic adds into the totals (default), or wave-
// private slabs summed by a reduction kernel afterwards (SSA_FWD_FLUSH=slab, when the slabs
// fit in SSA_SLAB_BYTES, default 1 GiB).  Both give identical sums; on the 4-species
// workloads they run at the same speed, and the atomic form needs no slab memory.
bool want_slabs(size_t slab_bytes, int32_t tuned = -1) {
    const char *e = std::getenv("SSA_FWD_FLUSH");
    const bool asked = tuned >= 0 ? tuned == 1 : (e && std::strcmp(e, "slab") == 0);
    if (!asked) return false;
    size_t b = (size_t)1 << 30;
    if (const char *q = std::getenv("SSA_SLAB_BYTES")) b = (size_t)std::strtoull(q, nullptr, 10);
    return slab_bytes <= b;
}

struct FwdKernel {
    bool jit = false;
    hipFunction_t f_slab = nullptr, f_atomic = nullptr;     // run-time specialised
    const void *g_slab = nullptr, *g_atomic = nullptr;      // generic
    size_t lds = 0;
};

template <int MM, bool BATCH>
void generic_fwd_kernels(FwdKernel &k) {
    k.g_slab = (const void *)fwd_kernel<MM, BATCH, true>;
    k.g_atomic = (const void *)fwd_kernel<MM, BATCH, false>;
}

template <bool BATCH>
bool pick_generic_fwd(int mm, FwdKernel &k) {
    if (mm == 8) generic_fwd_kernels<8, BATCH>(k);
    else if (mm == 16) generic_fwd_kernels<16, BATCH>(k);
    else if (mm == 32) generic_fwd_kernels<32, BATCH>(k);
    else if (mm == 0) generic_fwd_kernels<0, BATCH>(k);
    else return false;
    return true;
}

hipError_t fwd_blocks(const FwdKernel &k, bool slab, int dev, int64_t n_items, int64_t &blocks) {
    int per_cu = 0;
    hipError_t e = k.jit ? hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, slab ? k.f_slab : k.f_atomic,
                                                                                kBlock, k.lds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, slab ? k.g_slab : k.g_atomic, kBlock,
                                                                        k.lds);
    if (e != hipSuccess) return e;
    blocks = grid_blocks(per_cu, dev, n_items);
    return hipSuccess;
}

// lone: blocks of one wave (the specialised atomic-flush kernel only), for launches of at
// most one work item per CU
hipError_t fwd_launch(const FwdKernel &k, bool slab, int64_t blocks, WorkList &wl, hipStream_t st,
                      bool lone = false) {
    note_launch(k.jit ? SSA_FORM_GENERATIONS : SSA_FORM_TABLE, blocks, wl.perm != nullptr);
    if (k.jit) {
        void *args[] = {&wl};
        if (lone)
            return hipModuleLaunchKernel(k.f_atomic, (unsigned)blocks, 1, 1, kWave, 1, 1,
                                         (unsigned)(k.lds / (kBlock / kWave)), st, args, nullptr);
        return hipModuleLaunchKernel(slab ? k.f_slab : k.f_atomic, (unsigned)blocks, 1, 1, kBlock, 1, 1,
                                     (unsigned)k.lds, st, args, nullptr);
    }
    void *args[] = {&wl};
    return hipLaunchKernel(slab ? k.g_slab : k.g_atomic, dim3((unsigned)blocks), dim3(kBlock), args, k.lds, st);
}

// max_blocks > 0 caps the persistent grid (a tuned launch), else the occupancy limit.
hipError_t launch_jit(hipFunction_t f, WorkList &wl, int64_t n_items, int dev, hipStream_t st, uint32_t form,
                      int64_t max_blocks = 0) {
    int per_cu = 0;
    hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlock, 0);
    if (e != hipSuccess) return e;
    int64_t blocks = grid_blocks(per_cu, dev, n_items);
    if (max_blocks > 0) blocks = std::min(blocks, max_blocks);
    note_launch(form, blocks);
    void *args[] = {&wl};
    return hipModuleLaunchKernel(f, (unsigned)blocks, 1, 1, kBlock, 1, 1, 0, st, args, nullptr);
}

// Two-wave blocks (simulating wave + drawing wave), one work item at a time per block.
// The block count is at most 8 per CU, or max_blocks (a tuned launch), or
// SSA_DRAW_WAVE_BLOCKS (tests); blocks then run several generations each.
hipError_t launch_jit_pc(hipFunction_t f, WorkList &wl, int64_t n_items, int dev, hipStream_t st,
                         size_t dyn_lds = 0, int64_t max_blocks = 0) {
    int64_t cap = max_blocks > 0 ? max_blocks : (int64_t)8 * cu_count(dev);
    if (const char *e = std::getenv("SSA_DRAW_WAVE_BLOCKS")) cap = std::max<int64_t>(1, std::strtoll(e, nullptr, 10));
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(n_items, cap));
    note_launch(SSA_FORM_TWO_WAVE, blocks);
    void *args[] = {&wl};
    return hipModuleLaunchKernel(f, (unsigned)blocks, 1, 1, 2 * kWave, 1, 1, (unsigned)dyn_lds, st, args, nullptr);
}

// The control block of a single-network run: work counter at byte 0, status words
// (events, largest step count, flags) at byte 32, the grid description at byte 64.
constexpr size_t kCtlBytes = 64 + sizeof(GridInfo);
unsigned long long *ctl_flags(void *ctl) { return (unsigned long long *)((char *)ctl + 48); }
const unsigned long long *ctl_status(void *ctl) { return (const unsigned long long *)((char *)ctl + 32); }

// Describes a device grid and checks it (a grid that is not non-decreasing inside
// [0, t_end] refuses the run on the device; see grid_info_kernel).  ctl must be zeroed.
hipError_t launch_grid_info(const double *grid, int32_t G, double t_end, void *ctl, hipStream_t st) {
    hipLaunchKernelGGL(grid_info_kernel, dim3(1), dim3(256), 0, st, grid, G, t_end, (GridInfo *)((char *)ctl + 64),
                       (unsigned int *)ctl, ctl_flags(ctl));
    return hipGetLastError();
}

// Largest trajectory count a single-network call accepts: work items of 64 trajectories
// (one trajectory each in the 64-chunk order) stay below the refused-run sentinel.
int64_t max_traj(const ssa_model *m) { return m->order == SSA_SUM_BLOCK64 ? ((int64_t)1 << 30) : ((int64_t)1 << 36); }

// Host twin of grid_info_kernel for host grids.
GridInfo host_grid_info(const double *grid, int32_t G, double t_end) {
    GridInfo gi;
    std::memset(&gi, 0, sizeof gi);
    const double D = (double)(G - 1);
    const double Tc[2] = {t_end, grid[G - 1]};
    int ok[2] = {0, 0};
    for (int c = 0; c < 2; ++c) {
        ok[c] = (G >= 2 && Tc[c] > 0.0) ? 1 : 0;
        for (int32_t g = 0; g < G && ok[c]; ++g)
            if (grid[g] != (Tc[c] * (double)g) / D) ok[c] = 0;
    }
    gi.uniform = (ok[0] || ok[1]) ? 1 : 0;
    gi.T = ok[0] ? Tc[0] : Tc[1];
    gi.D = D;
    gi.lo = grid[0];
    const double span = grid[G - 1] - grid[0];
    gi.scale = (G > 1 && span > 0.0) ? (double)(G - 1) / span : 0.0;
    return gi;
}

hipError_t launch_fill(void *p, size_t words, unsigned long long v, hipStream_t st) {
    if (!words) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, st, (unsigned long long *)p, words, v);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    const size_t words = (bytes + 7) / 8;
    if (!words) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, (unsigned long long *)p, words);
    return hipGetLastError();
}

ssa_status collect_stats(unsigned long long *d_stats, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                         ssa_stats *stats) {
    unsigned long long h[3] = {0, 0, 0};
    HIP_TRY(hipMemcpyAsync(h, d_stats, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (stats) {
        stats->events = h[0];
        stats->max_steps = h[1];
        stats->flags = (uint32_t)h[2];
        float ms = 0.f;
        if (e0 && e1) (void)hipEventElapsedTime(&ms, e0, e1);
        stats->kernel_ms = ms;
        stats->form = g_launch.form;
        stats->blocks = g_launch.blocks;
        stats->ordered = g_launch.ordered;
    }
    if (h[2] & kFlagRefused)
        return fail(SSA_E_INVALID, "refused on the device: the grid is not non-decreasing inside [0, t_end], or a "
                                   "log rate is NaN or above 709 (outputs are NaN)");
    if (h[2] & kFlagTooManyEvents)
        return fail(SSA_E_UNSUPPORTED, "%llu events in one run: the exact integer sums hold at most 2^39 "
                                       "(outputs are NaN); split the trajectories over several calls",
                    (unsigned long long)h[0]);
    if (h[2] & kFlagOverflow) return fail(SSA_E_OVERFLOW, "a species count left the int32 range");
    if (h[2] & kFlagEventLimit) return fail(SSA_E_EVENT_LIMIT, "a trajectory reached max_events before t_end");
    return SSA_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    bool make() { return hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess; }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Device time of everything one call launches on stream st (fill kernels, scratch set-up,
// the simulation kernel, reductions, finalize), from events around the call: the tuners
// compare configurations by it, so that a configuration's extra launches count against it.
template <class Call>
ssa_status time_call(hipStream_t st, Call call, float &ms) {
    EventPair ev;
    if (!ev.make()) return fail(SSA_E_DEVICE, "hipEventCreate failed");
    HIP_TRY(hipEventRecord(ev.a, st));
    const ssa_status s = call();
    if (s) return s;
    HIP_TRY(hipEventRecord(ev.b, st));
    HIP_TRY(hipEventSynchronize(ev.b));
    HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
    return SSA_OK;
}

// One-trajectory-per-wave kernels (64-chunk sum order).
// Above kWaveMaxQ reactions per lane: one wave per block, chunk slots in LDS; the
// dependency-graph update unless SSA_WIDE_DEPG=0 (or no graph was built) asks for the full
// re-evaluation.  Both give the same bits.
template <int MODE, bool DEPG>
const void *wide_for(int32_t q) {
    if (q <= 16) return (const void *)wide_kernel<16, MODE, DEPG>;
    if (q <= 32) return (const void *)wide_kernel<32, MODE, DEPG>;
    if (q <= 64) return (const void *)wide_kernel<64, MODE, DEPG>;
    return nullptr;
}

bool wide_depg(const ssa_model *m) {
    const char *e = std::getenv("SSA_WIDE_DEPG");
    return m->d_dep_ptr != nullptr && !(e && e[0] == '0');
}

template <int MODE>
hipError_t launch_wide(const ssa_model *m, const WorkList &wl, int dev, hipStream_t st, Scratch &scr) {
    const bool depg = wide_depg(m);
    WorkList w = wl;
    if (depg && m->dep_nnz > 0 && w.net0.rate != m->d_rate) {
        // rates given for this run: gather them into the dependency entries' order
        void *dr = nullptr;
        hipError_t e = scr.alloc(&dr, sizeof(double) * (size_t)m->dep_nnz);
        if (e != hipSuccess) return e;
        const unsigned blocks = (unsigned)std::min<int64_t>((m->dep_nnz + 255) / 256, 65535);
        hipLaunchKernelGGL(dep_rate_kernel, dim3(blocks), dim3(256), 0, st, (const int2 *)m->d_dep, m->q,
                           w.net0.rate, m->dep_nnz, (double *)dr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        w.net0.dep_rate = (const double *)dr;
    }
    const void *kern = depg ? wide_for<MODE, true>(m->q) : wide_for<MODE, false>(m->q);
    if (!kern) return hipErrorInvalidValue;
    const int32_t Q = m->q <= 16 ? 16 : (m->q <= 32 ? 32 : 64);
    const size_t lds = (size_t)Q * kWave * ((depg ? 8 : 12) + (MODE == kBwd ? 16 : 0)) +
                       ((size_t)m->S + 1) * sizeof(int32_t);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kWave, lds);
    if (e != hipSuccess) return e;
    const int64_t n_traj = wl.range_end - wl.range_begin;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((int64_t)std::max(per_cu, 1) * cu_count(dev), n_traj));
    note_launch(SSA_FORM_WAVE, blocks);
    void *args[] = {&w};
    return hipLaunchKernel(kern, dim3((unsigned)blocks), dim3(kWave), args, lds, st);
}

template <int MODE>
hipError_t launch_wave(const ssa_model *m, const WorkList &wl, int dev, hipStream_t st, Scratch &scr) {
    if (m->q > kWaveMaxQ) return launch_wide<MODE>(m, wl, dev, st, scr);
    const void *kern = nullptr;
    if (m->q <= 1) kern = (const void *)wave_kernel<1, MODE>;
    else if (m->q <= 2) kern = (const void *)wave_kernel<2, MODE>;
    else if (m->q <= 4) kern = (const void *)wave_kernel<4, MODE>;
    else if (m->q <= 8) kern = (const void *)wave_kernel<8, MODE>;
    else return hipErrorInvalidValue;
    const size_t lds = (size_t)(kBlock / kWave) * (m->S + 1) * sizeof(int32_t);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, lds);
    if (e != hipSuccess) return e;
    const int64_t n_traj = wl.range_end - wl.range_begin;
    const int64_t blocks =
        std::max<int64_t>(1, std::min<int64_t>((int64_t)std::max(per_cu, 1) * cu_count(dev), (n_traj + 3) / 4));
    note_launch(SSA_FORM_WAVE, blocks);
    WorkList w = wl;
    void *args[] = {&w};
    return hipLaunchKernel(kern, dim3((unsigned)blocks), dim3(kBlock), args, lds, st);
}

// Finalize of one network: exact prefix over the grid and the moments.
// status: the run's status words (ctl_status), or NULL.
hipError_t launch_finalize(const unsigned long long *D, const unsigned long long *Dhi, int32_t G, int32_t S,
                           const int32_t *d_x0, int64_t n_traj, double *mean, double *var,
                           const unsigned long long *status, hipStream_t st) {
    hipLaunchKernelGGL(moment_final_kernel, dim3(S), dim3(1024), 0, st, D, Dhi, G, S, d_x0, n_traj, mean, var,
                       (int64_t *)nullptr, status);
    return hipGetLastError();
}

// Single-network launch of one simulation mode through the kernel specialised to the
// network, or the generic one (which reads rates in zero-padded slots: a caller's rates
// array is copied into a padded buffer first).
// tuned_form / tuned_blocks: a tuned launch of the specialised backward (0: by launch size).
ssa_status launch_single(int mode, const ssa_model *m, WorkList &wl, int64_t n_items, int dev, hipStream_t st,
                         const double *user_rates, Scratch &scr, bool quad = false, int32_t tuned_form = 0,
                         int32_t tuned_blocks = 0) {
    (void)n_items;
    if (m->order == SSA_SUM_BLOCK64) {
        HIP_TRY(mode == kRec   ? launch_wave<kRec>(m, wl, dev, st, scr)
                : mode == kEvt ? launch_wave<kEvt>(m, wl, dev, st, scr)
                               : launch_wave<kBwd>(m, wl, dev, st, scr));
        return SSA_OK;
    }
    if (jit_eligible(m)) {
        std::shared_ptr<JitKernels> k;
        const bool lat = latency_bound(n_items, dev);
        ssa_status s = get_jit(m, dev, k, lat);
        if (s) return s;
        // backward: two-wave blocks for launches of up to two work items per CU, else
        // generations (measured faster than refilling lanes at every size: 32.6 against
        // 37.2 ms at 10^6 trajectories on a 10^4-point grid, where trajectories differ little
        // in length and the simpler loop wins); the event log: two-wave blocks or refill; the
        // record always refills
        uint32_t form = SSA_FORM_REFILL;
        if (mode == kBwd) form = pc_launch(n_items, dev) ? SSA_FORM_TWO_WAVE : SSA_FORM_GENERATIONS;
        if (mode == kEvt && pc_launch(n_items, dev)) form = SSA_FORM_TWO_WAVE;
        int64_t max_blocks = 0;
        if (mode == kBwd && tuned_form >= SSA_FORM_TWO_WAVE && tuned_form <= SSA_FORM_REFILL) {
            form = (uint32_t)tuned_form;
            max_blocks = tuned_blocks;
        }
        const uint32_t forced = forced_form();
        if (forced != SSA_FORM_NONE && mode != kRec && !(mode == kEvt && forced == SSA_FORM_GENERATIONS))
            form = forced;
        if (form == SSA_FORM_TWO_WAVE) {
            HIP_TRY(launch_jit_pc(mode == kEvt ? k->evt_pc : (quad ? k->bwd_var_pc : k->bwd_pc), wl, n_items, dev,
                                  st, 0, max_blocks));
            return SSA_OK;
        }
        const bool gen = form == SSA_FORM_GENERATIONS;
        hipFunction_t f = mode == kRec   ? k->rec
                          : mode == kEvt ? k->evt
                          : quad         ? (gen ? k->bwd_var_gen : k->bwd_var)
                                         : (gen ? k->bwd_gen : k->bwd);
        HIP_TRY(launch_jit(f, wl, n_items, dev, st, form, max_blocks));
        return SSA_OK;
    }
    const int mm = generic_mm(m->M);
    if (mm == 0) return fail(SSA_E_UNSUPPORTED, "record / backward support at most %d reactions", kJitMaxReactions);
    if (m->max_changes > kChg)
        return fail(SSA_E_UNSUPPORTED, "the generic kernel handles at most %d changed species per reaction", kChg);
    if (user_rates) {
        void *pr = nullptr;
        HIP_TRY(scr.alloc(&pr, sizeof(double) * m->m_pad));
        HIP_TRY(launch_zero(pr, sizeof(double) * m->m_pad, st));
        HIP_TRY(hipMemcpyAsync(pr, user_rates, sizeof(double) * m->M, hipMemcpyDeviceToDevice, st));
        wl.net0.rate = (const double *)pr;
    }
    wl.s_rows = m->S;
    wl.m_rows = m->M;
    hipError_t e = mode == kRec   ? launch_generic<kRec, false>(mm, wl, n_items, dev, st)
                   : mode == kEvt ? launch_generic<kEvt, false>(mm, wl, n_items, dev, st)
                   : quad         ? launch_generic<kBwd, false, true>(mm, wl, n_items, dev, st)
                                  : launch_generic<kBwd, false>(mm, wl, n_items, dev, st);
    HIP_TRY(e);
    return SSA_OK;
}

// ---------------------------------------------------------------------------------------
// Autotuning of the launches.  A tuned configuration (forward: window bytes, flush target;
// forward and backward: launch form and block count) is kept per (direction, device
// architecture, kernel kind, S, M, network source hash, G and N rounded up to powers of
// two), in memory and, when SSA_TUNE_FILE names a file, in that JSON file (read at the
// first lookup, rewritten after each tuning).  Every configuration gives the same bits, so
// tuning only changes speed.
// ---------------------------------------------------------------------------------------
struct FwdTune {
    int32_t win_bytes = 0;   // 0: default
    int32_t slab = -1;       // -1: default
    int32_t form = 0;        // ssa_launch_form of the specialised kernels; 0: by launch size
    int32_t blocks = 0;      // grid size (persistent forms: at most the occupancy limit); 0: default
    float ms = 0.f;
};

std::mutex g_tune_mu;
std::map<std::string, FwdTune> g_tune;
bool g_tune_loaded = false;

uint64_t next_pow2(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Forward keys start with the architecture; backward keys with "bwd|".
std::string tune_key(const ssa_model *m, int64_t n_traj, int32_t G, int dev, bool backward = false) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : m->jit_src) h = (h ^ c) * 1099511628211ull;
    char buf[256];
    snprintf(buf, sizeof buf, "%s%s|%s|S%d|M%d|G%llu|N%llu|h%016llx", backward ? "bwd|" : "", device_arch(dev).c_str(),
             m->order == SSA_SUM_BLOCK64 ? "wave" : (jit_eligible(m) ? "jit" : "table"), m->S, m->M,
             (unsigned long long)next_pow2((uint64_t)G), (unsigned long long)next_pow2((uint64_t)n_traj),
             (unsigned long long)h);
    return buf;
}

// The cache file holds one entry per line inside the "entries" object:
//   "<key>": {"win_bytes": <int>, "slab": <int>, "form": <int>, "blocks": <int>, "ms": <float>}
void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("SSA_TUNE_FILE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        char key[512];
        int wb = 0, sl = -1, fo = 0, bl = 0;
        float ms = 0.f;
        if (std::sscanf(line, " \"%511[^\"]\": {\"win_bytes\": %d, \"slab\": %d, \"form\": %d, \"blocks\": %d, \"ms\": %f}",
                        key, &wb, &sl, &fo, &bl, &ms) == 6) {
            FwdTune t;
            t.win_bytes = wb;
            t.slab = sl;
            t.form = fo;
            t.blocks = bl;
            t.ms = ms;
            g_tune[key] = t;
        }
    }
    std::fclose(f);
}

void tune_save_locked() {
    const char *path = std::getenv("SSA_TUNE_FILE");
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n  \"format\": \"ssa launch tuning, one entry per line\",\n  \"entries\": {\n");
    size_t i = 0;
    for (const auto &kv : g_tune) {
        std::fprintf(f, "    \"%s\": {\"win_bytes\": %d, \"slab\": %d, \"form\": %d, \"blocks\": %d, \"ms\": %.4f}%s\n",
                     kv.first.c_str(), kv.second.win_bytes, kv.second.slab, kv.second.form, kv.second.blocks,
                     kv.second.ms, ++i < g_tune.size() ? "," : "");
    }
    std::fprintf(f, "  }\n}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

FwdTune tune_lookup(const ssa_model *m, int64_t n_traj, int32_t G, int dev, bool backward = false) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(tune_key(m, n_traj, G, dev, backward));
    return it == g_tune.end() ? FwdTune() : it->second;
}

void tune_store(const ssa_model *m, int64_t n_traj, int32_t G, int dev, bool backward, const FwdTune &t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[tune_key(m, n_traj, G, dev, backward)] = t;
    tune_save_locked();
}

// Forward launch of one network.  D receives the [G][S][2] difference sums, by atomic
// flushes of the windows into D directly or through wave-private slabs and a reduction
// (see want_slabs).  Dhi ([G][S], high parts) must be zero on entry.
// may_compile false: the specialised kernels only if this device has them compiled already
// (else the table-driven kernel, with the same results; networks with rate laws then fail).
// epoch: one epoch of a resumable run (the specialised kernels in generations or two-wave
// blocks, which save and resume trajectory states; D keeps the earlier epochs' sums).
ssa_status order_by_key(const uint32_t *key, int64_t n, Scratch &scr, hipStream_t st, const uint32_t **out);

// order_keys: event counts a previous forward recorded for these positions, or NULL; a
// specialised forward in generations then takes its trajectories longest first
ssa_status launch_forward(const ssa_model *m, WorkList &wl, int64_t n_items, int dev, hipStream_t st,
                          const double *user_rates, Scratch &scr, unsigned long long *D, float *kernel_ms,
                          const FwdTune &tune, bool may_compile = true, bool epoch = false,
                          const uint32_t *order_keys = nullptr) {
    const int32_t G = wl.net0.G, S = m->S;
    if (epoch && (m->order != SSA_SUM_SEQ || !jit_eligible(m)))
        return fail(SSA_E_UNSUPPORTED, "runs in epochs need the specialised kernels (sequential order, at most %d "
                                       "reactions and %d species)", kJitMaxReactions, kJitMaxSpecies);
    const bool use_jit = jit_eligible(m) && (may_compile || jit_cached(m, dev, latency_bound(n_items, dev)));
    if (m->has_laws && !use_jit)
        return fail(SSA_E_UNSUPPORTED, "a network with rate laws needs its specialised kernels compiled on this "
                                       "device first (one ssa_run_device call)");
    if (m->order == SSA_SUM_BLOCK64) {
        HIP_TRY(launch_zero(D, (size_t)G * S * 2 * sizeof(unsigned long long), st));
        EventPair ev;
        if (kernel_ms && ev.make()) HIP_TRY(hipEventRecord(ev.a, st));
        HIP_TRY(launch_wave<kFwd>(m, wl, dev, st, scr));
        if (kernel_ms && ev.b) {
            HIP_TRY(hipEventRecord(ev.b, st));
            HIP_TRY(hipEventSynchronize(ev.b));
            (void)hipEventElapsedTime(kernel_ms, ev.a, ev.b);
        }
        return SSA_OK;
    }
    FwdKernel k;
    wl.win_bins = window_bins(S, G, !use_jit, tune.win_bytes);
    wl.win_words = wl.win_bins * (use_jit ? win_stride(S * 2) : S * 2);
    // the specialised kernels run generations with one window per wave, the table-driven
    // kernel cohorts with kCohorts windows
    const size_t win_bytes = (size_t)(kBlock / kWave) * wl.win_words * sizeof(long long);
    if (use_jit) {
        std::shared_ptr<JitKernels> jk;
        ssa_status s = get_jit(m, dev, jk, latency_bound(n_items, dev));
        if (s) return s;
        k.jit = true;
        const bool hist = wl.net0.Hd != nullptr;
        k.f_slab = hist ? jk->fwd_slab_hist : jk->fwd;
        k.f_atomic = epoch ? (hist ? jk->fwd_hist_epoch : jk->fwd_epoch) : hist ? jk->fwd_hist : jk->fwd_atomic;
        k.lds = win_bytes;
        // the launch form: SSA_LAUNCH_FORM, else a tuned one, else by launch size
        uint32_t want = forced_form();
        if (want == SSA_FORM_NONE && (tune.form == SSA_FORM_TWO_WAVE || tune.form == SSA_FORM_GENERATIONS))
            want = (uint32_t)tune.form;
        const bool two_wave = want == SSA_FORM_TWO_WAVE || (want == SSA_FORM_NONE && pc_launch(n_items, dev));
        if (two_wave) {
            // one simulating wave per block: one window, flushed atomically into D (which a
            // run in epochs keeps from epoch to epoch)
            if (!epoch) HIP_TRY(launch_zero(D, (size_t)G * S * 2 * sizeof(unsigned long long), st));
            hipFunction_t f = epoch ? (hist ? jk->fwd_hist_epoch_pc : jk->fwd_epoch_pc)
                                    : (hist ? jk->fwd_hist_pc : jk->fwd_pc);
            EventPair ev;
            if (kernel_ms && ev.make()) HIP_TRY(hipEventRecord(ev.a, st));
            HIP_TRY(launch_jit_pc(f, wl, n_items, dev, st, (size_t)wl.win_words * sizeof(long long), tune.blocks));
            if (kernel_ms && ev.b) {
                HIP_TRY(hipEventRecord(ev.b, st));
                HIP_TRY(hipEventSynchronize(ev.b));
                (void)hipEventElapsedTime(kernel_ms, ev.a, ev.b);
            }
            return SSA_OK;
        }
    } else {
        if (m->max_changes > kChg)
            return fail(SSA_E_UNSUPPORTED, "the generic kernel handles at most %d changed species per reaction", kChg);
        if (!pick_generic_fwd<false>(generic_mm(m->M), k)) return fail(SSA_E_UNSUPPORTED, "no kernel");
        if (user_rates) {
            void *pr = nullptr;
            HIP_TRY(scr.alloc(&pr, sizeof(double) * m->m_pad));
            HIP_TRY(launch_zero(pr, sizeof(double) * m->m_pad, st));
            HIP_TRY(hipMemcpyAsync(pr, user_rates, sizeof(double) * m->M, hipMemcpyDeviceToDevice, st));
            wl.net0.rate = (const double *)pr;
        }
        wl.s_rows = S;
        wl.m_rows = m->M;
        k.lds = generic_int_words(wl.s_rows, wl.m_rows) * sizeof(int32_t) + kCohorts * win_bytes;
        if (k.lds > lds_max(dev))
            return fail(SSA_E_UNSUPPORTED,
                        "the sequential-order kernel needs %zu bytes of LDS for %d species and %d reactions "
                        "(limit %zu); the 64-chunk order runs such networks",
                        k.lds, S, m->M, lds_max(dev));
    }
    if (k.jit && order_keys && !epoch && wl.range_begin == 0) {
        const ssa_status s = order_by_key(order_keys, wl.range_end, scr, st, &wl.perm);
        if (s) return s;
    }
    const size_t cell_words = (size_t)G * S * 2;
    int64_t blocks = 0;
    HIP_TRY(fwd_blocks(k, true, dev, n_items, blocks));
    const size_t slab_bytes = (size_t)blocks * (kBlock / kWave) * cell_words * sizeof(unsigned long long);
    const bool slab = !epoch && want_slabs(slab_bytes, tune.slab);
    if (slab) {
        void *sl = nullptr;
        HIP_TRY(scr.alloc(&sl, slab_bytes));
        HIP_TRY(launch_zero(sl, slab_bytes, st));
        wl.slabs = (unsigned long long *)sl;
    } else {
        HIP_TRY(fwd_blocks(k, false, dev, n_items, blocks));
        if (tune.blocks > 0) blocks = std::min<int64_t>(blocks, tune.blocks);
        if (!epoch) HIP_TRY(launch_zero(D, cell_words * sizeof(unsigned long long), st));
    }
    // at most one work item per CU: one wave per block, so that each work item's wave has a
    // CU of its own instead of four sharing one (the HIV network's 32 items in epochs: 6-8 %
    // faster); the window's LDS is then one wave's
    const bool lone = k.jit && !slab && n_items <= (int64_t)cu_count(dev);
    if (lone) blocks = n_items;
    EventPair ev;
    if (kernel_ms && ev.make()) HIP_TRY(hipEventRecord(ev.a, st));
    HIP_TRY(fwd_launch(k, slab, blocks, wl, st, lone));
    if (kernel_ms && ev.b) HIP_TRY(hipEventRecord(ev.b, st));
    if (slab) {
        const int64_t words = (int64_t)cell_words;
        hipLaunchKernelGGL(slab_reduce_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st,
                           (const unsigned long long *)wl.slabs, blocks * (kBlock / kWave), words, D);
        HIP_TRY(hipGetLastError());
    }
    if (kernel_ms && ev.b) {
        HIP_TRY(hipEventSynchronize(ev.b));
        (void)hipEventElapsedTime(kernel_ms, ev.a, ev.b);
    }
    return SSA_OK;
}

}  // namespace

// The ssa_* definitions below take C linkage from their declarations in ssa.h; every
// other function of this file has internal linkage (anonymous namespaces).

const char *ssa_last_error(void) { return g_err.c_str(); }

ssa_status ssa_model_create(int32_t S, int32_t M, const int32_t *reac, const int32_t *prod, const double *rates,
                            const int32_t *x0, int32_t sum_order, ssa_model **out) {
    return ssa_model_create_laws(S, M, reac, prod, rates, x0, sum_order, nullptr, out);
}

ssa_status ssa_model_create_laws(int32_t S, int32_t M, const int32_t *reac, const int32_t *prod,
                                 const double *rates, const int32_t *x0, int32_t sum_order, const ssa_rate_law *laws,
                                 ssa_model **out) {
    if (!out) return fail(SSA_E_INVALID, "out is NULL");
    *out = nullptr;
    if (sum_order != SSA_SUM_SEQ && sum_order != SSA_SUM_BLOCK64) return fail(SSA_E_INVALID, "unknown sum order");
    if (S <= 0 || M <= 0 || S > kMaxSpecies || M > kMaxReactions)
        return fail(SSA_E_INVALID, "need 1 <= S <= %d and 1 <= M <= %d", kMaxSpecies, kMaxReactions);
    if (!reac || !prod || !rates || !x0) return fail(SSA_E_INVALID, "NULL model array");
    std::unique_ptr<ssa_model> m(new (std::nothrow) ssa_model);
    if (!m) return fail(SSA_E_NOMEM, "host allocation failed");
    m->S = S;
    m->M = M;
    m->order = sum_order;
    m->q = (M + kWave - 1) / kWave;
    if (laws) {
        for (int32_t j = 0; j < M; ++j) {
            const ssa_rate_law &L = laws[j];
            if (L.species < 0) continue;
            if (L.species >= S || !std::isfinite(L.slope) || !(L.lo >= 0.0) || !(L.hi >= L.lo) || std::isnan(L.hi))
                return fail(SSA_E_INVALID, "rate law of reaction %d: need 0 <= species < S, finite slope, "
                                           "0 <= lo <= hi", j);
            m->has_laws = true;
        }
        if (m->has_laws) {
            if (sum_order != SSA_SUM_SEQ || M > kJitMaxReactions || S > kJitMaxSpecies)
                return fail(SSA_E_UNSUPPORTED, "rate laws need the sequential order, M <= %d and S <= %d",
                            kJitMaxReactions, kJitMaxSpecies);
            m->laws.assign(laws, laws + M);
        }
    }
    m->reac.assign(reac, reac + (size_t)M * S);
    m->prod.assign(prod, prod + (size_t)M * S);
    m->rate.assign(rates, rates + M);
    m->x0.assign(x0, x0 + S);
    for (int32_t s = 0; s < S; ++s)
        if (x0[s] < 0) return fail(SSA_E_INVALID, "x0[%d] < 0", s);
    m->m_pad = ((M + kPadReactions - 1) / kPadReactions) * kPadReactions;
    std::vector<uint32_t> rx(m->m_pad, 0u);          // padding: rows 0, 0 -> h = 1, rate 0
    std::vector<double> rpad(m->m_pad, 0.0);
    std::vector<int32_t> chg((size_t)M * kChg, 0);
    for (int32_t j = 0; j < M; ++j) {
        if (!(rates[j] >= 0.0) || !std::isfinite(rates[j]))
            return fail(SSA_E_INVALID, "rate[%d] must be finite and >= 0", j);
        rpad[j] = rates[j];
        int32_t order = 0, sa = -1, sb = -1;
        for (int32_t s = 0; s < S; ++s) {
            const int32_t r = reac[(size_t)j * S + s], p = prod[(size_t)j * S + s];
            if (r < 0 || p < 0 || p > kMaxProduct)
                return fail(SSA_E_INVALID, "reaction %d: coefficients must be in [0, 2^19 - 4]", j);
            order += r;
            if (order > 2) return fail(SSA_E_INVALID, "reaction %d: order above 2", j);
            for (int32_t q = 0; q < r; ++q) (sa < 0 ? sa : sb) = s;
        }
        uint32_t ra = 0, rb = 0, d = 0;    // LDS rows: 0 = all ones, species s = row s + 1
        if (order >= 1) ra = (uint32_t)sa + 1;
        if (order == 2) {
            rb = (uint32_t)sb + 1;
            d = (sa == sb) ? 1u : 0u;
        }
        rx[j] = ra | (rb << 12) | (d << 24);
        int32_t nchg = 0;
        for (int32_t s = 0; s < S; ++s) {
            const int32_t dl = prod[(size_t)j * S + s] - reac[(size_t)j * S + s];
            if (!dl) continue;
            if (nchg < kChg) chg[(size_t)j * kChg + nchg] = (s + 1) | (dl << kRowBits);
            ++nchg;
        }
        m->max_changes = std::max(m->max_changes, nchg);
    }
    if (m->max_changes > kChg && (M > kJitMaxReactions || S > kJitMaxSpecies || sum_order == SSA_SUM_BLOCK64))
        return fail(SSA_E_UNSUPPORTED, "a reaction changes more than %d species in a network run by a table-driven kernel",
                    kChg);
    m->jit_src = generate_net_source(m.get());
    // dependency lists for the LDS-resident 64-chunk kernel: for each reaction, the
    // reactions (as LDS slot and reactant code) with a reactant among its changed species
    std::vector<int32_t> dep_ptr;
    std::vector<int2> dep;
    if (sum_order == SSA_SUM_BLOCK64 && m->q > kWaveMaxQ) {
        std::vector<std::vector<int32_t>> readers(S);
        for (int32_t k = 0; k < M; ++k) {
            const uint32_t code = rx[k];
            const int32_t ra = (int32_t)(code & 0xfffu), rb = (int32_t)((code >> 12) & 0xfffu);
            if (ra) readers[ra - 1].push_back(k);
            if (rb && rb != ra) readers[rb - 1].push_back(k);
        }
        dep_ptr.assign((size_t)M + 1, 0);
        std::vector<int32_t> mark(M, -1);
        bool too_big = false;
        for (int32_t j = 0; j < M && !too_big; ++j) {
            std::vector<int32_t> ks;
            for (int32_t s = 0; s < S; ++s) {
                if (prod[(size_t)j * S + s] == reac[(size_t)j * S + s]) continue;
                for (int32_t k : readers[s])
                    if (mark[k] != j) {
                        mark[k] = j;
                        ks.push_back(k);
                    }
            }
            std::sort(ks.begin(), ks.end());
            for (int32_t k : ks) {
                const int32_t slot = (k % m->q) * kWave + k / m->q;
                dep.push_back(make_int2(slot, (int)rx[k]));
            }
            dep_ptr[j + 1] = (int32_t)dep.size();
            too_big = (int64_t)dep.size() > kMaxDepEntries;
        }
        if (too_big) {
            dep.clear();
            dep_ptr.clear();
        }
    }
    hipError_t e = hipGetDevice(&m->device);
    if (e == hipSuccess) e = hipMalloc(&m->d_rx, sizeof(uint32_t) * m->m_pad);
    if (e == hipSuccess) e = hipMalloc(&m->d_rate, sizeof(double) * m->m_pad);
    if (e == hipSuccess) e = hipMalloc(&m->d_chg, sizeof(int32_t) * M * kChg);
    if (e == hipSuccess) e = hipMalloc(&m->d_x0, sizeof(int32_t) * S);
    if (e == hipSuccess) e = hipMemcpy(m->d_rx, rx.data(), sizeof(uint32_t) * m->m_pad, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_rate, rpad.data(), sizeof(double) * m->m_pad, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_chg, chg.data(), sizeof(int32_t) * M * kChg, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_x0, m->x0.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice);
    if (e == hipSuccess && !dep_ptr.empty()) {
        m->dep_nnz = (int64_t)dep.size();
        std::vector<double> dep_rate(dep.size());
        for (size_t p = 0; p < dep.size(); ++p)
            dep_rate[p] = rates[(dep[p].x & (kWave - 1)) * m->q + (dep[p].x >> 6)];
        const size_t nd = std::max<size_t>(dep.size(), 1);
        e = hipMalloc(&m->d_dep_ptr, sizeof(int32_t) * dep_ptr.size());
        if (e == hipSuccess) e = hipMalloc(&m->d_dep, sizeof(int2) * nd);
        if (e == hipSuccess) e = hipMalloc(&m->d_dep_rate, sizeof(double) * nd);
        if (e == hipSuccess)
            e = hipMemcpy(m->d_dep_ptr, dep_ptr.data(), sizeof(int32_t) * dep_ptr.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !dep.empty())
            e = hipMemcpy(m->d_dep, dep.data(), sizeof(int2) * dep.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !dep.empty())
            e = hipMemcpy(m->d_dep_rate, dep_rate.data(), sizeof(double) * dep.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        ssa_model_destroy(m.release());
        return fail(e == hipErrorOutOfMemory ? SSA_E_NOMEM : SSA_E_DEVICE, "model upload: %s", hipGetErrorString(e));
    }
    *out = m.release();
    return SSA_OK;
}

void ssa_model_destroy(ssa_model *m) {
    if (!m) return;
    if (m->d_rx) (void)hipFree(m->d_rx);
    if (m->d_rate) (void)hipFree(m->d_rate);
    if (m->d_chg) (void)hipFree(m->d_chg);
    if (m->d_x0) (void)hipFree(m->d_x0);
    if (m->d_dep) (void)hipFree(m->d_dep);
    if (m->d_dep_rate) (void)hipFree(m->d_dep_rate);
    if (m->d_dep_ptr) (void)hipFree(m->d_dep_ptr);
    for (void *p : m->cap_mem) (void)hipFree(p);
    for (void *p : m->hint_old) (void)hipFree(p);
    if (m->hint_len) (void)hipFree(m->hint_len);
    delete m;
}

namespace {

// ---------------------------------------------------------------------------------------
// Length hints.  A forward in generations records the event count of every trajectory
// into a buffer of the model, with the identity of its run; a backward of the same run
// (same trajectory count, horizon, seed, event cap, grid and rate arrays) then takes its
// trajectories longest first (len_max_kernel and after), so that the trajectories of one
// generation end close together.  The record is only a hint: a backward whose arrays
// changed contents since, or that overlaps a forward, still gets its exact results.
// ---------------------------------------------------------------------------------------
constexpr int64_t kMaxHintTraj = (int64_t)1 << 27;

struct RunId {
    int64_t n;
    double t_end;
    uint64_t seed, max_events;
    const double *grid, *rates, *log_rates;
    int32_t G;
    int dev;
};

// The buffer the forward of run id records into, or NULL (no record for this run).  Under
// graph capture the buffer is used only if it is large enough already, and the recorded
// identity is left as it is.
uint32_t *hint_begin(const ssa_model *m, const RunId &id, bool capturing) {
    if (m->order != SSA_SUM_SEQ || !jit_eligible(m) || id.n > kMaxHintTraj) return nullptr;
    std::lock_guard<std::mutex> lk(m->hint_mu);
    if (capturing) return (m->hint_cap >= id.n && m->hint_dev == id.dev) ? m->hint_len : nullptr;
    m->hint_valid = false;
    if (m->hint_cap < id.n || m->hint_dev != id.dev) {
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(uint32_t) * (size_t)id.n) != hipSuccess) return nullptr;
        if (m->hint_len) m->hint_old.push_back(m->hint_len);
        m->hint_len = (uint32_t *)p;
        m->hint_cap = id.n;
        m->hint_dev = id.dev;
    }
    return m->hint_len;
}

void hint_end(const ssa_model *m, const RunId &id, bool recorded) {
    std::lock_guard<std::mutex> lk(m->hint_mu);
    m->hint_valid = recorded;
    m->hint_n = id.n;
    m->hint_t_end = id.t_end;
    m->hint_seed = id.seed;
    m->hint_max_events = id.max_events;
    m->hint_grid = id.grid;
    m->hint_rates = id.rates;
    m->hint_log_rates = id.log_rates;
    m->hint_G = id.G;
}

hipError_t launch_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *sums, hipStream_t st);

// Positions 0..n-1 ordered by key, largest first in buckets of similar keys (len_max_kernel,
// len_count_kernel, the prefix sum of the counts, len_scatter_kernel).  Scratch: a copy of
// the keys, the per-tile counts and their prefix sums, the order.
ssa_status order_by_key(const uint32_t *key, int64_t n, Scratch &scr, hipStream_t st, const uint32_t **out) {
    const int64_t tile = std::max<int64_t>(4096, (n + 255) / 256);
    const int32_t n_tiles = (int32_t)((n + tile - 1) / tile);
    const int64_t n_cnt = (int64_t)kLenBuckets * n_tiles;
    void *snap = nullptr, *perm = nullptr, *cnt = nullptr, *incl = nullptr, *sums = nullptr, *mxw = nullptr;
    HIP_TRY(scr.alloc(&snap, sizeof(uint32_t) * (size_t)n));
    HIP_TRY(scr.alloc(&perm, sizeof(uint32_t) * (size_t)n));
    HIP_TRY(scr.alloc(&cnt, sizeof(int32_t) * (size_t)n_cnt));
    HIP_TRY(scr.alloc(&incl, sizeof(int32_t) * (size_t)n_cnt));
    HIP_TRY(scr.alloc(&sums, sizeof(int32_t) * (size_t)(n_cnt / kScanTile + 2)));
    HIP_TRY(scr.alloc(&mxw, 256));
    unsigned int *mx = (unsigned int *)mxw;
    HIP_TRY(launch_zero(mx, 8, st));
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(len_max_kernel, dim3(blocks), dim3(256), 0, st, key, n, (uint32_t *)snap, mx);
    hipLaunchKernelGGL(len_count_kernel, dim3((unsigned)n_tiles), dim3(256), 0, st, (const uint32_t *)snap, n, tile,
                       (const unsigned int *)mx, (int32_t *)cnt, n_tiles);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_scan((const int32_t *)cnt, (int32_t *)incl, n_cnt, (int32_t *)sums, st));
    hipLaunchKernelGGL(len_scatter_kernel, dim3((unsigned)n_tiles), dim3(256), 0, st, (const uint32_t *)snap, n, tile,
                       (const unsigned int *)mx, (const int32_t *)cnt, (const int32_t *)incl, n_tiles,
                       (uint32_t *)perm);
    HIP_TRY(hipGetLastError());
    *out = (const uint32_t *)perm;
    return SSA_OK;
}

// The order of the trajectories of a backward of run id (NULL: positions in order).
// Scratch: a copy of the counts, the bucket counters and the order.
ssa_status hint_order(const ssa_model *m, const RunId &id, Scratch &scr, hipStream_t st, const uint32_t **out) {
    *out = nullptr;
    const uint32_t *len = nullptr;
    {
        std::lock_guard<std::mutex> lk(m->hint_mu);
        const bool same = m->hint_valid && m->hint_n == id.n && m->hint_t_end == id.t_end && m->hint_seed == id.seed &&
                          m->hint_max_events == id.max_events && m->hint_grid == id.grid &&
                          m->hint_rates == id.rates && m->hint_log_rates == id.log_rates && m->hint_G == id.G &&
                          m->hint_dev == id.dev;
        if (!same) return SSA_OK;
        len = m->hint_len;
    }
    return order_by_key(len, id.n, scr, st, out);
}

// The event counts a forward of run id may take its trajectories in order of, or NULL: those
// of the last recorded forward with the same trajectory count, horizon, seed and event cap
// (the rates may have changed since: the counts are then a close hint, never a result).
// SSA_FWD_ORDER=0 turns the forward's order off (timing a run's first forward).
const uint32_t *fwd_hint(const ssa_model *m, const RunId &id) {
    if (id.n > kMaxHintTraj) return nullptr;
    if (const char *e = std::getenv("SSA_FWD_ORDER"))
        if (e[0] == '0' && e[1] == 0) return nullptr;
    std::lock_guard<std::mutex> lk(m->hint_mu);
    const bool same = m->hint_valid && m->hint_n == id.n && m->hint_t_end == id.t_end && m->hint_seed == id.seed &&
                      m->hint_max_events == id.max_events && m->hint_dev == id.dev;
    return same ? m->hint_len : nullptr;
}

// Launch form of the specialised backward: two-wave blocks up to two work items per CU,
// else generations; a tuned form, then SSA_LAUNCH_FORM, replace it (as launch_single does).
uint32_t bwd_form(int64_t n_items, int dev, int32_t tuned_form) {
    uint32_t form = pc_launch(n_items, dev) ? SSA_FORM_TWO_WAVE : SSA_FORM_GENERATIONS;
    if (tuned_form >= SSA_FORM_TWO_WAVE && tuned_form <= SSA_FORM_REFILL) form = (uint32_t)tuned_form;
    const uint32_t forced = forced_form();
    if (forced != SSA_FORM_NONE) form = forced;
    return form;
}

// Rate constants of a run: the caller's rates, or c = e^theta of the caller's log rates
// formed on the device (zero-padded to the model's table width; an invalid theta refuses the
// run), or NULL for the model's own.  ctl must be zeroed.
ssa_status run_rates(const ssa_model *m, const double *rates, const double *log_rates, void *ctl,
                     Scratch &scr, hipStream_t st, const double **out) {
    *out = rates;
    if (!log_rates) return SSA_OK;
    void *p = nullptr;
    HIP_TRY(scr.alloc(&p, sizeof(double) * (size_t)m->m_pad));
    hipLaunchKernelGGL(rates_from_log_kernel, dim3((unsigned)((m->m_pad + 255) / 256)), dim3(256), 0, st, log_rates,
                       m->M, m->m_pad, (double *)p, (unsigned int *)ctl, ctl_flags(ctl));
    HIP_TRY(hipGetLastError());
    *out = (const double *)p;
    return SSA_OK;
}

// The forward pass with a given launch configuration (tune == nullptr: the cached tuned
// one, else the defaults).
// fixed != nullptr: every piece of scratch comes from that area and the call allocates
// nothing, compiles nothing (see launch_forward), flushes the windows by atomics and does
// not time its kernel.
ssa_status run_device_impl(const ssa_model *m, const double *rates, const double *log_rates, int64_t n_traj,
                           double t_end, const double *grid, int32_t G, uint64_t seed, uint64_t max_events,
                           double *mean, double *var, const ssa_hist_spec *hist, uint32_t *d_hist, void *stream,
                           ssa_stats *stats, const FwdTune *tune, Scratch *fixed = nullptr) {
    if (!m) return fail(SSA_E_INVALID, "model is NULL");
    if (n_traj <= 0) return fail(SSA_E_INVALID, "n_traj must be > 0");
    if (G <= 0 || !grid || !mean || !var) return fail(SSA_E_INVALID, "grid / mean / var missing");
    if (!(t_end >= 0.0) || !std::isfinite(t_end)) return fail(SSA_E_INVALID, "t_end must be finite and >= 0");
    if ((hist == nullptr) != (d_hist == nullptr)) return fail(SSA_E_INVALID, "hist spec and buffer go together");
    if (hist && (hist->species < 0 || hist->species >= m->S || hist->width <= 0 || hist->nbins <= 0 ||
                 hist->nbins > 4096))
        return fail(SSA_E_INVALID, "bad histogram spec");
    if (rates && log_rates) return fail(SSA_E_INVALID, "rates and log_rates are alternatives");
    if (n_traj > max_traj(m)) return fail(SSA_E_INVALID, "n_traj above %lld", (long long)max_traj(m));
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const int64_t n_items = (n_traj + kChunk - 1) / kChunk;
    bool cap = false;
    ssa_status s = capture_check(m, st, dev, stats, m->order == SSA_SUM_SEQ && jit_eligible(m),
                                 latency_bound(n_items, dev), &cap);
    if (s) return s;
    if (!fixed && !cap) keep_pool(dev);
    StreamScratch pooled(st);
    CaptureScratch kept(m);
    Scratch &scr = fixed ? *fixed : cap ? (Scratch &)kept : (Scratch &)pooled;

    const RunId rid{n_traj, t_end, seed, max_events, grid, rates, log_rates, G, dev};
    const size_t cells = (size_t)G * m->S;
    const size_t H_bytes = hist ? sizeof(int32_t) * (size_t)G * hist->nbins : 0;
    void *D = nullptr, *Dhi = nullptr, *Hd = nullptr, *ctl = nullptr;
    HIP_TRY(scr.alloc(&D, sizeof(unsigned long long) * 2 * cells));
    HIP_TRY(scr.alloc(&Dhi, sizeof(unsigned long long) * cells));
    HIP_TRY(scr.alloc(&ctl, kCtlBytes));
    if (hist) HIP_TRY(scr.alloc(&Hd, H_bytes));
    HIP_TRY(launch_zero(Dhi, sizeof(unsigned long long) * cells, st));
    HIP_TRY(launch_zero(ctl, 64, st));
    if (hist) HIP_TRY(launch_zero(Hd, H_bytes, st));
    s = run_rates(m, rates, log_rates, ctl, scr, st, &rates);
    if (s) return s;
    NetDev n = base_net(m, rates, n_traj, t_end, grid, G, seed, max_events);
    n.ginfo = (const GridInfo *)((char *)ctl + 64);
    HIP_TRY(launch_grid_info(grid, G, t_end, ctl, st));
    n.D = (unsigned long long *)D;
    n.Dhi = (unsigned long long *)Dhi;
    if (hist) {
        n.Hd = (int32_t *)Hd;
        n.nb_hist = hist->nbins;
        n.h_species = hist->species;
        n.h_lo = hist->lo;
        n.h_width = hist->width;
    }
    // the forward tuner (tune given) times a run's first forward: index order
    const uint32_t *order_keys = (fixed || tune) ? nullptr : fwd_hint(m, rid);
    n.len_out = fixed ? nullptr : hint_begin(m, rid, cap);
    WorkList wl;
    std::memset(&wl, 0, sizeof wl);
    wl.net0 = n;
    wl.range_begin = 0;
    wl.range_end = n_traj;
    wl.n_items = (int32_t)n_items;
    wl.counter = (unsigned int *)ctl;
    wl.stats = (unsigned long long *)((char *)ctl + 32);

    float kms = 0.f;
    FwdTune cfg = tune ? *tune : (fixed ? FwdTune() : tune_lookup(m, n_traj, G, dev));
    if (fixed) cfg.slab = 0;
    s = launch_forward(m, wl, n_items, dev, st, rates, scr, n.D, (stats && !fixed) ? &kms : nullptr, cfg,
                       !fixed && !cap, false, order_keys);
    if (n.len_out && !cap) hint_end(m, rid, s == SSA_OK && g_launch.form == SSA_FORM_GENERATIONS);
    if (s) return s;
    HIP_TRY(launch_finalize(n.D, n.Dhi, G, m->S, m->d_x0, n_traj, mean, var, ctl_status(ctl), st));
    if (hist) {
        const int32_t xv = m->x0[hist->species];
        const int32_t ib = xv < hist->lo ? 0 : std::min((xv - hist->lo) / hist->width, hist->nbins - 1);
        hipLaunchKernelGGL(hist_prefix_kernel, dim3(hist->nbins), dim3(1024), 0, st, (const int32_t *)Hd, G,
                           hist->nbins, ib, n_traj, d_hist, (const unsigned long long *)ctl_flags(ctl));
        HIP_TRY(hipGetLastError());
    }
    if (stats) {
        s = collect_stats(wl.stats, st, nullptr, nullptr, stats);
        stats->kernel_ms = kms;
        return s;
    }
    return SSA_OK;
}

}  // namespace

ssa_status ssa_run_device(const ssa_model *m, const double *rates, const double *log_rates, int64_t n_traj,
                          double t_end, const double *grid, int32_t G, uint64_t seed, uint64_t max_events,
                          double *mean, double *var, const ssa_hist_spec *hist, uint32_t *d_hist, void *stream,
                          ssa_stats *stats) {
    return run_device_impl(m, rates, log_rates, n_traj, t_end, grid, G, seed, max_events, mean, var, hist, d_hist,
                           stream, stats, nullptr);
}

ssa_status ssa_run_device_static(const ssa_model *m, const double *rates, const double *log_rates, int64_t n_traj,
                                 double t_end, const double *grid, int32_t G, uint64_t seed, uint64_t max_events,
                                 double *mean, double *var, const ssa_hist_spec *hist, uint32_t *d_hist,
                                 void *stream, ssa_stats *stats) {
    if (!m) return fail(SSA_E_INVALID, "model is NULL");
    if (G <= 0) return fail(SSA_E_INVALID, "grid must have at least one point");
    // upper bound of the pieces run_device_impl and launch_forward take, in their order
    const size_t cells = (size_t)G * m->S;
    size_t need = FixedScratch::piece(16 * cells) + FixedScratch::piece(8 * cells) + FixedScratch::piece(kCtlBytes);
    if (hist && hist->nbins > 0) need += FixedScratch::piece(sizeof(int32_t) * cells / m->S * (size_t)hist->nbins);
    if (log_rates) need += FixedScratch::piece(sizeof(double) * (size_t)m->m_pad);
    if (rates || log_rates)
        need += FixedScratch::piece(sizeof(double) * std::max<size_t>((size_t)m->m_pad, (size_t)m->dep_nnz));
    if (need > kStaticScratchBytes)
        return fail(SSA_E_INVALID,
                    "the call needs %zu bytes of scratch and the static area holds %zu: fewer grid points, species "
                    "or histogram bins, or ssa_run_device",
                    need, kStaticScratchBytes);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    void *base = nullptr;
    ssa_status s = static_scratch(dev, &base);
    if (s) return s;
    FixedScratch area(base, kStaticScratchBytes);
    return run_device_impl(m, rates, log_rates, n_traj, t_end, grid, G, seed, max_events, mean, var, hist, d_hist,
                           stream, stats, nullptr, &area);
}

void ssa_run_destroy(ssa_run_state *r) {
    if (!r) return;
    for (void *p : {(void *)r->d_grid, (void *)r->d_rates, (void *)r->D, (void *)r->Dhi, (void *)r->Hd, r->ctl,
                    (void *)r->sx[0], (void *)r->sx[1], (void *)r->st[0], (void *)r->st[1], (void *)r->sk[0],
                    (void *)r->sk[1], (void *)r->sev[0], (void *)r->sev[1]})
        if (p) (void)hipFree(p);
    delete r;
}

ssa_status ssa_run_begin(const ssa_model *m, const double *rates, int64_t n_traj, double t_end, const double *grid,
                         int32_t G, uint64_t seed, uint64_t max_events, const ssa_hist_spec *hist, ssa_run_state **out) {
    if (!out) return fail(SSA_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!m) return fail(SSA_E_INVALID, "model is NULL");
    if (n_traj <= 0 || n_traj > max_traj(m)) return fail(SSA_E_INVALID, "n_traj must be in 1 .. %lld", (long long)max_traj(m));
    ssa_status s = validate_grid_host(grid, G, t_end);
    if (s) return s;
    if (hist && (hist->species < 0 || hist->species >= m->S || hist->width <= 0 || hist->nbins <= 0 ||
                 hist->nbins > 4096))
        return fail(SSA_E_INVALID, "bad histogram spec");
    if (rates)
        for (int32_t j = 0; j < m->M; ++j)
            if (!(rates[j] >= 0.0) || !std::isfinite(rates[j])) return fail(SSA_E_INVALID, "rates[%d] invalid", j);
    if (m->order != SSA_SUM_SEQ || !jit_eligible(m))
        return fail(SSA_E_UNSUPPORTED, "runs in epochs need the specialised kernels (sequential order, at most %d "
                                       "reactions and %d species)", kJitMaxReactions, kJitMaxSpecies);
    auto *r = new (std::nothrow) ssa_run_state;
    if (!r) return fail(SSA_E_NOMEM, "host allocation failed");
    r->m = m;
    r->n_traj = n_traj;
    r->t_end = t_end;
    r->G = G;
    r->seed = seed;
    r->max_events = max_events;
    r->has_hist = hist != nullptr;
    if (hist) r->hist = *hist;
    auto bad = [&](hipError_t e) {
        ssa_run_destroy(r);
        return fail(e == hipErrorOutOfMemory ? SSA_E_NOMEM : SSA_E_DEVICE, "%s", hipGetErrorString(e));
    };
    hipError_t e = hipGetDevice(&r->device);
    const size_t cells = (size_t)G * m->S;
    if (e == hipSuccess) e = hipMalloc(&r->d_grid, sizeof(double) * G);
    if (e == hipSuccess) e = hipMemcpy(r->d_grid, grid, sizeof(double) * G, hipMemcpyHostToDevice);
    if (e == hipSuccess && rates) e = hipMalloc(&r->d_rates, sizeof(double) * m->M);
    if (e == hipSuccess && rates) e = hipMemcpy(r->d_rates, rates, sizeof(double) * m->M, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&r->D, sizeof(unsigned long long) * 2 * cells);
    if (e == hipSuccess) e = hipMalloc(&r->Dhi, sizeof(unsigned long long) * cells);
    if (e == hipSuccess && hist) e = hipMalloc(&r->Hd, sizeof(int32_t) * (size_t)G * hist->nbins);
    if (e == hipSuccess) e = hipMalloc(&r->ctl, kCtlBytes);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipMalloc(&r->sx[b], sizeof(int32_t) * (size_t)n_traj * m->S);
        if (e == hipSuccess) e = hipMalloc(&r->st[b], sizeof(double) * (size_t)n_traj);
        if (e == hipSuccess) e = hipMalloc(&r->sk[b], sizeof(uint64_t) * (size_t)n_traj);
        if (e == hipSuccess) e = hipMalloc(&r->sev[b], sizeof(uint64_t) * (size_t)n_traj);
    }
    if (e == hipSuccess) e = hipMemset(r->D, 0, sizeof(unsigned long long) * 2 * cells);
    if (e == hipSuccess) e = hipMemset(r->Dhi, 0, sizeof(unsigned long long) * cells);
    if (e == hipSuccess && hist) e = hipMemset(r->Hd, 0, sizeof(int32_t) * (size_t)G * hist->nbins);
    if (e == hipSuccess) {
        const GridInfo gi = host_grid_info(grid, G, t_end);
        e = hipMemcpy((char *)r->ctl + 64, &gi, sizeof gi, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return bad(e);
    *out = r;
    return SSA_OK;
}

ssa_status ssa_run_advance(ssa_run_state *r, double t_until, void *stream, ssa_stats *stats) {
    if (!r) return fail(SSA_E_INVALID, "run is NULL");
    if (std::isnan(t_until)) return fail(SSA_E_INVALID, "t_until is NaN");
    const double t1 = std::min(t_until, r->t_end);
    if (r->started && !(t1 > r->t_done)) {
        if (stats) std::memset(stats, 0, sizeof *stats);
        return SSA_OK;
    }
    const ssa_model *m = r->m;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != r->device) return fail(SSA_E_INVALID, "the run was begun on device %d", r->device);
    StreamScratch scr(st);
    HIP_TRY(launch_zero(r->ctl, 64, st));
    NetDev n = base_net(m, r->d_rates, r->n_traj, r->t_end, r->d_grid, r->G, r->seed, r->max_events);
    n.ginfo = (const GridInfo *)((char *)r->ctl + 64);
    n.D = r->D;
    n.Dhi = r->Dhi;
    if (r->has_hist) {
        n.Hd = r->Hd;
        n.nb_hist = r->hist.nbins;
        n.h_species = r->hist.species;
        n.h_lo = r->hist.lo;
        n.h_width = r->hist.width;
    }
    const int wb = r->cur < 0 ? 0 : 1 - r->cur;
    if (r->cur >= 0) {
        n.rs_x = r->sx[r->cur];
        n.rs_t = r->st[r->cur];
        n.rs_k = r->sk[r->cur];
        n.rs_ev = r->sev[r->cur];
    }
    n.ws_x = r->sx[wb];
    n.ws_t = r->st[wb];
    n.ws_k = r->sk[wb];
    n.ws_ev = r->sev[wb];
    n.t_pause = t1;
    WorkList wl;
    std::memset(&wl, 0, sizeof wl);
    wl.net0 = n;
    wl.range_begin = 0;
    wl.range_end = r->n_traj;
    const int64_t n_items = (r->n_traj + kChunk - 1) / kChunk;
    wl.n_items = (int32_t)n_items;
    wl.counter = (unsigned int *)r->ctl;
    wl.stats = (unsigned long long *)((char *)r->ctl + 32);
    FwdTune cfg = tune_lookup(m, r->n_traj, r->G, dev);
    cfg.slab = 0;
    float kms = 0.f;
    ssa_status s = launch_forward(m, wl, n_items, dev, st, r->d_rates, scr, r->D, &kms, cfg, true, true);
    if (s) return s;
    unsigned long long h[3] = {0, 0, 0};
    HIP_TRY(hipMemcpyAsync(h, wl.stats, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    r->cur = wb;
    r->started = true;
    r->t_done = t1;
    r->events += h[0];
    r->max_steps = std::max(r->max_steps, h[1]);
    r->flags |= (uint32_t)h[2];
    r->kernel_ms += kms;
    if (stats) {
        stats->events = h[0];
        stats->max_steps = h[1];
        stats->flags = (uint32_t)h[2];
        stats->kernel_ms = kms;
        stats->form = g_launch.form;
        stats->blocks = g_launch.blocks;
    }
    if (h[2] & kFlagOverflow) return fail(SSA_E_OVERFLOW, "a species count left the int32 range");
    if (h[2] & kFlagEventLimit) return fail(SSA_E_EVENT_LIMIT, "a trajectory reached max_events before t_end");
    if (r->events >= kMaxExactEvents)
        return fail(SSA_E_UNSUPPORTED, "%llu events in one run: the exact integer sums hold at most 2^39",
                    (unsigned long long)r->events);
    return SSA_OK;
}

ssa_status ssa_run_finish(ssa_run_state *r, double *mean, double *var, uint32_t *d_hist, void *stream,
                          ssa_stats *stats) {
    if (!r || !mean || !var) return fail(SSA_E_INVALID, "NULL argument");
    if (r->has_hist != (d_hist != nullptr)) return fail(SSA_E_INVALID, "the histogram buffer goes with the run's spec");
    if (!r->started || r->t_done < r->t_end)
        return fail(SSA_E_INVALID, "the run has reached t = %g of %g: advance it to t_end first", r->t_done, r->t_end);
    if (r->events >= kMaxExactEvents || (r->flags & (kFlagOverflow | kFlagEventLimit)))
        return fail(SSA_E_UNSUPPORTED, "the run did not complete with exact sums");
    hipStream_t st = (hipStream_t)stream;
    // the finalize reads the run's totals from the status words
    const unsigned long long tot[3] = {r->events, r->max_steps, 0ull};
    HIP_TRY(hipMemcpyAsync((char *)r->ctl + 32, tot, sizeof tot, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_finalize(r->D, r->Dhi, r->G, r->m->S, r->m->d_x0, r->n_traj, mean, var, ctl_status(r->ctl), st));
    if (r->has_hist) {
        const int32_t xv = r->m->x0[r->hist.species];
        const int32_t ib = xv < r->hist.lo ? 0 : std::min((xv - r->hist.lo) / r->hist.width, r->hist.nbins - 1);
        hipLaunchKernelGGL(hist_prefix_kernel, dim3(r->hist.nbins), dim3(1024), 0, st, (const int32_t *)r->Hd, r->G,
                           r->hist.nbins, ib, r->n_traj, d_hist, (const unsigned long long *)ctl_flags(r->ctl));
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (stats) {
        stats->events = r->events;
        stats->max_steps = r->max_steps;
        stats->flags = r->flags;
        stats->kernel_ms = r->kernel_ms;
        stats->form = SSA_FORM_GENERATIONS;
        stats->blocks = 0;
    }
    return SSA_OK;
}

ssa_status ssa_autotune_forward(const ssa_model *m, const double *rates, int64_t n_traj, double t_end,
                                const double *grid, int32_t G, uint64_t seed, void *stream, ssa_tune_result *result) {
    if (!m || !grid || G <= 0 || n_traj <= 0) return fail(SSA_E_INVALID, "bad argument");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipStream_t st = (hipStream_t)stream;
    const size_t cells = (size_t)G * m->S;
    double *mean = nullptr, *var = nullptr;
    HIP_TRY(hipMallocAsync((void **)&mean, sizeof(double) * cells, st));
    HIP_TRY(hipMallocAsync((void **)&var, sizeof(double) * cells, st));
    // candidates: the default first, then the window sizes, with and without slabs
    std::vector<FwdTune> cand(1);
    if (m->order != SSA_SUM_BLOCK64) {
        for (int32_t wb : {2048, 4096, 8192, 16384}) {
            FwdTune t;
            t.win_bytes = wb;
            t.slab = 0;
            cand.push_back(t);
            t.slab = 1;
            cand.push_back(t);
        }
    }
    FwdTune best;
    float best_ms = 0.f, default_ms = 0.f;
    ssa_status status = SSA_OK;
    // a configuration's time: the best of two timed calls after one with statistics (which
    // warms up, checks the run and reports the grid)
    auto time_cfg = [&](const FwdTune &c, float &ms, ssa_stats &stt) {
        status = run_device_impl(m, rates, nullptr, n_traj, t_end, grid, G, seed, 0, mean, var, nullptr, nullptr,
                                 stream, &stt, &c);
        for (int rep = 0; rep < 2 && status == SSA_OK; ++rep) {
            float t = 0.f;
            status = time_call(st, [&] {
                return run_device_impl(m, rates, nullptr, n_traj, t_end, grid, G, seed, 0, mean, var, nullptr,
                                       nullptr, stream, nullptr, &c);
            }, t);
            ms = rep ? std::min(ms, t) : t;
        }
    };
    for (size_t c = 0; c < cand.size() && status == SSA_OK; ++c) {
        float ms = 0.f;
        ssa_stats stt;
        time_cfg(cand[c], ms, stt);
        if (status) break;
        if (c == 0) default_ms = ms;
        if (c == 0 || ms < best_ms) {
            best_ms = ms;
            best = cand[c];
        }
    }
    // then, with the best window, the launch form of the specialised kernels (two-wave blocks
    // at their default count and at 2 and 4 per CU; generations at the occupancy limit and at
    // 1/2 and 1/4 of it); the table-driven and 64-chunk kernels have one form
    if (status == SSA_OK && m->order == SSA_SUM_SEQ && jit_eligible(m)) {
        const int64_t n_items = (n_traj + kChunk - 1) / kChunk;
        const FwdTune win = best;
        for (int32_t form : {(int32_t)SSA_FORM_TWO_WAVE, (int32_t)SSA_FORM_GENERATIONS}) {
            int64_t b0 = 0;
            for (int k2 : {1, 2, 4}) {
                FwdTune c = win;
                c.form = form;
                c.blocks = k2 == 1 ? 0
                                   : (form == SSA_FORM_TWO_WAVE ? k2 * cu_count(dev)
                                                                : (int32_t)std::max<int64_t>(1, b0 / k2));
                if (k2 > 1 && !(c.blocks < b0 && c.blocks < n_items)) continue;
                if (form == SSA_FORM_TWO_WAVE && (c.slab == 1)) c.slab = 0;   // two-wave blocks flush atomically
                float ms = 0.f;
                ssa_stats stt;
                time_cfg(c, ms, stt);
                if (status == SSA_OK && k2 == 1) b0 = stt.blocks;
                if (status) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        }
    }
    (void)hipFreeAsync(mean, st);
    (void)hipFreeAsync(var, st);
    if (status) return status;
    best.ms = best_ms;
    tune_store(m, n_traj, G, dev, false, best);
    if (result) {
        result->win_bytes = best.win_bytes;
        result->slab = best.slab;
        result->best_ms = best_ms;
        result->default_ms = default_ms;
        result->form = best.form;
        result->blocks = best.blocks;
    }
    return SSA_OK;
}

ssa_status ssa_run_jacobian_device(const ssa_model *m, const double *rates, const double *log_rates, int64_t n_traj,
                                   double t_end, const double *grid, int32_t G, uint64_t seed, uint64_t max_events,
                                   double *mean, double *var, double *jac, void *stream, ssa_stats *stats) {
    if (!m) return fail(SSA_E_INVALID, "model is NULL");
    if (n_traj <= 0) return fail(SSA_E_INVALID, "n_traj must be > 0");
    if (G <= 0 || !grid || !mean || !var || !jac) return fail(SSA_E_INVALID, "grid / mean / var / jac missing");
    if (!(t_end >= 0.0) || !std::isfinite(t_end)) return fail(SSA_E_INVALID, "t_end must be finite and >= 0");
    if (rates && log_rates) return fail(SSA_E_INVALID, "rates and log_rates are alternatives");
    if (n_traj > max_traj(m)) return fail(SSA_E_INVALID, "n_traj above %lld", (long long)max_traj(m));
    if (m->order != SSA_SUM_SEQ || m->M > kJitMaxReactions || m->S > kJitMaxSpecies)
        return fail(SSA_E_UNSUPPORTED, "the forward Jacobian needs a sequential-order network with at most %d "
                    "reactions and %d species", kJitMaxReactions, kJitMaxSpecies);
    if (m->has_laws) return fail(SSA_E_UNSUPPORTED, "the score of a rate law is not n_j - A_j: no Jacobian");
    const int64_t n_items = (n_traj + kChunk - 1) / kChunk;
    const size_t jrow = (size_t)(m->S + 1) * m->M;
    const size_t slab_bytes = (size_t)n_items * G * jrow * sizeof(double);
    size_t budget = (size_t)4 << 30;
    if (const char *e = std::getenv("SSA_JAC_BYTES")) budget = (size_t)std::strtoull(e, nullptr, 10);
    if (slab_bytes > budget)
        return fail(SSA_E_UNSUPPORTED, "forward Jacobian scratch %zu bytes exceeds %zu (use ssa_backward_device)",
                    slab_bytes, budget);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    bool cap = false;
    ssa_status s = capture_check(m, st, dev, stats, true, false, &cap);
    if (s) return s;
    if (!cap) keep_pool(dev);
    StreamScratch pooled(st);
    CaptureScratch kept(m);
    Scratch &scr = cap ? (Scratch &)kept : (Scratch &)pooled;
    std::shared_ptr<JitKernels> jk;
    s = get_jit(m, dev, jk);
    if (s) return s;

    const size_t cells = (size_t)G * m->S;
    void *D = nullptr, *Dhi = nullptr, *ctl = nullptr, *slabs = nullptr;
    HIP_TRY(scr.alloc(&D, sizeof(unsigned long long) * 2 * cells));
    HIP_TRY(scr.alloc(&Dhi, sizeof(unsigned long long) * cells));
    HIP_TRY(scr.alloc(&ctl, kCtlBytes));
    HIP_TRY(scr.alloc(&slabs, slab_bytes));
    HIP_TRY(launch_zero(D, sizeof(unsigned long long) * 2 * cells, st));
    HIP_TRY(launch_zero(Dhi, sizeof(unsigned long long) * cells, st));
    HIP_TRY(launch_zero(ctl, 64, st));
    s = run_rates(m, rates, log_rates, ctl, scr, st, &rates);
    if (s) return s;
    NetDev n = base_net(m, rates, n_traj, t_end, grid, G, seed, max_events);
    n.ginfo = (const GridInfo *)((char *)ctl + 64);
    HIP_TRY(launch_grid_info(grid, G, t_end, ctl, st));
    n.D = (unsigned long long *)D;
    n.Dhi = (unsigned long long *)Dhi;
    WorkList wl;
    std::memset(&wl, 0, sizeof wl);
    wl.net0 = n;
    wl.range_begin = 0;
    wl.range_end = n_traj;
    wl.n_items = (int32_t)n_items;
    wl.counter = (unsigned int *)ctl;
    wl.stats = (unsigned long long *)((char *)ctl + 32);
    wl.jac_slabs = (double *)slabs;
    // window: moments (S x 2 words) and Jacobian ((S+1) x M words) per bin, 16 KB per wave
    const size_t per_bin = (size_t)m->S * 2 + jrow;
    int32_t W = 1;
    while (W < 1024 && (size_t)(2 * W) * per_bin * 8 <= (size_t)16384 && W < G) W *= 2;
    wl.win_bins = W;
    wl.win_words = (int32_t)(W * per_bin);
    const size_t lds = (size_t)(kBlock / kWave) * wl.win_words * sizeof(long long);
    int per_cu = 0;
    HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, jk->fwd_jac, kBlock, lds));
    const int64_t blocks = grid_blocks(per_cu, dev, n_items);
    EventPair ev;
    if (stats && ev.make()) HIP_TRY(hipEventRecord(ev.a, st));
    {
        void *args[] = {&wl};
        note_launch(SSA_FORM_GENERATIONS, blocks);
        HIP_TRY(hipModuleLaunchKernel(jk->fwd_jac, (unsigned)blocks, 1, 1, kBlock, 1, 1, (unsigned)lds, st, args,
                                      nullptr));
    }
    if (stats && ev.b) HIP_TRY(hipEventRecord(ev.b, st));
    HIP_TRY(launch_finalize(n.D, n.Dhi, G, m->S, m->d_x0, n_traj, mean, var, ctl_status(ctl), st));
    {
        const int64_t jc = (int64_t)cells * m->M;
        hipLaunchKernelGGL(jacobian_final_kernel, dim3((unsigned)((jc + 255) / 256)), dim3(256), 0, st,
                           (const double *)slabs, n_items, G, m->S, m->M, n_traj, (const double *)mean, jac,
                           (const unsigned long long *)ctl_flags(ctl));
        HIP_TRY(hipGetLastError());
    }
    if (stats) return collect_stats(wl.stats, st, ev.a, ev.b, stats);
    return SSA_OK;
}

ssa_status ssa_run_cov_device(const ssa_model *m, const double *rates, int64_t n_traj, double t_end,
                              const double *grid, int32_t G, uint64_t seed, uint64_t max_events, double *mean,
                              double *cov, void *stream, ssa_stats *stats) {
    if (!m) return fail(SSA_E_INVALID, "model is NULL");
    if (n_traj <= 0) return fail(SSA_E_INVALID, "n_traj must be > 0");
    if (G <= 0 || !grid || !mean || !cov) return fail(SSA_E_INVALID, "grid / mean / cov missing");
    if (!(t_end >= 0.0) || !std::isfinite(t_end)) return fail(SSA_E_INVALID, "t_end must be finite and >= 0");
    if (n_traj > max_traj(m)) return fail(SSA_E_INVALID, "n_traj above %lld", (long long)max_traj(m));
    if (m->order != SSA_SUM_SEQ || m->M > kJitMaxReactions || m->S > kJitMaxSpecies)
        return fail(SSA_E_UNSUPPORTED, "the covariance pass needs a sequential-order network with at most %d "
                    "reactions and %d species", kJitMaxReactions, kJitMaxSpecies);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    bool cap = false;
    ssa_status s = capture_check(m, st, dev, stats, true, false, &cap);
    if (s) return s;
    if (!cap) keep_pool(dev);
    StreamScratch pooled(st);
    CaptureScratch kept(m);
    Scratch &scr = cap ? (Scratch &)kept : (Scratch &)pooled;
    std::shared_ptr<JitKernels> jk;
    s = get_jit(m, dev, jk);
    if (s) return s;
    const int32_t S = m->S, npairs = S * (S - 1) / 2;
    const size_t row = (size_t)2 * S + npairs, hrow = (size_t)S + npairs;
    NetDev n = base_net(m, rates, n_traj, t_end, grid, G, seed, max_events);
    void *D = nullptr, *Dhi = nullptr, *ctl = nullptr, *sx = nullptr, *sxx = nullptr;
    HIP_TRY(scr.alloc(&D, sizeof(unsigned long long) * row * G));
    HIP_TRY(scr.alloc(&Dhi, sizeof(unsigned long long) * hrow * G));
    HIP_TRY(scr.alloc(&ctl, kCtlBytes));
    HIP_TRY(scr.alloc(&sx, sizeof(int64_t) * (size_t)G * S));
    HIP_TRY(scr.alloc(&sxx, sizeof(i128s) * hrow * G));
    HIP_TRY(launch_zero(D, sizeof(unsigned long long) * row * G, st));
    HIP_TRY(launch_zero(Dhi, sizeof(unsigned long long) * hrow * G, st));
    HIP_TRY(launch_zero(ctl, 64, st));
    n.ginfo = (const GridInfo *)((char *)ctl + 64);
    HIP_TRY(launch_grid_info(grid, G, t_end, ctl, st));
    n.D = (unsigned long long *)D;
    n.Dhi = (unsigned long long *)Dhi;
    WorkList wl;
    std::memset(&wl, 0, sizeof wl);
    wl.net0 = n;
    wl.range_begin = 0;
    wl.range_end = n_traj;
    const int64_t n_items = (n_traj + kChunk - 1) / kChunk;
    wl.n_items = (int32_t)n_items;
    wl.counter = (unsigned int *)ctl;
    wl.stats = (unsigned long long *)((char *)ctl + 32);
    int32_t W = 1;
    while (W < 1024 && (size_t)(2 * W) * row * 8 <= window_budget(false) && W < G) W *= 2;
    wl.win_bins = W;
    wl.win_words = (int32_t)(W * win_stride((int32_t)row));
    const size_t lds = (size_t)(kBlock / kWave) * wl.win_words * sizeof(long long);
    int per_cu = 0;
    HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, jk->fwd_cov, kBlock, lds));
    const int64_t blocks = grid_blocks(per_cu, dev, n_items);
    EventPair ev;
    if (stats && ev.make()) HIP_TRY(hipEventRecord(ev.a, st));
    {
        void *args[] = {&wl};
        note_launch(SSA_FORM_GENERATIONS, blocks);
        HIP_TRY(hipModuleLaunchKernel(jk->fwd_cov, (unsigned)blocks, 1, 1, kBlock, 1, 1, (unsigned)lds, st, args,
                                      nullptr));
    }
    if (stats && ev.b) HIP_TRY(hipEventRecord(ev.b, st));
    hipLaunchKernelGGL(cov_prefix_kernel, dim3((unsigned)hrow), dim3(1024), 0, st, (const unsigned long long *)D,
                       (const unsigned long long *)Dhi, G, S, m->d_x0, n_traj, (int64_t *)sx, (i128s *)sxx);
    HIP_TRY(hipGetLastError());
    const int64_t cells = (int64_t)G * S * S;
    hipLaunchKernelGGL(cov_final_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st,
                       (const int64_t *)sx, (const i128s *)sxx, G, S, n_traj, mean, cov, ctl_status(ctl));
    HIP_TRY(hipGetLastError());
    if (stats) return collect_stats(wl.stats, st, ev.a, ev.b, stats);
    return SSA_OK;
}

ssa_status ssa_hist_quantiles(const uint32_t *hist, int32_t G, const ssa_hist_spec *spec, int64_t n_traj,
                              const double *qs, int32_t nq, int32_t *out, void *stream) {
    if (!hist || !spec || !qs || !out || G <= 0 || nq <= 0 || n_traj <= 0 || spec->nbins <= 0 || spec->width <= 0)
        return fail(SSA_E_INVALID, "bad argument");
    const int64_t cells = (int64_t)G * nq;
    hipLaunchKernelGGL(hist_quantile_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, hist, G, spec->nbins, spec->lo, spec->width, n_traj, qs, nq, out);
    HIP_TRY(hipGetLastError());
    return SSA_OK;
}

ssa_status ssa_jacobian_vjp(const double *jac, const double *w, int32_t G, int32_t S, int32_t M, double *grad,
                            void *stream) {
    if (!jac || !w || !grad || G <= 0 || S <= 0 || M <= 0) return fail(SSA_E_INVALID, "bad argument");
    hipLaunchKernelGGL(jacobian_vjp_kernel, dim3((unsigned)M), dim3(256), 0, (hipStream_t)stream, jac, w,
                       (int64_t)G * S, M, grad);
    HIP_TRY(hipGetLastError());
    return SSA_OK;
}

ssa_status ssa_rates_from_log(const double *log_rates, int32_t n, double *rates, void *stream) {
    if (!log_rates || !rates || n <= 0) return fail(SSA_E_INVALID, "bad argument");
    hipLaunchKernelGGL(rates_from_log_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       log_rates, n, n, rates, (unsigned int *)nullptr, (unsigned long long *)nullptr);
    HIP_TRY(hipGetLastError());
    return SSA_OK;
}

ssa_status ssa_run(const ssa_model *m, int64_t n_traj, double t_end, const double *grid, int32_t G, uint64_t seed,
                   double *mean, double *var, ssa_stats *stats) {
    if (!m || !mean || !var) return fail(SSA_E_INVALID, "NULL argument");
    ssa_status s = validate_grid_host(grid, G, t_end);
    if (s) return s;
    double *dg = nullptr, *dm = nullptr, *dv = nullptr;
    const size_t cells = (size_t)G * m->S;
    auto cleanup = [&] {
        if (dg) (void)hipFree(dg);
        if (dm) (void)hipFree(dm);
        if (dv) (void)hipFree(dv);
    };
    hipError_t e = hipMalloc(&dg, sizeof(double) * G);
    if (e == hipSuccess) e = hipMalloc(&dm, sizeof(double) * cells);
    if (e == hipSuccess) e = hipMalloc(&dv, sizeof(double) * cells);
    if (e == hipSuccess) e = hipMemcpy(dg, grid, sizeof(double) * G, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        cleanup();
        return fail(e == hipErrorOutOfMemory ? SSA_E_NOMEM : SSA_E_DEVICE, "%s", hipGetErrorString(e));
    }
    ssa_stats local;
    s = ssa_run_device(m, nullptr, nullptr, n_traj, t_end, dg, G, seed, 0, dm, dv, nullptr, nullptr, nullptr,
                       stats ? stats : &local);
    if (s == SSA_OK) {
        e = hipMemcpy(mean, dm, sizeof(double) * cells, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(var, dv, sizeof(double) * cells, hipMemcpyDeviceToHost);
        if (e != hipSuccess) s = fail(SSA_E_DEVICE, "%s", hipGetErrorString(e));
    }
    cleanup();
    return s;
}

ssa_status ssa_backward_device(const ssa_model *m, const double *rates, const double *log_rates, int64_t n_traj,
                               double t_end, const double *grid, int32_t G, uint64_t seed, uint64_t max_events,
                               const double *w, const double *mhat, double *grad, void *stream, ssa_stats *stats) {
    return ssa_backward_moments_device(m, rates, log_rates, n_traj, t_end, grid, G, seed, max_events, w, mhat, nullptr,
                                       nullptr, grad, stream, stats);
}

namespace {

// The backward with a given launch configuration (tune == nullptr: the cached tuned one).
ssa_status backward_impl(const ssa_model *m, const double *rates, const double *log_rates, int64_t n_traj,
                         double t_end, const double *grid, int32_t G, uint64_t seed, uint64_t max_events,
                         const double *w, const double *mhat, const double *wv, const double *vhat, double *grad,
                         void *stream, ssa_stats *stats, const FwdTune *tune) {
    if (!m) return fail(SSA_E_INVALID, "model is NULL");
    if (n_traj <= 0 || G <= 0 || !grid || !w || !mhat || !grad) return fail(SSA_E_INVALID, "bad argument");
    if ((wv == nullptr) != (vhat == nullptr)) return fail(SSA_E_INVALID, "wv and vhat go together");
    const bool quad = wv != nullptr;
    if (!(t_end >= 0.0) || !std::isfinite(t_end)) return fail(SSA_E_INVALID, "t_end must be finite and >= 0");
    if (m->order == SSA_SUM_SEQ && m->M > kJitMaxReactions)
        return fail(SSA_E_UNSUPPORTED, "backward supports at most %d reactions", kJitMaxReactions);
    if (m->has_laws) return fail(SSA_E_UNSUPPORTED, "the score of a rate law is not n_j - A_j: no backward");
    if (rates && log_rates) return fail(SSA_E_INVALID, "rates and log_rates are alternatives");
    if (n_traj > max_traj(m)) return fail(SSA_E_INVALID, "n_traj above %lld", (long long)max_traj(m));
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const int64_t n_items = (n_traj + kChunk - 1) / kChunk;
    bool cap = false;
    ssa_status s = capture_check(m, st, dev, stats, m->order == SSA_SUM_SEQ && jit_eligible(m),
                                 latency_bound(n_items, dev), &cap);
    if (s) return s;
    if (!cap) keep_pool(dev);
    StreamScratch pooled(st);
    CaptureScratch kept(m);
    Scratch &scr = cap ? (Scratch &)kept : (Scratch &)pooled;
    const RunId rid{n_traj, t_end, seed, max_events, grid, rates, log_rates, G, dev};
    void *gt = nullptr, *gt2 = nullptr, *ctl = nullptr, *bp = nullptr;
    const size_t rows_bytes = sizeof(double) * (size_t)n_traj * m->M;
    const int32_t ncol = quad ? 4 * m->S + 2 : 2 * m->S + 2;
    void *bpt = nullptr;
    HIP_TRY(scr.alloc(&bp, (size_t)12 * ncol * ((size_t)G + 1)));
    HIP_TRY(scr.alloc(&bpt, sizeof(double) * ncol * (size_t)G));
    HIP_TRY(scr.alloc(&gt, rows_bytes));
    HIP_TRY(scr.alloc(&gt2, rows_bytes / 2 + sizeof(double) * m->M));
    HIP_TRY(scr.alloc(&ctl, kCtlBytes));
    HIP_TRY(launch_zero(ctl, 64, st));
    s = run_rates(m, rates, log_rates, ctl, scr, st, &rates);
    if (s) return s;
    NetDev n = base_net(m, rates, n_traj, t_end, grid, G, seed, max_events);
    n.ginfo = (const GridInfo *)((char *)ctl + 64);
    HIP_TRY(launch_grid_info(grid, G, t_end, ctl, st));
    hipLaunchKernelGGL(bwd_prefix_kernel, dim3((unsigned)ncol), dim3(256), 0, st, w, mhat, wv, vhat, grid, G, m->S,
                       bp, (double *)bpt);
    HIP_TRY(hipGetLastError());
    n.bp = bp;
    n.bpt = (const double *)bpt;
    n.bp_quad = quad ? 1 : 0;
    n.gtraj = (double *)gt;
    WorkList wl;
    std::memset(&wl, 0, sizeof wl);
    wl.net0 = n;
    wl.range_begin = 0;
    wl.range_end = n_traj;
    wl.n_items = (int32_t)n_items;
    wl.counter = (unsigned int *)ctl;
    wl.stats = (unsigned long long *)((char *)ctl + 32);
    const FwdTune cfg = tune ? *tune : tune_lookup(m, n_traj, G, dev, true);
    // the lane kernels take the trajectories longest first when the forward of this run
    // recorded their lengths
    if (m->order == SSA_SUM_SEQ && (!jit_eligible(m) || bwd_form(n_items, dev, cfg.form) != SSA_FORM_TWO_WAVE)) {
        s = hint_order(m, rid, scr, st, &wl.perm);
        if (s) return s;
    }
    EventPair ev;
    if (stats && ev.make()) HIP_TRY(hipEventRecord(ev.a, st));
    s = launch_single(kBwd, m, wl, n_items, dev, st, rates, scr, quad, cfg.form, cfg.blocks);
    if (s) return s;
    g_launch.ordered = wl.perm ? 1u : 0u;
    if (stats && ev.b) HIP_TRY(hipEventRecord(ev.b, st));
    // fixed-order pairwise reduction of the per-trajectory rows
    double *src = (double *)gt, *dst = (double *)gt2;
    int64_t rows = n_traj;
    while (rows > 1) {
        int32_t L = 0;          // up to 8 levels per launch (tiles of 256 rows)
        while (L < 8 && ((int64_t)1 << L) < rows) ++L;
        const int64_t tiles = (rows + ((int64_t)1 << L) - 1) >> L;
        hipLaunchKernelGGL(pair_sum_kernel, dim3((unsigned)tiles, (unsigned)m->M), dim3(256), 0, st, src, rows,
                           m->M, L, dst);
        HIP_TRY(hipGetLastError());
        std::swap(src, dst);
        rows = tiles;
    }
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((m->M + 255) / 256)), dim3(256), 0, st, src, m->M,
                       1.0 / (double)n_traj, grad, (const unsigned long long *)ctl_flags(ctl));
    HIP_TRY(hipGetLastError());
    if (stats) return collect_stats(wl.stats, st, ev.a, ev.b, stats);
    return SSA_OK;
}

}  // namespace

ssa_status ssa_backward_moments_device(const ssa_model *m, const double *rates, const double *log_rates,
                                       int64_t n_traj, double t_end, const double *grid, int32_t G, uint64_t seed,
                                       uint64_t max_events, const double *w, const double *mhat, const double *wv,
                                       const double *vhat, double *grad, void *stream, ssa_stats *stats) {
    return backward_impl(m, rates, log_rates, n_traj, t_end, grid, G, seed, max_events, w, mhat, wv, vhat, grad,
                         stream, stats, nullptr);
}

ssa_status ssa_autotune_backward(const ssa_model *m, const double *rates, int64_t n_traj, double t_end,
                                 const double *grid, int32_t G, uint64_t seed, void *stream, ssa_tune_result *result) {
    if (!m || !grid || G <= 0 || n_traj <= 0) return fail(SSA_E_INVALID, "bad argument");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipStream_t st = (hipStream_t)stream;
    const size_t cells = (size_t)G * m->S;
    double *w = nullptr, *mhat = nullptr, *grad = nullptr;
    HIP_TRY(hipMallocAsync((void **)&w, sizeof(double) * cells, st));
    HIP_TRY(hipMallocAsync((void **)&mhat, sizeof(double) * cells, st));
    HIP_TRY(hipMallocAsync((void **)&grad, sizeof(double) * (size_t)m->M, st));
    double one = 1.0;
    unsigned long long one_bits = 0;
    std::memcpy(&one_bits, &one, sizeof one_bits);
    HIP_TRY(launch_fill(w, cells, one_bits, st));      // weights and centring: any values time the same work
    HIP_TRY(launch_zero(mhat, sizeof(double) * cells, st));
    ssa_status status = SSA_OK;
    // a configuration's time: the best of two timed calls after one with statistics
    auto time_cfg = [&](const FwdTune &c, float &ms, ssa_stats &last) {
        ms = 0.f;
        status = backward_impl(m, rates, nullptr, n_traj, t_end, grid, G, seed, 0, w, mhat, nullptr, nullptr, grad,
                               stream, &last, &c);
        for (int rep = 0; rep < 2 && status == SSA_OK; ++rep) {
            float t = 0.f;
            status = time_call(st, [&] {
                return backward_impl(m, rates, nullptr, n_traj, t_end, grid, G, seed, 0, w, mhat, nullptr, nullptr,
                                     grad, stream, nullptr, &c);
            }, t);
            ms = rep ? std::min(ms, t) : t;
        }
    };
    // the forward of the same run first: a backward after it takes the trajectories in the
    // order of their recorded lengths, as it will in use
    {
        double *mv = nullptr;
        if (hipMallocAsync((void **)&mv, 2 * sizeof(double) * cells, st) != hipSuccess) {
            status = fail(SSA_E_NOMEM, "autotune scratch");
        } else {
            status = run_device_impl(m, rates, nullptr, n_traj, t_end, grid, G, seed, 0, mv, mv + cells, nullptr,
                                     nullptr, stream, nullptr, nullptr);
            (void)hipFreeAsync(mv, st);
        }
    }
    FwdTune base;
    float default_ms = 0.f;
    ssa_stats s0;
    time_cfg(base, default_ms, s0);
    FwdTune best = base;
    float best_ms = default_ms;
    // candidates (specialised kernels only): each form at its default grid and at 1/2 and
    // 1/4 of it (the persistent forms), or at 2 and 4 blocks per CU (two-wave blocks)
    auto consider = [&](const FwdTune &c, ssa_stats &sx) {
        float ms = 0.f;
        time_cfg(c, ms, sx);
        if (status == SSA_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    };
    if (status == SSA_OK && m->order == SSA_SUM_SEQ && jit_eligible(m)) {
        const int64_t n_items = (n_traj + kChunk - 1) / kChunk;
        for (int32_t form : {(int32_t)SSA_FORM_TWO_WAVE, (int32_t)SSA_FORM_GENERATIONS, (int32_t)SSA_FORM_REFILL}) {
            FwdTune c;
            c.form = form;
            ssa_stats sx;
            consider(c, sx);
            const int64_t b0 = sx.blocks;
            for (int k2 : {2, 4}) {
                if (status) break;
                c.blocks = form == SSA_FORM_TWO_WAVE ? k2 * cu_count(dev) : (int32_t)std::max<int64_t>(1, b0 / k2);
                if (c.blocks < b0 && c.blocks < n_items) consider(c, sx);
            }
        }
    }
    (void)hipFreeAsync(w, st);
    (void)hipFreeAsync(mhat, st);
    (void)hipFreeAsync(grad, st);
    if (status) return status;
    best.ms = best_ms;
    tune_store(m, n_traj, G, dev, true, best);
    if (result) {
        result->win_bytes = 0;
        result->slab = -1;
        result->best_ms = best_ms;
        result->default_ms = default_ms;
        result->form = best.form;
        result->blocks = best.blocks;
    }
    return SSA_OK;
}

ssa_status ssa_record(const ssa_model *m, const double *rates, int64_t traj_begin, int64_t count, double t_end,
                      const double *grid, int32_t G, uint64_t seed, uint64_t max_events, int32_t *states,
                      uint64_t *events, uint64_t *draws, double *t_last, int64_t *n_fired, double *a_int) {
    if (!m || !states || !events || !draws || !t_last) return fail(SSA_E_INVALID, "NULL argument");
    if (traj_begin < 0 || count <= 0) return fail(SSA_E_INVALID, "bad trajectory range");
    if (count > ((int64_t)1 << 31) * kChunk) return fail(SSA_E_INVALID, "count too large");
    ssa_status s = validate_grid_host(grid, G, t_end);
    if (s) return s;
    if (m->order == SSA_SUM_SEQ && m->M > kJitMaxReactions)
        return fail(SSA_E_UNSUPPORTED, "record supports at most %d reactions", kJitMaxReactions);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipStream_t st = nullptr;
    StreamScratch scr(st);
    const size_t sb = sizeof(int32_t) * (size_t)count * G * m->S;
    void *d_grid = nullptr, *d_states = nullptr, *d_ev = nullptr, *d_dr = nullptr, *d_tl = nullptr, *d_nf = nullptr,
         *d_ai = nullptr, *d_rates = nullptr, *ctl = nullptr;
    HIP_TRY(scr.alloc(&d_grid, sizeof(double) * G));
    HIP_TRY(scr.alloc(&d_states, sb));
    HIP_TRY(scr.alloc(&d_ev, sizeof(uint64_t) * count));
    HIP_TRY(scr.alloc(&d_dr, sizeof(uint64_t) * count));
    HIP_TRY(scr.alloc(&d_tl, sizeof(double) * count));
    HIP_TRY(scr.alloc(&d_nf, sizeof(int64_t) * count * m->M));
    HIP_TRY(scr.alloc(&d_ai, sizeof(double) * count * m->M));
    HIP_TRY(scr.alloc(&ctl, 64 + sizeof(GridInfo)));
    if (rates) HIP_TRY(scr.alloc(&d_rates, sizeof(double) * m->M));
    HIP_TRY(hipMemcpyAsync(d_grid, grid, sizeof(double) * G, hipMemcpyHostToDevice, st));
    if (rates) HIP_TRY(hipMemcpyAsync(d_rates, rates, sizeof(double) * m->M, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_zero(ctl, 64, st));
    const GridInfo hgi = host_grid_info(grid, G, t_end);
    HIP_TRY(hipMemcpyAsync((char *)ctl + 64, &hgi, sizeof hgi, hipMemcpyHostToDevice, st));
    NetDev n = base_net(m, (const double *)d_rates, traj_begin + count, t_end, (const double *)d_grid, G, seed,
                        max_events);
    n.ginfo = (const GridInfo *)((char *)ctl + 64);
    n.rec_begin = traj_begin;
    n.rec_states = (int32_t *)d_states;
    n.rec_events = (uint64_t *)d_ev;
    n.rec_draws = (uint64_t *)d_dr;
    n.rec_tlast = (double *)d_tl;
    n.rec_nf = (int64_t *)d_nf;
    n.rec_aint = (double *)d_ai;
    WorkList wl;
    std::memset(&wl, 0, sizeof wl);
    wl.net0 = n;
    wl.range_begin = traj_begin;
    wl.range_end = traj_begin + count;
    const int64_t n_items = (count + kChunk - 1) / kChunk;
    wl.n_items = (int32_t)n_items;
    wl.counter = (unsigned int *)ctl;
    wl.stats = (unsigned long long *)((char *)ctl + 32);
    s = launch_single(kRec, m, wl, n_items, dev, st, (const double *)d_rates, scr);
    if (s) return s;
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpy(states, d_states, sb, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(events, d_ev, sizeof(uint64_t) * count, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(draws, d_dr, sizeof(uint64_t) * count, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t_last, d_tl, sizeof(double) * count, hipMemcpyDeviceToHost));
    if (n_fired) HIP_TRY(hipMemcpy(n_fired, d_nf, sizeof(int64_t) * count * m->M, hipMemcpyDeviceToHost));
    if (a_int) HIP_TRY(hipMemcpy(a_int, d_ai, sizeof(double) * count * m->M, hipMemcpyDeviceToHost));
    unsigned long long h[3] = {0, 0, 0};
    HIP_TRY(hipMemcpy(h, (char *)ctl + 32, sizeof h, hipMemcpyDeviceToHost));
    if (h[2] & kFlagOverflow) return fail(SSA_E_OVERFLOW, "a species count left the int32 range");
    if (h[2] & kFlagEventLimit) return fail(SSA_E_EVENT_LIMIT, "a trajectory reached max_events before t_end");
    return SSA_OK;
}

namespace {

// Inclusive prefix sum of n int32 values (in place allowed); sums holds n / kScanTile + 1
// int32 of scratch.
hipError_t launch_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *sums, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3((unsigned)tiles), dim3(256), 0, st, in, n, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, st, sums, tiles);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)tiles), dim3(256), 0, st, in, n, (const int32_t *)sums, out);
    return hipGetLastError();
}

// Time order of one epoch's event log (see time_bin): the R records among the first
// n_slots slots of (key, val), whose times lie in [t0, t1], end sorted by key in the first R
// slots of (okey, oval); (key, val) serve as the radix sort's second buffer and hold no
// records afterwards.  Scratch: bins [>= B] and big [>= B] int32, n_big one int32, cnt and
// incl [256 rdx_tiles(n_slots)] int32, sums as launch_scan's for 256 rdx_tiles(n_slots).
// B: about R / 16 bins (SSA_SORT_BINS overrides).
int64_t rdx_tiles(int64_t n_slots) { return (n_slots + kRdxTile - 1) / kRdxTile; }

hipError_t sort_event_log(unsigned long long *key, unsigned long long *val, int64_t n_slots, int64_t R, double t0,
                          double t1, unsigned long long *okey, unsigned long long *oval, int32_t *bins, int32_t *big,
                          int32_t *n_big, int32_t *cnt, int32_t *incl, int32_t *sums, int64_t max_bins,
                          hipStream_t st) {
    int64_t B = 1;
    while (B < R / 16 && B < ((int64_t)1 << 25)) B <<= 1;
    if (const char *e = std::getenv("SSA_SORT_BINS")) B = std::max<int64_t>(1, std::strtoll(e, nullptr, 10));
    B = std::min(B, std::max<int64_t>(1, max_bins));
    TimeBins tb;
    tb.t0 = t0;
    tb.scale = t1 > t0 ? (double)B / (t1 - t0) : 0.0;
    tb.B = (int32_t)B;
    tb.pad = 0;
    // bin indices 0 .. B (B: no record) need nbits bits; an odd number of passes of at most
    // 8 bits each leaves the result in (okey, oval)
    int32_t nbits = 1;
    while (((int64_t)1 << nbits) <= B) ++nbits;
    int32_t passes = (nbits + 7) / 8;
    if (passes % 2 == 0) ++passes;
    const int32_t width = (nbits + passes - 1) / passes;
    const uint32_t mask = (1u << width) - 1u;
    const int64_t tiles = rdx_tiles(n_slots);
    unsigned long long *src_k = key, *src_v = val, *dst_k = okey, *dst_v = oval;
    hipError_t e = hipSuccess;
    for (int32_t p = 0; p < passes && e == hipSuccess; ++p) {
        const int32_t shift = p * width;
        hipLaunchKernelGGL(rdx_count_kernel, dim3((unsigned)tiles), dim3(256), 0, st, (const unsigned long long *)src_k,
                           n_slots, tb, shift, mask, (int32_t)tiles, cnt);
        e = launch_scan(cnt, incl, 256 * tiles, sums, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(rdx_scatter_kernel, dim3((unsigned)tiles), dim3(256), 0, st, (const unsigned long long *)src_k,
                           (const unsigned long long *)src_v, n_slots, tb, shift, mask, width, (int32_t)tiles,
                           (const int32_t *)cnt, (const int32_t *)incl, dst_k, dst_v);
        e = hipGetLastError();
        std::swap(src_k, dst_k);
        std::swap(src_v, dst_v);
    }
    if (e != hipSuccess) return e;
    e = launch_zero(n_big, sizeof(int32_t), st);
    if (e != hipSuccess) return e;
    const unsigned gs = (unsigned)std::min<int64_t>((R + 1 + 255) / 256, 8192);
    hipLaunchKernelGGL(bin_start_kernel, dim3(gs), dim3(256), 0, st, (const unsigned long long *)okey, R, tb, bins);
    const unsigned gb = (unsigned)std::min<int64_t>((B + 3) / 4, 8192);
    hipLaunchKernelGGL(bin_sort_small_kernel, dim3(gb), dim3(256), 0, st, okey, oval, (const int32_t *)bins,
                       (int32_t)B, R, big, n_big);
    hipLaunchKernelGGL(bin_sort_big_kernel, dim3(1024), dim3(256), 0, st, okey, oval, (const int32_t *)bins,
                       (int32_t)B, R, (const int32_t *)big, (const int32_t *)n_big);
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Adaptive selective memory: event log -> sort by time -> moments at every distinct event
// time (Avg-Y) -> averages of k successive points (Avg-XY).
// ------------------------------------------------------------------------------------------
// Records per epoch of the event log (SSA_ADAPTIVE_RECORDS overrides; at least 4096).  At
// 2^27 records an epoch holds about 17 GB of log, sums and points.
int64_t adaptive_budget() {
    int64_t b = (int64_t)1 << 27;
    if (const char *e = std::getenv("SSA_ADAPTIVE_RECORDS")) b = std::strtoll(e, nullptr, 10);
    return std::max<int64_t>(std::min<int64_t>(b, (int64_t)INT32_MAX - 1), 4096);
}

ssa_status ssa_adaptive_device(const ssa_model *m, const double *rates, int64_t n_traj, double t_end, uint64_t seed,
                               uint64_t max_events, int64_t k, double *xy_time, double *xy_mean, double *xy_var,
                               int64_t xy_cap, double *y_time, double *y_mean, double *y_var, int64_t y_cap,
                               int64_t *n_points, void *stream, ssa_stats *stats) {
    if (!m || !n_points) return fail(SSA_E_INVALID, "NULL argument");
    n_points[0] = n_points[1] = 0;
    if (n_traj <= 0 || n_traj > ((int64_t)1 << 30)) return fail(SSA_E_INVALID, "need 1 <= n_traj <= 2^30");
    if (k <= 0) return fail(SSA_E_INVALID, "k must be >= 1");
    if (!(t_end >= 0.0) || !std::isfinite(t_end)) return fail(SSA_E_INVALID, "t_end must be finite and >= 0");
    if (m->order == SSA_SUM_SEQ && m->M > kJitMaxReactions)
        return fail(SSA_E_UNSUPPORTED, "the event log in the sequential order supports at most %d reactions",
                    kJitMaxReactions);
    if (m->max_changes > kChg)
        return fail(SSA_E_UNSUPPORTED, "the event log records at most %d changed species per event", kChg);
    if (xy_time && (!xy_mean || !xy_var)) return fail(SSA_E_INVALID, "Avg-XY outputs need time, mean and variance");
    if (y_time && (!y_mean || !y_var)) return fail(SSA_E_INVALID, "Avg-Y outputs need time, mean and variance");
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    keep_pool(dev);
    StreamScratch scr(st);
    EventPair evp;
    const bool timed = stats && evp.make();
    const int32_t S = m->S;
    const bool sizing = !xy_time && !y_time;

    // one-point grid at t_end (the event loop reads a grid view; nothing is aligned to it)
    const double h_grid[1] = {t_end};
    void *d_grid = nullptr, *ctl = nullptr, *cur = nullptr, *carry = nullptr;
    HIP_TRY(scr.alloc(&d_grid, sizeof(double)));
    HIP_TRY(scr.alloc(&ctl, 64 + sizeof(GridInfo)));
    HIP_TRY(scr.alloc(&cur, 2 * sizeof(unsigned long long)));    // record count, reserved slots
    HIP_TRY(scr.alloc(&carry, sizeof(long long) * 3 * (size_t)S));
    HIP_TRY(hipMemcpyAsync(d_grid, h_grid, sizeof(double), hipMemcpyHostToDevice, st));
    const GridInfo hgi = host_grid_info(h_grid, 1, t_end);
    HIP_TRY(hipMemcpyAsync((char *)ctl + 64, &hgi, sizeof hgi, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_zero(carry, sizeof(long long) * 3 * (size_t)S, st));
    NetDev n0 = base_net(m, rates, n_traj, t_end, (const double *)d_grid, 1, seed, max_events);
    n0.ginfo = (const GridInfo *)((char *)ctl + 64);
    n0.ev_cursor = (unsigned long long *)cur;
    n0.ev_resv = (unsigned long long *)cur + 1;
    n0.t_pause = t_end;
    WorkList wl;
    std::memset(&wl, 0, sizeof wl);
    wl.range_begin = 0;
    wl.range_end = n_traj;
    const int64_t n_items = (n_traj + kChunk - 1) / kChunk;
    if (n_items > INT32_MAX) return fail(SSA_E_INVALID, "n_traj too large");
    wl.n_items = (int32_t)n_items;
    wl.counter = (unsigned int *)ctl;
    wl.stats = (unsigned long long *)((char *)ctl + 32);
    unsigned long long tot_events = 0, max_steps = 0;
    uint32_t all_flags = 0;

    // One pass of the event log over the epoch (t0, t1] (the whole run when rs is NULL and
    // t1 == t_end); R receives the records (counted even when they did not fit), Rs the
    // extent of the slots they occupy (R plus the unused ends of the waves' reservations;
    // 0 for kernels that place records at the count).
    unsigned long long Rs = 0;
    auto log_pass = [&](NetDev n, unsigned long long &R, unsigned long long (&h)[3]) -> ssa_status {
        HIP_TRY(launch_zero(ctl, 64, st));
        HIP_TRY(launch_zero(cur, 2 * sizeof(unsigned long long), st));
        wl.net0 = n;
        ssa_status s = launch_single(kEvt, m, wl, n_items, dev, st, rates, scr);
        if (s) return s;
        HIP_TRY(hipMemcpyAsync(&R, cur, sizeof R, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&Rs, (unsigned long long *)cur + 1, sizeof Rs, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(h, (char *)ctl + 32, sizeof h, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h[2] & kFlagOverflow) return fail(SSA_E_OVERFLOW, "a species count left the int32 range");
        if (h[2] & kFlagEventLimit) return fail(SSA_E_EVENT_LIMIT, "a trajectory reached max_events before t_end");
        return SSA_OK;
    };

    if (timed) HIP_TRY(hipEventRecord(evp.a, st));
    // count the whole run's records once: a run that fits the budget is one epoch
    unsigned long long R_all = 0, h0[3] = {0, 0, 0};
    ssa_status s = log_pass(n0, R_all, h0);
    if (s) return s;
    const int64_t budget = adaptive_budget();
    const bool epochs = (int64_t)R_all > budget;
    void *keys0 = nullptr, *keys1 = nullptr, *vals0 = nullptr, *vals1 = nullptr, *stf = nullptr, *rk = nullptr;
    // slots: the records plus the unused ends of each wave's last two reservations (a wave
    // reserves only while it holds work, so at most one wave per work item; a launch holds
    // at most 8192 waves)
    const int64_t waste = std::min<int64_t>(n_items, 8192) * 2 * (int64_t)kLogChunk;
    const int64_t cap =
        std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>((int64_t)R_all, budget), INT32_MAX - 1 - waste));
    const int64_t slots = cap + waste;
    HIP_TRY(scr.alloc(&keys0, sizeof(unsigned long long) * (size_t)slots));
    HIP_TRY(scr.alloc(&keys1, sizeof(unsigned long long) * (size_t)slots));
    HIP_TRY(scr.alloc(&vals0, sizeof(unsigned long long) * (size_t)slots));
    HIP_TRY(scr.alloc(&vals1, sizeof(unsigned long long) * (size_t)slots));
    HIP_TRY(scr.alloc(&stf, sizeof(int32_t) * (size_t)cap));
    HIP_TRY(scr.alloc(&rk, sizeof(int32_t) * (size_t)cap));
    void *scan_sums = nullptr, *n_big = nullptr, *rdx_cnt = nullptr, *rdx_incl = nullptr;
    const int64_t rdx_n = 256 * rdx_tiles(slots);
    HIP_TRY(scr.alloc(&scan_sums, sizeof(int32_t) * (size_t)(std::max<int64_t>(cap, rdx_n) / kScanTile + 2)));
    HIP_TRY(scr.alloc(&n_big, sizeof(int32_t)));
    HIP_TRY(scr.alloc(&rdx_cnt, sizeof(int32_t) * (size_t)rdx_n));
    HIP_TRY(scr.alloc(&rdx_incl, sizeof(int32_t) * (size_t)rdx_n));
    // epochs: saved trajectory states, double-buffered
    void *sx[2] = {nullptr, nullptr}, *stt[2] = {nullptr, nullptr}, *skk[2] = {nullptr, nullptr},
         *sev[2] = {nullptr, nullptr};
    if (epochs) {
        for (int b = 0; b < 2; ++b) {
            HIP_TRY(scr.alloc(&sx[b], sizeof(int32_t) * (size_t)n_traj * S));
            HIP_TRY(scr.alloc(&stt[b], sizeof(double) * (size_t)n_traj));
            HIP_TRY(scr.alloc(&skk[b], sizeof(uint64_t) * (size_t)n_traj));
            HIP_TRY(scr.alloc(&sev[b], sizeof(uint64_t) * (size_t)n_traj));
        }
    }

    // Avg-XY across epochs: the points of a group not yet complete wait in front of the
    // next epoch's points (work arrays: pending points, then this epoch's)
    int64_t U_tot = 0, P_done = 0, n_pend = 0;
    void *pend_t = nullptr, *pend_m = nullptr, *pend_v = nullptr;
    if (epochs && !sizing) {
        HIP_TRY(scr.alloc(&pend_t, sizeof(double) * (size_t)k));
        HIP_TRY(scr.alloc(&pend_m, sizeof(double) * (size_t)k * S));
        HIP_TRY(scr.alloc(&pend_v, sizeof(double) * (size_t)k * S));
    }
    double t0 = 0.0, span = epochs ? t_end * (double)budget / (1.25 * (double)R_all) : t_end;
    int sb = 0;          // state buffer holding the current states (epochs)
    bool first = true;
    for (;;) {
        const double t1 = (!epochs || t0 + span >= t_end) ? t_end : t0 + span;
        NetDev n = n0;
        n.t_pause = t1;
        n.ev_key = (unsigned long long *)keys0;
        n.ev_val = (unsigned long long *)vals0;
        n.ev_cap = slots;
        // slots no record takes keep the key ~0, which sorts after every event time
        HIP_TRY(launch_fill(keys0, (size_t)slots, ~0ull, st));
        if (epochs) {
            if (!first) {
                n.rs_x = (const int32_t *)sx[sb];
                n.rs_t = (const double *)stt[sb];
                n.rs_k = (const uint64_t *)skk[sb];
                n.rs_ev = (const uint64_t *)sev[sb];
            }
            n.ws_x = (int32_t *)sx[1 - sb];
            n.ws_t = (double *)stt[1 - sb];
            n.ws_k = (uint64_t *)skk[1 - sb];
            n.ws_ev = (uint64_t *)sev[1 - sb];
        }
        unsigned long long R = 0, h[3] = {0, 0, 0};
        s = log_pass(n, R, h);
        if (s) return s;
        if ((int64_t)R > cap) {
            // the epoch did not fit: shorten it and run it again from the same states
            if (!epochs) return fail(SSA_E_DEVICE, "the event log changed between passes");
            span = (t1 - t0) * 0.8 * (double)cap / (double)R;
            if (!(span > 0.0) || t0 + span <= t0) return fail(SSA_E_UNSUPPORTED, "too many events at one time");
            continue;
        }
        tot_events += h[0];
        max_steps = std::max(max_steps, h[1]);
        all_flags |= (uint32_t)h[2];
        if (tot_events >= kMaxExactEvents)
            return fail(SSA_E_UNSUPPORTED, "%llu events in one run: the exact integer sums hold at most 2^39",
                        (unsigned long long)tot_events);

        // time order and the distinct-time ranks of this epoch's records (the first R of
        // the sorted slots)
        const int32_t nR = (int32_t)R;
        const int32_t nSlots = (int32_t)std::max<unsigned long long>(R, Rs);
        if (nSlots > slots) return fail(SSA_E_DEVICE, "event log slots beyond the reservation bound");
        int32_t n_distinct = 0;
        unsigned long long first_key = 0;
        if (R > 0) {
            // bins and the big-bin list borrow the rank arrays (both >= R >= the bin count)
            HIP_TRY(sort_event_log((unsigned long long *)keys0, (unsigned long long *)vals0, nSlots, (int64_t)R, t0, t1,
                                   (unsigned long long *)keys1, (unsigned long long *)vals1, (int32_t *)rk,
                                   (int32_t *)stf, (int32_t *)n_big, (int32_t *)rdx_cnt, (int32_t *)rdx_incl,
                                   (int32_t *)scan_sums, cap, st));
            const unsigned gb = (unsigned)std::min<int64_t>(((int64_t)R + 255) / 256, 65535);
            hipLaunchKernelGGL(evt_start_kernel, dim3(gb), dim3(256), 0, st, (const unsigned long long *)keys1,
                               (int64_t)R, (int32_t *)stf);
            HIP_TRY(hipGetLastError());
            HIP_TRY(launch_scan((const int32_t *)stf, (int32_t *)rk, nR, (int32_t *)scan_sums, st));
            HIP_TRY(hipMemcpyAsync(&n_distinct, (int32_t *)rk + (R - 1), sizeof n_distinct, hipMemcpyDeviceToHost,
                                   st));
            HIP_TRY(hipMemcpyAsync(&first_key, keys1, sizeof first_key, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        // the point at time 0 (initial state) unless an event happened exactly then
        const int32_t off = (first && (R == 0 || first_key != 0ull)) ? 1 : 0;
        const int64_t U_e = (int64_t)n_distinct + off;
        if (U_tot + U_e > INT32_MAX) return fail(SSA_E_UNSUPPORTED, "more than 2^31 - 1 Avg-Y points");

        const bool last = t1 >= t_end;
        if (!sizing && (U_e > 0 || (last && n_pend > 0))) {
            // Avg-Y of this epoch's points into the work arrays, after the pending ones
            // (scratch of this epoch only: returned to the pool at the end of the block)
            StreamScratch escr(st);
            const int64_t W = n_pend + U_e;
            void *D = nullptr, *Dhi = nullptr, *wt = nullptr, *wm = nullptr, *wv = nullptr, *T = nullptr;
            HIP_TRY(escr.alloc(&wt, sizeof(double) * (size_t)W));
            HIP_TRY(escr.alloc(&wm, sizeof(double) * (size_t)W * S));
            HIP_TRY(escr.alloc(&wv, sizeof(double) * (size_t)W * S));
            double *et = (double *)wt + n_pend, *em = (double *)wm + n_pend * S, *evv = (double *)wv + n_pend * S;
            if (U_e > 0) {
                HIP_TRY(escr.alloc(&D, sizeof(unsigned long long) * (size_t)U_e * S * 2));
                HIP_TRY(escr.alloc(&Dhi, sizeof(unsigned long long) * (size_t)U_e * S));
                HIP_TRY(launch_zero(D, sizeof(unsigned long long) * (size_t)U_e * S * 2, st));
                HIP_TRY(launch_zero(Dhi, sizeof(unsigned long long) * (size_t)U_e * S, st));
                HIP_TRY(launch_zero(et, sizeof(double), st));   // time 0 (overwritten if an event happened there)
                if (R > 0) {
                    const unsigned gb = (unsigned)std::min<int64_t>(((int64_t)R + 255) / 256, 65535);
                    hipLaunchKernelGGL(evt_diff_kernel, dim3(gb), dim3(256), 0, st, (const unsigned long long *)keys1,
                                       (const unsigned long long *)vals1, (const int32_t *)stf, (const int32_t *)rk,
                                       (int64_t)R, off, S, (unsigned long long *)D, (unsigned long long *)Dhi, et);
                    HIP_TRY(hipGetLastError());
                }
                const int64_t n_chunks = (U_e + kFinChunk - 1) / kFinChunk;
                HIP_TRY(escr.alloc(&T, sizeof(long long) * (size_t)n_chunks * S * 3));
                hipLaunchKernelGGL(chunk_total_kernel, dim3((unsigned)n_chunks), dim3(256), 0, st,
                                   (const unsigned long long *)D, (const unsigned long long *)Dhi, U_e, S, (long long *)T);
                HIP_TRY(hipGetLastError());
                hipLaunchKernelGGL(chunk_scan_kernel, dim3((unsigned)S), dim3(1024), 0, st, (long long *)T, n_chunks, S,
                                   (long long *)carry);
                HIP_TRY(hipGetLastError());
                hipLaunchKernelGGL(chunk_final_kernel, dim3((unsigned)n_chunks), dim3(256), 0, st,
                                   (const unsigned long long *)D, (const unsigned long long *)Dhi, U_e, S,
                                   (const long long *)T, (const int32_t *)m->d_x0, n_traj, em, evv);
                HIP_TRY(hipGetLastError());
                if (y_time && U_tot + U_e <= y_cap) {
                    HIP_TRY(hipMemcpyAsync(y_time + U_tot, et, sizeof(double) * (size_t)U_e, hipMemcpyDeviceToDevice, st));
                    HIP_TRY(hipMemcpyAsync(y_mean + U_tot * S, em, sizeof(double) * (size_t)U_e * S,
                                           hipMemcpyDeviceToDevice, st));
                    HIP_TRY(hipMemcpyAsync(y_var + U_tot * S, evv, sizeof(double) * (size_t)U_e * S,
                                           hipMemcpyDeviceToDevice, st));
                }
            }
            if (n_pend > 0) {
                HIP_TRY(hipMemcpyAsync(wt, pend_t, sizeof(double) * (size_t)n_pend, hipMemcpyDeviceToDevice, st));
                HIP_TRY(hipMemcpyAsync(wm, pend_m, sizeof(double) * (size_t)n_pend * S, hipMemcpyDeviceToDevice, st));
                HIP_TRY(hipMemcpyAsync(wv, pend_v, sizeof(double) * (size_t)n_pend * S, hipMemcpyDeviceToDevice, st));
            }
            // the complete groups (all of them after the last epoch)
            const int64_t P_e = last ? (W + k - 1) / k : W / k;
            if (xy_time && P_e > 0 && P_done + P_e <= xy_cap) {
                hipLaunchKernelGGL(xy_kernel, dim3((unsigned)P_e, (unsigned)((2 * S + 1 + kWave - 1) / kWave)),
                                   dim3(kXyThreads), 0, st,
                                   (const double *)wt, (const double *)wm, (const double *)wv, W, S, k, P_e,
                                   xy_time + P_done, xy_mean + P_done * S, xy_var + P_done * S);
                HIP_TRY(hipGetLastError());
            }
            const int64_t rest = W - P_e * k;
            if (rest > 0 && epochs) {
                HIP_TRY(hipMemcpyAsync(pend_t, (double *)wt + P_e * k, sizeof(double) * (size_t)rest,
                                       hipMemcpyDeviceToDevice, st));
                HIP_TRY(hipMemcpyAsync(pend_m, (double *)wm + P_e * k * S, sizeof(double) * (size_t)rest * S,
                                       hipMemcpyDeviceToDevice, st));
                HIP_TRY(hipMemcpyAsync(pend_v, (double *)wv + P_e * k * S, sizeof(double) * (size_t)rest * S,
                                       hipMemcpyDeviceToDevice, st));
            }
            P_done += P_e;
            n_pend = rest;
            HIP_TRY(hipStreamSynchronize(st));   // the epoch's scratch is reused by the next one
        }
        U_tot += U_e;
        first = false;
        if (t1 >= t_end) break;
        // the next epoch's length from this one's fill (records are not uniform in time)
        const double fill = 0.85 * (double)cap / (double)std::max<unsigned long long>(R, 1ull);
        span = std::min((t1 - t0) * std::min(std::max(fill, 0.5), 4.0), t_end);
        t0 = t1;
        sb = 1 - sb;
    }
    const int64_t P = (U_tot + k - 1) / k;
    n_points[0] = U_tot;
    n_points[1] = P;
    if (timed) HIP_TRY(hipEventRecord(evp.b, st));
    if (stats) {
        HIP_TRY(hipStreamSynchronize(st));
        stats->events = epochs ? tot_events : h0[0];
        stats->max_steps = epochs ? max_steps : h0[1];
        stats->flags = epochs ? all_flags : (uint32_t)h0[2];
        stats->kernel_ms = 0.0f;
        stats->form = g_launch.form;
        stats->blocks = g_launch.blocks;
        if (timed) (void)hipEventElapsedTime(&stats->kernel_ms, evp.a, evp.b);
    }
    if (sizing) return SSA_OK;
    if (xy_time && xy_cap < P) return fail(SSA_E_INVALID, "Avg-XY needs %lld points (capacity %lld)", (long long)P,
                                           (long long)xy_cap);
    if (y_time && y_cap < U_tot)
        return fail(SSA_E_INVALID, "Avg-Y needs %lld points (capacity %lld)", (long long)U_tot, (long long)y_cap);
    return SSA_OK;
}

// ------------------------------------------------------------------------------------------
// Batched form: one persistent launch of the generic kernel over all networks.
// ------------------------------------------------------------------------------------------
ssa_status ssa_batch_create(int32_t B, const ssa_model *const *models, const int64_t *n_traj, const double *t_end,
                            const double *const *grids, const int32_t *n_grid, const uint64_t *seeds,
                            ssa_batch **out) {
    if (!out) return fail(SSA_E_INVALID, "out is NULL");
    *out = nullptr;
    if (B <= 0 || !models || !n_traj || !t_end || !grids || !n_grid || !seeds) return fail(SSA_E_INVALID, "bad batch");
    std::unique_ptr<ssa_batch, void (*)(ssa_batch *)> bt(new (std::nothrow) ssa_batch, ssa_batch_destroy);
    if (!bt) return fail(SSA_E_NOMEM, "host allocation failed");
    bt->B = B;
    HIP_TRY(hipGetDevice(&bt->device));
    std::vector<int32_t> item_net;
    std::vector<int64_t> item_begin;
    std::vector<int32_t> item_count;
    size_t D_words = 0;
    int32_t mmax = 0;
    for (int32_t b = 0; b < B; ++b) {
        const ssa_model *m = models[b];
        if (!m) return fail(SSA_E_INVALID, "model %d is NULL", b);
        if (n_traj[b] <= 0) return fail(SSA_E_INVALID, "n_traj[%d] must be > 0", b);
        if (n_traj[b] > ((int64_t)1 << 31)) return fail(SSA_E_INVALID, "n_traj[%d] too large", b);
        ssa_status s = validate_grid_host(grids[b], n_grid[b], t_end[b]);
        if (s) return s;
        if (m->max_changes > kChg)
            return fail(SSA_E_UNSUPPORTED, "batched networks may change at most %d species per reaction", kChg);
        if (m->order != SSA_SUM_SEQ) return fail(SSA_E_UNSUPPORTED, "batched networks use the sequential sum order");
        if (m->has_laws) return fail(SSA_E_UNSUPPORTED, "batched networks are mass action");
        mmax = std::max(mmax, m->M);
        bt->s_rows = std::max(bt->s_rows, m->S);
        bt->m_rows = std::max(bt->m_rows, m->M);
        bt->models.push_back(m);
        bt->n_traj.push_back(n_traj[b]);
        bt->G.push_back(n_grid[b]);
        bt->D_off.push_back(D_words);
        D_words += (size_t)3 * n_grid[b] * m->S;
        for (int64_t i = 0; i < n_traj[b]; i += kChunk) {
            item_net.push_back(b);
            item_begin.push_back(i);
            item_count.push_back((int32_t)std::min<int64_t>(kChunk, n_traj[b] - i));
        }
    }
    if (item_net.size() > (size_t)INT32_MAX) return fail(SSA_E_INVALID, "too many work items");
    bt->mm = generic_mm(mmax);
    bt->n_items = (int32_t)item_net.size();
    bt->D_words = D_words;
    for (int32_t b = 0; b < B; ++b) {
        double *dg = nullptr;
        HIP_TRY(hipMalloc(&dg, sizeof(double) * n_grid[b]));
        bt->d_grids.push_back(dg);
        HIP_TRY(hipMemcpy(dg, grids[b], sizeof(double) * n_grid[b], hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMalloc(&bt->d_D, sizeof(unsigned long long) * D_words));
    HIP_TRY(hipMalloc(&bt->d_counter, 64));
    HIP_TRY(hipMalloc(&bt->d_nets, sizeof(NetDev) * B));
    HIP_TRY(hipMalloc(&bt->d_ginfo, sizeof(GridInfo) * B));
    HIP_TRY(hipMalloc(&bt->d_item_net, sizeof(int32_t) * bt->n_items));
    HIP_TRY(hipMalloc(&bt->d_item_begin, sizeof(int64_t) * bt->n_items));
    HIP_TRY(hipMalloc(&bt->d_item_count, sizeof(int32_t) * bt->n_items));
    bt->d_stats = (unsigned long long *)((char *)bt->d_counter + 32);
    std::vector<NetDev> nets;
    std::vector<GridInfo> gis;
    for (int32_t b = 0; b < B; ++b) {
        NetDev n = base_net(models[b], nullptr, n_traj[b], t_end[b], bt->d_grids[b], n_grid[b], seeds[b], 0);
        n.D = bt->d_D + bt->D_off[b];
        n.Dhi = n.D + (size_t)2 * n_grid[b] * models[b]->S;
        n.ginfo = bt->d_ginfo + b;
        nets.push_back(n);
        gis.push_back(host_grid_info(grids[b], n_grid[b], t_end[b]));
    }
    HIP_TRY(hipMemcpy(bt->d_nets, nets.data(), sizeof(NetDev) * B, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bt->d_ginfo, gis.data(), sizeof(GridInfo) * B, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bt->d_item_net, item_net.data(), sizeof(int32_t) * bt->n_items, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bt->d_item_begin, item_begin.data(), sizeof(int64_t) * bt->n_items, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bt->d_item_count, item_count.data(), sizeof(int32_t) * bt->n_items, hipMemcpyHostToDevice));
    // finalize tables: one block per (network, species)
    std::vector<int32_t> bn, bs;
    bt->fin.resize(B);
    for (int32_t b = 0; b < B; ++b) {
        FinalNet &f = bt->fin[b];
        f.D = bt->d_D + bt->D_off[b];
        f.Dhi = f.D + (size_t)2 * n_grid[b] * models[b]->S;
        f.x0 = models[b]->d_x0;
        f.mean = f.var = nullptr;
        f.n_traj = n_traj[b];
        f.G = n_grid[b];
        f.S = models[b]->S;
        for (int32_t s = 0; s < f.S; ++s) {
            bn.push_back(b);
            bs.push_back(s);
        }
    }
    bt->n_fin_blocks = (int32_t)bn.size();
    HIP_TRY(hipMalloc(&bt->d_fin, sizeof(FinalNet) * B));
    HIP_TRY(hipMalloc(&bt->d_block_net, sizeof(int32_t) * bn.size()));
    HIP_TRY(hipMalloc(&bt->d_block_species, sizeof(int32_t) * bs.size()));
    HIP_TRY(hipMemcpy(bt->d_block_net, bn.data(), sizeof(int32_t) * bn.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bt->d_block_species, bs.data(), sizeof(int32_t) * bs.size(), hipMemcpyHostToDevice));
    *out = bt.release();
    return SSA_OK;
}

namespace {

// The launch sequence of one batched run: zero the sums and the work counter, the
// persistent kernel over all networks, one finalize launch for all networks.
ssa_status batch_enqueue(ssa_batch *bt, hipStream_t st) {
    HIP_TRY(launch_zero(bt->d_D, sizeof(unsigned long long) * bt->D_words, st));
    HIP_TRY(launch_zero(bt->d_counter, 64, st));
    WorkList wl;
    std::memset(&wl, 0, sizeof wl);
    wl.nets = bt->d_nets;
    wl.item_net = bt->d_item_net;
    wl.item_begin = bt->d_item_begin;
    wl.item_count = bt->d_item_count;
    wl.n_items = bt->n_items;
    wl.s_rows = bt->s_rows;
    wl.m_rows = bt->m_rows;
    wl.counter = bt->d_counter;
    wl.stats = bt->d_stats;
    int32_t gmax = 0;
    for (int32_t g : bt->G) gmax = std::max(gmax, g);
    wl.win_bins = window_bins(bt->s_rows, gmax, true, bt->win_bytes);
    wl.win_words = wl.win_bins * bt->s_rows * 2;
    FwdKernel k;
    if (!pick_generic_fwd<true>(bt->mm, k)) return fail(SSA_E_UNSUPPORTED, "no kernel");
    k.lds = generic_int_words(wl.s_rows, wl.m_rows) * sizeof(int32_t) +
            (size_t)(kBlock / kWave) * kCohorts * wl.win_words * sizeof(long long);
    if (k.lds > lds_max(bt->device))
        return fail(SSA_E_UNSUPPORTED, "the batch needs %zu bytes of LDS per block (limit %zu)", k.lds,
                    lds_max(bt->device));
    int64_t blocks = 0;
    HIP_TRY(fwd_blocks(k, false, bt->device, bt->n_items, blocks));
    HIP_TRY(fwd_launch(k, false, blocks, wl, st));
    bt->launch = g_launch;
    hipLaunchKernelGGL(moment_final_batched_kernel, dim3((unsigned)bt->n_fin_blocks), dim3(1024), 0, st,
                       (const FinalNet *)bt->d_fin, (const int32_t *)bt->d_block_net,
                       (const int32_t *)bt->d_block_species);
    HIP_TRY(hipGetLastError());
    return SSA_OK;
}

// Graph replay is the default; SSA_BATCH_GRAPH=0 launches the same sequence directly.
bool batch_use_graph() {
    const char *e = std::getenv("SSA_BATCH_GRAPH");
    return !(e && std::strcmp(e, "0") == 0);
}

}  // namespace

ssa_status ssa_batch_run(ssa_batch *bt, double *const *means, double *const *vars, void *stream, ssa_stats *stats) {
    if (!bt || !means || !vars) return fail(SSA_E_INVALID, "NULL argument");
    for (int32_t b = 0; b < bt->B; ++b)
        if (!means[b] || !vars[b]) return fail(SSA_E_INVALID, "output %d is NULL", b);
    hipStream_t st = (hipStream_t)stream;
    // output pointers live in the device finalize table, so a captured graph stays valid
    // when they change; the table is rewritten only then, after the stream is idle
    bool changed = false;
    for (int32_t b = 0; b < bt->B; ++b) changed |= bt->fin[b].mean != means[b] || bt->fin[b].var != vars[b];
    if (changed) {
        HIP_TRY(hipStreamSynchronize(st));
        for (int32_t b = 0; b < bt->B; ++b) {
            bt->fin[b].mean = means[b];
            bt->fin[b].var = vars[b];
        }
        HIP_TRY(hipMemcpy(bt->d_fin, bt->fin.data(), sizeof(FinalNet) * bt->B, hipMemcpyHostToDevice));
    }
    EventPair ev;
    if (stats && ev.make()) HIP_TRY(hipEventRecord(ev.a, st));
    if (batch_use_graph()) {
        if (!bt->exec) {
            // capture on a private stream (the caller's may be the null stream)
            if (!bt->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking));
            HIP_TRY(hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal));
            ssa_status s = batch_enqueue(bt, bt->cap_stream);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(bt->cap_stream, &g);
            if (s) {
                if (g) (void)hipGraphDestroy(g);
                return s;
            }
            HIP_TRY(ce);
            bt->graph = g;
            HIP_TRY(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
        }
        HIP_TRY(hipGraphLaunch(bt->exec, st));
    } else {
        ssa_status s = batch_enqueue(bt, st);
        if (s) return s;
    }
    if (stats && ev.b) HIP_TRY(hipEventRecord(ev.b, st));
    g_launch = bt->launch;     // a graph replay launches nothing through the host helpers
    if (stats) return collect_stats(bt->d_stats, st, ev.a, ev.b, stats);
    return SSA_OK;
}

ssa_status ssa_batch_autotune(ssa_batch *bt, void *stream, ssa_tune_result *result) {
    if (!bt) return fail(SSA_E_INVALID, "batch is NULL");
    hipStream_t st = (hipStream_t)stream;
    // the trial runs finalize into scratch outputs; the caller's are put back afterwards
    HIP_TRY(hipStreamSynchronize(st));
    StreamScratch scr(st);
    std::vector<FinalNet> trial = bt->fin;
    for (int32_t b = 0; b < bt->B; ++b) {
        void *mp = nullptr, *vp = nullptr;
        const size_t bytes = sizeof(double) * (size_t)bt->G[b] * bt->models[b]->S;
        HIP_TRY(scr.alloc(&mp, bytes));
        HIP_TRY(scr.alloc(&vp, bytes));
        trial[b].mean = (double *)mp;
        trial[b].var = (double *)vp;
    }
    HIP_TRY(hipMemcpyAsync(bt->d_fin, trial.data(), sizeof(FinalNet) * bt->B, hipMemcpyHostToDevice, st));
    struct Restore {
        ssa_batch *bt;
        hipStream_t st;
        ~Restore() {
            (void)hipStreamSynchronize(st);
            (void)hipMemcpy(bt->d_fin, bt->fin.data(), sizeof(FinalNet) * bt->B, hipMemcpyHostToDevice);
        }
    } restore{bt, st};
    EventPair ev;
    if (!ev.make()) return fail(SSA_E_DEVICE, "hipEventCreate failed");
    const int32_t saved = bt->win_bytes;
    float best_ms = 0.0f, default_ms = 0.0f;
    int32_t best = -1;
    for (int32_t wb : {0, 2048, 4096, 8192, 16384}) {
        bt->win_bytes = wb;
        float ms = 0.0f;
        bool ok = true;
        for (int rep = 0; rep < 2 && ok; ++rep) {   // the first run warms up, the second is timed
            HIP_TRY(hipEventRecord(ev.a, st));
            const ssa_status s = batch_enqueue(bt, st);
            if (s == SSA_E_UNSUPPORTED) {
                ok = false;   // window too large for the LDS: skip the candidate
                break;
            }
            if (s) {
                bt->win_bytes = saved;
                return s;
            }
            HIP_TRY(hipEventRecord(ev.b, st));
            HIP_TRY(hipEventSynchronize(ev.b));
            HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
        }
        if (!ok) continue;
        if (wb == 0) default_ms = ms;
        if (best < 0 || ms < best_ms) {
            best = wb;
            best_ms = ms;
        }
    }
    bt->win_bytes = best < 0 ? saved : best;
    // the captured graph holds the old window: capture again at the next run
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;
    if (result) {
        result->win_bytes = bt->win_bytes;
        result->slab = -1;
        result->best_ms = best_ms;
        result->form = 0;
        result->blocks = 0;
        result->default_ms = default_ms;
    }
    return SSA_OK;
}

void ssa_batch_destroy(ssa_batch *bt) {
    if (!bt) return;
    for (double *p : bt->d_grids) (void)hipFree(p);
    if (bt->d_D) (void)hipFree(bt->d_D);
    if (bt->d_counter) (void)hipFree(bt->d_counter);
    if (bt->d_nets) (void)hipFree(bt->d_nets);
    if (bt->d_ginfo) (void)hipFree(bt->d_ginfo);
    if (bt->d_item_net) (void)hipFree(bt->d_item_net);
    if (bt->d_item_begin) (void)hipFree(bt->d_item_begin);
    if (bt->d_item_count) (void)hipFree(bt->d_item_count);
    if (bt->d_fin) (void)hipFree(bt->d_fin);
    if (bt->d_block_net) (void)hipFree(bt->d_block_net);
    if (bt->d_block_species) (void)hipFree(bt->d_block_species);
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
    delete bt;
}
